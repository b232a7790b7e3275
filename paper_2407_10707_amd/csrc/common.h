// Internal helpers shared by the HIP sources of the library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rga.h"

namespace rga {

// Record an error message for rga_last_error() and return `code`.
int fail(int code, const char* fmt, ...);
// Check the launch that was just issued; returns RGA_OK or RGA_EHIP.
int check_launch(const char* what);

// Optional event timing around kernel launches (see rga_timing_enable).
bool timing_on();
void timing_mark(const char* name, hipStream_t s, bool start);

struct TimedLaunch {
  const char* name;
  hipStream_t s;
  bool on;
  TimedLaunch(const char* n, hipStream_t st) : name(n), s(st), on(timing_on()) {
    if (on) timing_mark(name, s, true);
  }
  ~TimedLaunch() {
    if (on) timing_mark(name, s, false);
  }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Launch `kernel` under an optional timing scope and check for launch errors.
#define RGA_LAUNCH(name, kernel, grid, block, shmem, stream, ...)                \
  do {                                                                          \
    ::rga::TimedLaunch _rga_tl((name), (stream));                               \
    hipLaunchKernelGGL((kernel), (grid), (block), (shmem), (stream), __VA_ARGS__); \
  } while (0)

#define RGA_CHECK_LAUNCH(name)                     \
  do {                                             \
    int _rc = ::rga::check_launch(name);           \
    if (_rc != RGA_OK) return _rc;                 \
  } while (0)

// ---- device helpers ------------------------------------------------------
// Sum over the 64 lanes of a wave with DPP: row shifts build per-row
// prefix sums, two row broadcasts carry them to lane 63, whose value is
// returned to every lane.  All 64 lanes must be active.
__device__ inline float wave_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, false));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Sums of N values over each row of 16 lanes, in place: DPP row shifts
// build per-row prefix sums, so lane 15 of each row ends with that row's
// totals.  The N chains are interleaved step by step so that no DPP read
// has to wait for the write just before it.  All 64 lanes must be active.
template <int N>
__device__ inline void row_sums(float (&v)[N]) {
#pragma unroll
  for (int q = 0; q < N; ++q)
    v[q] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[q]), 0x111, 0xf, 0xf, true));
#pragma unroll
  for (int q = 0; q < N; ++q)
    v[q] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[q]), 0x112, 0xf, 0xf, true));
#pragma unroll
  for (int q = 0; q < N; ++q)
    v[q] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[q]), 0x114, 0xf, 0xf, true));
#pragma unroll
  for (int q = 0; q < N; ++q)
    v[q] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[q]), 0x118, 0xf, 0xf, true));
}

// Float add into LDS through an integer compare-and-swap loop.  On gfx950
// the LDS float atomic add is several times slower than the integer atomic
// path when a whole wave adds to distinct addresses; a compare-and-swap then
// almost always succeeds at once.  (Where only a few lanes add and the
// result is needed soon, the returned-value latency makes it the slower
// choice.)  A failed swap means another lane's add landed first, so the
// loop always finishes.
__device__ inline void lds_add(float* p, float x) {
  unsigned* u = reinterpret_cast<unsigned*>(p);
  unsigned old = *u;
  for (;;) {
    const unsigned seen = old;
    old = atomicCAS(u, seen, __float_as_uint(__uint_as_float(seen) + x));
    if (old == seen) break;
  }
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

}  // namespace rga
