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

// Inclusive prefix sum over the 64 lanes of a wave (integers): row shifts
// by 1, 2, 4, 8 (lanes past the row start read 0), then the last lane of
// rows 0 and 2 is added to rows 1 and 3, and lane 31 to rows 2 and 3.
// All 64 lanes must be active.
__device__ inline uint32_t wave_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
  return v;
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

// Lane exchanges of gfx950: swap_halves exchanges the upper half-wave of
// `a` with the lower half-wave of `b` (v_permlane32_swap); swap_rows
// exchanges the odd rows of `a` with the even rows of `b`
// (v_permlane16_swap).
__device__ inline void swap_halves(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}

__device__ inline void swap_rows(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}

template <int CTRL>
__device__ inline float dpp_add(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

// Sums over all 64 lanes of a wave for four slots of N values each; slot s
// ends, fully summed, in every lane of row s (lanes 16s .. 16s+15) of
// `out`.  Two halving steps each hand half of the slots to the partner lane
// and keep the other half (half-wave swap, then odd/even row swap); four
// butterflies inside the row (lane xor 15, 7, 2, 1: row mirror, half-row
// mirror, two quad permutations) finish the sums.  10 instructions per
// value for four slots, against 4 DPP adds per value and slot for a row
// sum alone.  All 64 lanes must be active.
template <int N>
__device__ inline void slot_sums4(float (&v)[4][N], float (&out)[N]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int q = 0; q < N; ++q) {   // lanes 0-31 keep slots 0-1, lanes 32-63 slots 2-3
      swap_halves(v[s][q], v[s + 2][q]);
      v[s][q] += v[s + 2][q];
    }
#pragma unroll
  for (int q = 0; q < N; ++q) {     // row s keeps slot s
    swap_rows(v[0][q], v[1][q]);
    out[q] = v[0][q] + v[1][q];
  }
#pragma unroll
  for (int q = 0; q < N; ++q) out[q] = dpp_add<0x140>(out[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) out[q] = dpp_add<0x141>(out[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) out[q] = dpp_add<0x4E>(out[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) out[q] = dpp_add<0xB1>(out[q]);
}

// The same for eight slots: slot s ends, fully summed, in lanes 8s .. 8s+7.
// Three halving steps (half-wave swap, odd/even row swap, row mirror with a
// select), then three butterflies over the eight lanes of a slot (lane xor
// 7, 2, 1).  18 instructions per value for eight slots.
template <int N>
__device__ inline void slot_sums8(float (&v)[8][N], float (&out)[N]) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int q = 0; q < N; ++q) {   // lanes 0-31 keep slots 0-3, lanes 32-63 slots 4-7
      swap_halves(v[s][q], v[s + 4][q]);
      v[s][q] += v[s + 4][q];
    }
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int q = 0; q < N; ++q) {   // rows 0 and 2 keep v[0], v[1]; rows 1 and 3 v[2], v[3]
      swap_rows(v[s][q], v[s + 2][q]);
      v[s][q] += v[s + 2][q];
    }
  const bool low = (__lane_id() & 8) == 0;
#pragma unroll
  for (int q = 0; q < N; ++q) {     // lanes 0-7 of a row keep v[0], lanes 8-15 v[1]
    const float a = dpp_add<0x140>(v[0][q]);
    const float b = dpp_add<0x140>(v[1][q]);
    out[q] = low ? a : b;
  }
#pragma unroll
  for (int q = 0; q < N; ++q) out[q] = dpp_add<0x141>(out[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) out[q] = dpp_add<0x4E>(out[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) out[q] = dpp_add<0xB1>(out[q]);
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

// Three such adds to consecutive floats: one compare-and-swap attempt for
// each, all three issued before waiting (one LDS round trip when no other
// lane interferes); a failed attempt falls back to the loop above.
__device__ inline void lds_add3(float* p, float x0, float x1, float x2) {
  unsigned* u = reinterpret_cast<unsigned*>(p);
  const unsigned o0 = u[0], o1 = u[1], o2 = u[2];
  const unsigned r0 = atomicCAS(u, o0, __float_as_uint(__uint_as_float(o0) + x0));
  const unsigned r1 = atomicCAS(u + 1, o1, __float_as_uint(__uint_as_float(o1) + x1));
  const unsigned r2 = atomicCAS(u + 2, o2, __float_as_uint(__uint_as_float(o2) + x2));
  if (r0 != o0) lds_add(p, x0);
  if (r1 != o1) lds_add(p + 1, x1);
  if (r2 != o2) lds_add(p + 2, x2);
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Runs of equal keys in consecutive lanes of a wave (a scatter-add whose
// targets repeat, e.g. Gaussians stored grouped by vertex, adding into the
// vertex): `end` is one past the lane's run, and the run's first lane is
// the one to add.  Every lane of the wave must call it; equal keys that
// are not adjacent form separate runs.
__device__ inline bool wave_run(int key, int& end) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1, 64);
  const bool head = lane == 0 || prev != key;
  const uint64_t heads = __ballot(head);
  const uint64_t after = lane == 63 ? 0ull : (heads & (~0ull << (lane + 1)));
  end = after ? (int)__builtin_ctzll(after) : 64;
  return head;
}

// v summed over the lane's run of equal keys (a segmented suffix sum: the
// run's first lane gets the whole run); returns whether this lane is first.
__device__ inline bool wave_run_sum(int key, float& v) {
  const int lane = threadIdx.x & 63;
  int end;
  const bool head = wave_run(key, end);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const float t = __shfl_down(v, o, 64);
    if (lane + o < end) v += t;
  }
  return head;
}

}  // namespace rga
