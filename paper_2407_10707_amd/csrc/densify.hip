// Density-based densification (App. B, Alg. 1), bit-exact.
//
//   count   D_v[k] = number of Gaussians whose K_g nearest vertices include k
//           (integer atomics: the counts do not depend on the order)
//   faces   one workgroup: per triangle the vertex sum S, the density
//           d_f = S / (6 K_g), and the sampling weight held as an exact
//           integer Q = max(0, T - 65536 S), T = round(d0 6 K_g 65536),
//           i.e. P = max(0, d0 - d_f) in units of 1 / (6 K_g 65536);
//           an inclusive scan of Q over the triangles (a contiguous run
//           per thread, then the runs' sums across the workgroup);
//           the number of added Gaussians N' = floor(sum(Q) p0 / unit)
//   draw    draw j takes the j-th triple of a counter-based generator
//           (SplitMix64 outputs 3j+1, 3j+2, 3j+3): the first picks the
//           triangle whose cumulative range of Q holds floor(r sum(Q) / 2^64)
//           (the multinomial with probabilities P / sum(P)), the other two a
//           uniform point of that triangle (s = sqrt(u1), barycentric
//           (1 - s, s (1 - u2), s u2))
// The work is tiny next to a training iteration (one pass over the K_g
// lists, one over the triangles, N' of about 0.02 nf draws) and runs every
// hundred iterations, so each step is one short launch.
#include "common.h"

namespace {

constexpr int kBlock = 256;
constexpr int kFaceBlock = 1024;

__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(kBlock)
densify_clear_kernel(int nv, int32_t* __restrict__ Dv, int nf, int32_t* __restrict__ ng) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < nv) Dv[i] = 0;
  if (i < nf) ng[i] = 0;
}

// one thread per (neighbour slot, Gaussian) entry; entries of consecutive
// lanes that name the same vertex (Gaussians stored grouped by vertex) are
// counted with one atomic per run
__global__ void __launch_bounds__(kBlock)
densify_count_kernel(int64_t total, const int32_t* __restrict__ sg, int nv,
                     int32_t* __restrict__ Dv) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool ok = e < total;
  const int v = ok ? rga::clampi(sg[e], 0, nv - 1) : -1 - lane;
  int end;
  if (rga::wave_run(v, end) && ok) atomicAdd(&Dv[v], end - lane);
}

// inclusive scan of 64-bit values over a wave (shuffles), then over the
// sixteen waves of the workgroup through LDS; returns the inclusive prefix
// and sets `block_total`
__device__ inline int64_t block_scan(int64_t v, int64_t* wave_tot, int64_t& block_total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  if (lane == 63) wave_tot[wave] = v;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int w = 0; w < kFaceBlock / 64; ++w) {
    const int64_t t = wave_tot[w];
    if (w < wave) before += t;
    all += t;
  }
  __syncthreads();   // wave_tot is reused by the next call
  block_total = all;
  return v + before;
}

__global__ void __launch_bounds__(kFaceBlock)
densify_faces_kernel(int nf, const int32_t* __restrict__ faces, int nv,
                     const int32_t* __restrict__ Dv, int kg, int64_t T, double p0, int64_t unit,
                     float* __restrict__ df, int64_t* __restrict__ cum,
                     int64_t* __restrict__ summary /* [0] sum(Q), [1] N' */) {
  __shared__ int64_t wave_tot[kFaceBlock / 64];
  const double denom = (double)(6 * kg);
  // each thread owns a contiguous run of triangles: their loads are
  // independent of one another, so they overlap instead of forming one
  // dependent chain per 1024 triangles
  const int per = (nf + kFaceBlock - 1) / kFaceBlock;
  const int f0 = min(nf, (int)threadIdx.x * per), f1 = min(nf, f0 + per);
  int64_t local = 0;
  for (int f = f0; f < f1; ++f) {
    int64_t S = 0;
    for (int c = 0; c < 3; ++c) S += Dv[rga::clampi(faces[3 * f + c], 0, nv - 1)];
    df[f] = (float)((double)S / denom);
    int64_t q = T - 65536 * S;
    if (q < 0) q = 0;
    cum[f] = q;
    local += q;
  }
  int64_t total;
  int64_t run = block_scan(local, wave_tot, total) - local;   // exclusive prefix
  for (int f = f0; f < f1; ++f) {   // the thread's own writes above
    run += cum[f];
    cum[f] = run;
  }
  if (threadIdx.x == 0) {
    summary[0] = total;
    summary[1] = total > 0 ? (int64_t)floor((double)total * p0 / (double)unit) : 0;
  }
}

// one draw per thread, grid-stride over the N' draws read from the device
__global__ void __launch_bounds__(kBlock)
densify_draw_kernel(int nf, const int32_t* __restrict__ faces, int nv,
                    const float* __restrict__ verts, const int64_t* __restrict__ cum,
                    const int64_t* __restrict__ summary, uint64_t seed, int64_t cap,
                    int32_t* __restrict__ ng, float* __restrict__ x_out,
                    int32_t* __restrict__ f_out) {
  const uint64_t total = (uint64_t)summary[0];
  const int64_t N = summary[1];
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < N;
       j += (int64_t)gridDim.x * kBlock) {
    const uint64_t r = splitmix64(seed, 3 * (uint64_t)j + 1);
    const int64_t u = (int64_t)__umul64hi(r, total);   // floor(r total / 2^64) < total
    int lo = 0, hi = nf - 1;   // first triangle whose inclusive cumulative sum exceeds u
    while (lo < hi) {
      const int mid = lo + (hi - lo) / 2;
      if (cum[mid] > u) hi = mid; else lo = mid + 1;
    }
    atomicAdd(&ng[lo], 1);
    if (j < cap) {
      const float u1 = (float)(splitmix64(seed, 3 * (uint64_t)j + 2) >> 40) * 0x1p-24f;
      const float u2 = (float)(splitmix64(seed, 3 * (uint64_t)j + 3) >> 40) * 0x1p-24f;
      const float s = sqrtf(u1);
      const float b0 = 1.f - s, b1 = s * (1.f - u2), b2 = s * u2;
      const int a = rga::clampi(faces[3 * lo], 0, nv - 1);
      const int b = rga::clampi(faces[3 * lo + 1], 0, nv - 1);
      const int c = rga::clampi(faces[3 * lo + 2], 0, nv - 1);
#pragma unroll
      for (int k = 0; k < 3; ++k)
        x_out[(size_t)k * cap + j] =
            fmaf(b2, verts[(size_t)k * nv + c],
                 fmaf(b1, verts[(size_t)k * nv + b], b0 * verts[(size_t)k * nv + a]));
      f_out[j] = lo;
    }
  }
}

}  // namespace

extern "C" size_t densify_workspace(int nf) {
  if (nf < 0) return 0;
  return rga::align_up(sizeof(int64_t) * (size_t)(nf > 0 ? nf : 1), 256);
}

extern "C" int densify(void* stream, int n, int kg, const int32_t* sg, int nv,
                       const float* verts, int nf, const int32_t* faces, double d0, double p0,
                       uint64_t seed, int64_t cap, int32_t* Dv, float* df, int32_t* ng,
                       float* x_out, int32_t* f_out, int64_t* summary, void* ws,
                       size_t ws_bytes) {
  if (n < 0 || nv < 1 || nf < 0 || cap < 0)
    return rga::fail(RGA_EINVAL, "densify: n >= 0, nv >= 1, nf >= 0, cap >= 0");
  if (kg < 1 || kg > 64) return rga::fail(RGA_EINVAL, "densify: kg must be in 1..64");
  if (!(d0 >= 0.0 && d0 <= 1e6) || !(p0 >= 0.0 && p0 <= 1e6))
    return rga::fail(RGA_EINVAL, "densify: d0 and p0 must be in [0, 1e6]");
  if ((n > 0 && !sg) || !verts || (nf > 0 && !faces) || !Dv || !summary ||
      (nf > 0 && (!df || !ng || !ws)) || (cap > 0 && (!x_out || !f_out)))
    return rga::fail(RGA_EINVAL, "densify: null pointer");
  if (nf > 0 && ws_bytes < densify_workspace(nf))
    return rga::fail(RGA_ECAPACITY, "densify: workspace %zu < %zu bytes", ws_bytes,
                     densify_workspace(nf));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t unit = 6LL * kg * 65536LL;
  const int64_t T = llround(d0 * (double)unit);
  const int clear_n = nv > nf ? nv : nf;
  RGA_LAUNCH("densify_clear", densify_clear_kernel, dim3(rga::ceil_div(clear_n, kBlock)),
             dim3(kBlock), 0, s, nv, Dv, nf, ng);
  const int64_t entries = (int64_t)n * kg;
  if (entries > 0)
    RGA_LAUNCH("densify_count", densify_count_kernel, dim3(rga::ceil_div(entries, kBlock)),
               dim3(kBlock), 0, s, entries, sg, nv, Dv);
  int64_t* cum = static_cast<int64_t*>(ws);
  RGA_LAUNCH("densify_faces", densify_faces_kernel, dim3(1), dim3(kFaceBlock), 0, s, nf, faces,
             nv, Dv, kg, T, p0, unit, df, cum, summary);
  if (nf > 0)
    RGA_LAUNCH("densify_draw", densify_draw_kernel, dim3(256), dim3(kBlock), 0, s, nf, faces, nv,
               verts, cum, summary, seed, cap, ng, x_out, f_out);
  RGA_CHECK_LAUNCH("densify");
  return RGA_OK;
}
