// Per-Gaussian shading (Sec. 3.1 rendering equation, App. A BRDF) and its
// adjoint, FP32 form.
//
// Work mapping: one wave64 per Gaussian, lanes over light directions.  Per
// chunk of 64 directions each lane evaluates n.w_k and the interpolated
// visibility v_g[k] (three coalesced byte loads from the vertex-major count
// rows); a wave ballot compacts the live directions (n.w_k > 0 and
// v_g[k] > 0) into a 128-slot LDS ring, and the BRDF weights are evaluated
// only for full waves of live directions.  For a typical body roughly a
// third of the K directions are live, so the expensive part (GGX, Fresnel,
// Smith) runs at full SIMD width on that third only.  The per-lane sums are
// reduced across the wave once per Gaussian.
//
// The direction table (unit direction, radiance x solid angle, view index)
// is built in LDS by every workgroup; workgroups are persistent and loop
// over Gaussians.
//
// Given a tape, the forward also writes each Gaussian's live (direction,
// visibility) pairs, in the order and 64-pair groups of its walk; the
// adjoint of the same inputs then replays them instead of walking every
// direction again (same pairs, same lanes, same sums), which removes the
// direction test, the count rows and the ring from the adjoint.  The BF16X3
// form's MFMA forward writes the same tape (its pairs in step order), and
// its adjoint given one is this replay.
#include "common.h"

#include <math.h>

namespace {

constexpr int kWaves = 8;
constexpr int kThreads = kWaves * 64;
constexpr int kRing = 128;
constexpr float kPi = 3.14159265358979323846f;

struct ShadeArgs {
  int n, nv, V, kv, he, we, hv, wv, K;
  float cam[3];
  const float *x, *nrm, *albedo, *rough, *tint, *vw, *env;
  const int32_t* vidx;
  const uint8_t* count;
  int patch;   // table slots in 4 x 8 texel patches (the MFMA kernels), else texel order
  // the live-pair tape (NULL: none): per Gaussian its count and its live
  // (direction, visibility) pairs in the order visited, [n][K]
  int32_t* tape_n;
  uint2* tape;
};

// Direction k held by table slot s.  In texel order s = k.  In patch order
// (he % 4 == 0, we % 8 == 0) the slots run over patches of 4 texel rows x 8
// columns, patch-major along each band of 4 rows: slot 32 p + 8 i + j is
// texel (4 (p / (we / 8)) + i, 8 (p % (we / 8)) + j).  A patch is the
// 32-direction reduction step of the MFMA kernels, so the directions of one
// step lie close together and are often all below the horizon (or all
// occluded) for the 16 Gaussians of a tile.
__device__ inline int slot_k(int s, int we, int patch) {
  if (!patch) return s;
  const int p = s >> 5, q = s & 31;
  const int pw = we >> 3;
  const int pr = p / pw, pc = p - pr * pw;
  return (4 * pr + (q >> 3)) * we + 8 * pc + (q & 7);
}

// Table in LDS, two float4 per slot s (direction k = slot_k(s)): [s] =
// (direction x, y, z, view index as int bits), [K + s] = (E = radiance x
// texel solid angle, r, g, b, and the solid angle).  One 16-byte LDS read
// fetches either half.
__device__ inline void build_table(const ShadeArgs& a, float* tab) {
  float4* t4 = reinterpret_cast<float4*>(tab);
  const int K = a.K;
  const float dth = kPi / (float)a.he, dph = 2.f * kPi / (float)a.we;
  // exact solid angle of a texel row: (2 pi / we) * 2 sin(theta_r) sin(pi / (2 he))
  const float band = (2.f * kPi / (float)a.we) * 2.f * sinf(0.5f * dth);
  for (int sl = threadIdx.x; sl < K; sl += blockDim.x) {
    const int k = slot_k(sl, a.we, a.patch);
    const int r = k / a.we, c = k - r * a.we;
    float st, ct, sp, cp;
    sincosf(((float)r + 0.5f) * dth, &st, &ct);
    sincosf(((float)c + 0.5f) * dph, &sp, &cp);
    const float area = band * st;
    const int view = ((r * a.hv) / a.he) * a.wv + (c * a.wv) / a.we;
    t4[sl] = make_float4(st * sp, ct, st * cp, __int_as_float(view));
    t4[K + sl] = make_float4(a.env[3 * k] * area, a.env[3 * k + 1] * area,
                             a.env[3 * k + 2] * area, area);
  }
}

__device__ inline float4 dir_of(const float* tab, int k) {
  return reinterpret_cast<const float4*>(tab)[k];
}
__device__ inline float4 rad_of(const float* tab, int K, int k) {
  return reinterpret_cast<const float4*>(tab)[K + k];
}

struct Attr {
  float x[3], m[3], alb[3], rough, tint, vw[3];
  int vidx[3];
};

// In the wave-per-Gaussian forward (UNI = true) one Gaussian's attributes
// and derived constants are the same in every lane: they are pinned to
// scalar registers, which lowers the vector register count enough for one
// more wave per SIMD.  (The adjoint gains no occupancy from it and pays
// the extra scalar-to-vector moves, so it keeps them in vector registers;
// the MFMA kernels hold a different Gaussian per lane row.)
__device__ inline float uni(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <bool UNI, typename T>
__device__ inline T pin(T v) {
  if constexpr (UNI) return uni(v);
  return v;
}

template <bool UNI>
__device__ inline void attr_load(const ShadeArgs& a, int g, Attr& A) {
  const int n = a.n, nvm = a.nv - 1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    A.x[c] = pin<UNI>(a.x[(size_t)c * n + g]);
    A.m[c] = pin<UNI>(a.nrm[(size_t)c * n + g]);
    A.alb[c] = pin<UNI>(a.albedo[(size_t)c * n + g]);
    A.vw[c] = pin<UNI>(a.vw[(size_t)c * n + g]);
    A.vidx[c] = pin<UNI>(rga::clampi(a.vidx[(size_t)c * n + g], 0, nvm));
  }
  A.rough = pin<UNI>(a.rough[g]);
  A.tint = pin<UNI>(a.tint[g]);
}

// The three visibility-count rows of a Gaussian (3 V bytes, V % 16 == 0) are
// copied straight from global memory into the wave's LDS slot with
// global_load_lds (16 bytes per lane, NQ = ceil(3 V / 1024) per lane), one
// Gaussian ahead, into the other half of a double buffer.
template <int NQ>
__device__ inline void rows_dma(const ShadeArgs& a, const Attr& A, uint8_t* lds, int lane) {
  const int nq = 3 * a.V / 16;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q = lane + 64 * i;
    if (q < nq) {
      const int byte = 16 * q;
      const int j = byte / a.V;
      const int off = byte - j * a.V;
      const int vi = j == 0 ? A.vidx[0] : (j == 1 ? A.vidx[1] : A.vidx[2]);
      __builtin_amdgcn_global_load_lds(a.count + (size_t)vi * a.V + off, lds + 1024 * i, 16, 0, 0);
    }
  }
}

// Wait for every outstanding memory operation of the wave (the row copies).
__device__ inline void wait_all() {
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reciprocal and reciprocal square root on the transcendental unit (about
// 1 ulp).  The shading sums are compared with the FP64 oracle under a
// relative tolerance, never bit for bit, so the correctly rounded
// division sequence buys nothing here.
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

struct GaussCtx {
  float nn[3], wo[3], co, a2, kG, Go, Gq, inn, iwo, alpha, ialpha, gamma;
  float u0, u1, u2;
  const uint8_t* rows;   // LDS copy of the three count rows
  bool front;
};

template <bool UNI>
__device__ inline void gauss_setup(const ShadeArgs& a, const Attr& A, const uint8_t* rows,
                                   GaussCtx& G) {
  const float m0 = A.m[0], m1 = A.m[1], m2 = A.m[2];
  const float w0 = a.cam[0] - A.x[0], w1 = a.cam[1] - A.x[1], w2 = a.cam[2] - A.x[2];
  // back-face decision in FP32 with a fixed operation order
  const float dotf = fmaf(m2, w2, fmaf(m1, w1, m0 * w0));
  G.front = dotf > 0.f;
  G.inn = rsq(fmaf(m2, m2, fmaf(m1, m1, m0 * m0)));
  G.nn[0] = m0 * G.inn;
  G.nn[1] = m1 * G.inn;
  G.nn[2] = m2 * G.inn;
  G.iwo = rsq(fmaf(w2, w2, fmaf(w1, w1, w0 * w0)));
  G.wo[0] = w0 * G.iwo;
  G.wo[1] = w1 * G.iwo;
  G.wo[2] = w2 * G.iwo;
  G.co = fmaf(G.nn[2], G.wo[2], fmaf(G.nn[1], G.wo[1], G.nn[0] * G.wo[0]));
  G.gamma = A.rough;
  G.alpha = G.gamma * G.gamma;
  G.ialpha = rcp(G.alpha);
  G.a2 = G.alpha * G.alpha;
  G.kG = (G.gamma + 1.f) * (G.gamma + 1.f) * 0.125f;
  G.Go = rcp(fmaf(G.co, 1.f - G.kG, G.kG));
  G.Gq = G.Go * (0.25f / kPi);                      // the constant factors of W0
  const float ikv = 1.f / (float)a.kv;
  G.u0 = A.vw[0] * ikv;
  G.u1 = A.vw[1] * ikv;
  G.u2 = A.vw[2] * ikv;
  G.rows = rows;
  if constexpr (UNI) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      G.nn[c] = uni(G.nn[c]);
      G.wo[c] = uni(G.wo[c]);
    }
    G.co = uni(G.co);
    G.a2 = uni(G.a2);
    G.kG = uni(G.kG);
    G.Go = uni(G.Go);
    G.Gq = uni(G.Gq);
    G.inn = uni(G.inn);
    G.iwo = uni(G.iwo);
    G.alpha = uni(G.alpha);
    G.gamma = uni(G.gamma);
    G.u0 = uni(G.u0);
    G.u1 = uni(G.u1);
    G.u2 = uni(G.u2);
  }
}

// Live-direction test for direction k; returns the visibility (0 if dead).
__device__ inline float live_vis(const GaussCtx& G, const float* tab, int K, int V, int k) {
  const float4 dv = dir_of(tab, k);
  const float ci = fmaf(G.nn[2], dv.z, fmaf(G.nn[1], dv.y, G.nn[0] * dv.x));
  if (!(ci > 0.f)) return 0.f;
  const int view = __float_as_int(dv.w);
  const float c0 = (float)G.rows[view], c1 = (float)G.rows[V + view],
              c2 = (float)G.rows[2 * V + view];
  return fmaf(G.u2, c2, fmaf(G.u1, c1, G.u0 * c0));
}

struct Pair {
  float d[3], E[3], ci, ok, hh, nht, s2, den, invh, nh, oh, e2, F, hd, D, G1i, deni, ideni, W0F, W0, Ws,
      Wd;
};

// BRDF weights of one live (Gaussian, direction) pair.  The GGX denominator
// 1 - nh^2 (1 - alpha^2) is formed as (|n x h~|^2 + (n.h~)^2 alpha^2)/|h~|^2
// with h~ = w_k + w_o, which keeps its relative accuracy when nh -> 1.
__device__ inline void pair_eval(const GaussCtx& G, const float* tab, int K, int k, float v,
                                 Pair& P) {
  const float4 dv = dir_of(tab, k), er = rad_of(tab, K, k);
  P.d[0] = dv.x;
  P.d[1] = dv.y;
  P.d[2] = dv.z;
  P.E[0] = er.x;
  P.E[1] = er.y;
  P.E[2] = er.z;
  P.ci = fmaf(G.nn[2], P.d[2], fmaf(G.nn[1], P.d[1], G.nn[0] * P.d[0]));
  P.ok = fmaf(G.wo[2], P.d[2], fmaf(G.wo[1], P.d[1], G.wo[0] * P.d[0]));
  const float h0 = P.d[0] + G.wo[0], h1 = P.d[1] + G.wo[1], h2 = P.d[2] + G.wo[2];
  P.hh = fmaf(h2, h2, fmaf(h1, h1, h0 * h0));
  P.nht = P.ci + G.co;
  const float s0 = G.nn[1] * h2 - G.nn[2] * h1;
  const float s1 = G.nn[2] * h0 - G.nn[0] * h2;
  const float s2 = G.nn[0] * h1 - G.nn[1] * h0;
  P.s2 = fmaf(s2, s2, fmaf(s1, s1, s0 * s0));
  P.den = fmaf(P.nht * P.nht, G.a2, P.s2);           // (1 - nh^2 (1 - a^2)) |h~|^2
  P.invh = rsq(P.hh);
  P.nh = P.nht * P.invh;
  P.oh = (1.f + P.ok) * P.invh;
  // exponent in [-12.6, 0] (o.h in [0, 1]): the hardware exp2 needs no range step
  P.e2 = __builtin_amdgcn_exp2f((-5.55473f * P.oh - 6.98316f) * P.oh);
  P.F = 0.04f + 0.96f * P.e2;
  P.hd = P.hh * rcp(P.den);                         // 1 / (1 - nh^2 (1 - a^2))
  P.D = G.a2 * P.hd * P.hd;                         // pi D
  P.deni = fmaf(P.ci, 1.f - G.kG, G.kG);
  P.ideni = rcp(P.deni);
  P.G1i = P.ci * P.ideni;
  P.W0F = v * P.D * G.Gq;                          // W0 / F
  P.W0 = P.W0F * P.F;
  P.Ws = P.W0 * P.G1i;
  P.Wd = v * P.ci;
}

// x^p for x > 0 (normal) as 2^(p log2 x) on the transcendental unit: a
// few ulp, where the library powf spends ~180 instructions on special
// cases that cannot occur here.
__device__ inline float pos_pow(float x, float p) {
  return __builtin_amdgcn_exp2f(p * __builtin_amdgcn_logf(x));
}

// sRGB transfer curve (gamma correction of L_o)
__device__ inline float srgb(float L) {
  return L <= 0.0031308f ? 12.92f * L : 1.055f * pos_pow(L, 1.f / 2.4f) - 0.055f;
}

// dL/dL_o from dL/dcolour, with L_o recovered from the colour by inverting
// the transfer curve
__device__ inline float srgb_adjoint(float col, float dc) {
  if (col <= 0.04045f) return dc * 12.92f;
  const float Lo = pos_pow((col + 0.055f) / 1.055f, 2.4f);
  return dc * (col + 0.055f) / (2.4f * Lo);
}

__device__ inline void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- FP32 form: one wave per front-facing Gaussian ---------------------------
// A wave owns the Gaussians first, first + stride, first + 2 stride, ...
// (stride = number of waves in the grid).  It takes them 64 at a time: each
// lane loads one Gaussian's position and normal and decides the back-face
// rule; a back-facing Gaussian's outputs are written at once (it needs
// nothing else, and its count rows are never copied), and a ballot gives
// the front-facing ones, which the wave shades one after the other: per
// chunk of 64 directions each lane tests its direction, a ballot compacts
// the live ones into the wave's LDS ring, and whole waves of ring entries
// go to the BRDF stage.  The next front Gaussian's count rows are copied
// into the other half of an LDS double buffer, and its attributes loaded,
// while the current one is shaded.

// Per-lane plan of the count-row copies (depends only on the lane and V):
// 16-byte piece q = lane + 64 i is byte 16 q of the three rows laid end to
// end, i.e. row j = 16 q / V at offset 16 q - j V; packed as off << 2 | j
// (j = 3: no piece).
template <int NQ>
struct RowPlan {
  int p[NQ];
};

template <int NQ>
__device__ inline void row_plan(int V, int lane, RowPlan<NQ>& P) {
  const int nq = 3 * V / 16;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q = lane + 64 * i;
    const int j = (16 * q) / V;
    P.p[i] = q < nq ? ((16 * q - j * V) << 2) | j : 3;
  }
}

template <class Plan>
__device__ inline void rows_copy(const ShadeArgs& a, const Plan& P, const int* vidx,
                                 uint8_t* lds) {
  constexpr int NQ = sizeof(P.p) / sizeof(P.p[0]);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int j = P.p[i] & 3;
    if (j != 3) {
      const int vi = j == 0 ? vidx[0] : (j == 1 ? vidx[1] : vidx[2]);
#if defined(__HIP_DEVICE_COMPILE__)   // a device builtin: the host pass only parses the body
      __builtin_amdgcn_global_load_lds(a.count + (size_t)vi * a.V + (P.p[i] >> 2),
                                       lds + 1024 * i, 16, 0, 0);
#endif
    }
  }
}

// One lane's candidate Gaussian of a block: its index, the back-face rule
// and, if it faces the camera, its three nearest vertices.
struct Cand {
  int g;
  bool front;
  int vidx[3];
};

// The wave's slots of the walk: first, first + stride, ... below `end`.
// With a grid of whole groups of 8 workgroups, the workgroups that share a
// remainder modulo 8 (dispatched to the same XCD, whose L2 they share)
// take one contiguous eighth of the Gaussians: with the Gaussians stored
// grouped by nearest vertex, each XCD then gathers count rows from about an
// eighth of the table, and its L2 holds them.
struct Walk {
  int first, stride, end;
};

__device__ inline Walk wave_walk(int n, int wave) {
  Walk w;
  const int grid = gridDim.x, b = blockIdx.x;
  if (grid % 8 == 0 && grid >= 8) {
    const int x = b % 8, j = b / 8;
    const int lo = (int)((int64_t)n * x / 8), hi = (int)((int64_t)n * (x + 1) / 8);
    w.first = lo + j * kWaves + wave;
    w.stride = (grid / 8) * kWaves;
    w.end = hi;
  } else {
    w.first = b * kWaves + wave;
    w.stride = grid * kWaves;
    w.end = n;
  }
  return w;
}

__device__ inline int walk_count(const Walk& w) {
  return w.first < w.end ? (w.end - 1 - w.first) / w.stride + 1 : 0;
}

// Load block bb of the wave's Gaussians (lane i: Gaussian first + (64 bb + i)
// stride) and decide the back-face rule (FP32, fixed order, as gauss_setup).
__device__ inline void cand_load(const ShadeArgs& a, const Walk& w, int bb, int lane, Cand& C) {
  const int64_t idx = (int64_t)(64 * bb + lane) * w.stride + w.first;
  const bool valid = idx < w.end;
  C.g = valid ? (int)idx : -1;
  C.front = false;
  if (valid) {
    const int n = a.n, g = C.g;
    float x[3], m[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[c] = a.x[(size_t)c * n + g];
      m[c] = a.nrm[(size_t)c * n + g];
    }
    const float w0 = a.cam[0] - x[0], w1 = a.cam[1] - x[1], w2 = a.cam[2] - x[2];
    C.front = fmaf(m[2], w2, fmaf(m[1], w1, m[0] * w0)) > 0.f;
    if (C.front) {
#pragma unroll
      for (int c = 0; c < 3; ++c) C.vidx[c] = rga::clampi(a.vidx[(size_t)c * n + g], 0, a.nv - 1);
    }
  }
}

// The front Gaussian held by lane j of the block: its index and vertices
// from that lane, the other attributes loaded with a wave-uniform address
// (scalar loads into scalar registers).
__device__ inline int cand_take(const ShadeArgs& a, const Cand& C, int j, Attr& A) {
  const int n = a.n;
  const int g = __builtin_amdgcn_readlane(C.g, j);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    A.vidx[c] = __builtin_amdgcn_readlane(C.vidx[c], j);
    A.x[c] = uni(a.x[(size_t)c * n + g]);
    A.m[c] = uni(a.nrm[(size_t)c * n + g]);
    A.alb[c] = uni(a.albedo[(size_t)c * n + g]);
    A.vw[c] = uni(a.vw[(size_t)c * n + g]);
  }
  A.rough = uni(a.rough[g]);
  A.tint = uni(a.tint[g]);
  return g;
}


// Walk the K directions of one Gaussian 64 at a time: lane = direction,
// the live ones (n.w_k > 0 and visibility > 0) appended with their
// visibility to the wave's ring; flush(k, v, on, base) on every whole wave
// of ring entries as it fills and on the remainder (base = the number of
// live pairs flushed before).  Returns the number of live pairs.
template <class Flush>
__device__ inline int live_walk(const GaussCtx& G, const float* tab, int K, int V, int* qk,
                                float* qv, int lane, uint64_t lt, Flush&& flush) {
  int head = 0, tail = 0;
  for (int k0 = 0; k0 < K; k0 += 64) {
    const int k = k0 + lane;
    const float v = k < K ? live_vis(G, tab, K, V, k) : 0.f;
    const bool live = v > 0.f;
    const uint64_t m = __ballot(live);
    if (live) {
      const int slot = (tail + __popcll(m & lt)) & (kRing - 1);
      qk[slot] = k;
      qv[slot] = v;
    }
    tail += __popcll(m);
    if (tail - head >= 64) {
      wave_fence();
      const int slot = (head + lane) & (kRing - 1);
      flush(qk[slot], qv[slot], true, head);
      head += 64;
      wave_fence();
    }
  }
  if (tail > head) {
    wave_fence();
    const int slot = (head + lane) & (kRing - 1);
    flush(qk[slot], qv[slot], lane < tail - head, head);
    wave_fence();
  }
  return tail;
}

// (up to 512 views: three workgroups per CU, six waves per SIMD)
template <int NQ>
__global__ void __launch_bounds__(kThreads, NQ <= 2 ? 6 : 4)
shade_fwd_kernel(ShadeArgs a, float* __restrict__ color, uint8_t* __restrict__ front) {
  extern __shared__ __align__(16) float tab[];
  __shared__ int qk[kWaves][kRing];
  __shared__ float qv[kWaves][kRing];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int K = a.K, n = a.n, V = a.V;
  uint8_t* rows0 = reinterpret_cast<uint8_t*>(tab + 8 * K) + (size_t)wave * 6 * V;
  build_table(a, tab);
  __syncthreads();
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  RowPlan<NQ> plan;
  row_plan<NQ>(V, lane, plan);
  const Walk walk = wave_walk(n, wave);
  const int nblk = (walk_count(walk) + 63) / 64;
  Cand C;
  int b = -1;
  uint64_t fm = 0ull;
  // next block with a front-facing Gaussian; back-facing ones are finished here
  auto advance = [&]() {
    while (fm == 0ull && b + 1 < nblk) {
      ++b;
      cand_load(a, walk, b, lane, C);
      if (C.g >= 0) {
        front[C.g] = C.front ? 1 : 0;
        if (!C.front) {
#pragma unroll
          for (int c = 0; c < 3; ++c) color[(size_t)c * n + C.g] = 0.f;
          if (a.tape_n) a.tape_n[C.g] = 0;
        }
      }
      fm = __ballot(C.front);
    }
  };
  advance();
  if (fm == 0ull) return;
  Attr A;
  int g = cand_take(a, C, __builtin_ctzll(fm), A);
  fm &= fm - 1;
  rows_copy(a, plan, A.vidx, rows0);
  wait_all();
  int cur = 0;
  int og = -1;   // each Gaussian's colour is stored when the next one starts
  float o_col = 0.f;
  for (;;) {
    if (og >= 0 && lane < 3) color[(size_t)lane * n + og] = o_col;
    // the next front-facing Gaussian: its rows and attributes are fetched
    // while this one is shaded
    advance();
    const bool more = fm != 0ull;
    Attr An;
    int gn = -1;
    if (more) {
      gn = cand_take(a, C, __builtin_ctzll(fm), An);
      fm &= fm - 1;
      rows_copy(a, plan, An.vidx, rows0 + (cur ^ 1) * 3 * V);
    }
    GaussCtx G;
    gauss_setup<true>(a, A, rows0 + cur * 3 * V, G);
    float sd0 = 0.f, sd1 = 0.f, sd2 = 0.f, ss0 = 0.f, ss1 = 0.f, ss2 = 0.f;
    // this Gaussian's row of the tape (a wave-uniform address)
    uint2* const trow = a.tape ? a.tape + (size_t)uni(g) * K : nullptr;
    const int nlive = live_walk(G, tab, K, V, qk[wave], qv[wave], lane, lt,
                                [&](int k, float v, bool on, int base) {
      if (on) {
        if (trow) trow[base + lane] = make_uint2((uint32_t)k, __float_as_uint(v));
        Pair P;
        pair_eval(G, tab, K, k, v, P);
        sd0 = fmaf(P.Wd, P.E[0], sd0);
        sd1 = fmaf(P.Wd, P.E[1], sd1);
        sd2 = fmaf(P.Wd, P.E[2], sd2);
        ss0 = fmaf(P.Ws, P.E[0], ss0);
        ss1 = fmaf(P.Ws, P.E[1], ss1);
        ss2 = fmaf(P.Ws, P.E[2], ss2);
      }
    });
    if (trow && lane == 0) a.tape_n[g] = nlive;
    sd0 = rga::wave_sum(sd0);
    sd1 = rga::wave_sum(sd1);
    sd2 = rga::wave_sum(sd2);
    ss0 = rga::wave_sum(ss0);
    ss1 = rga::wave_sum(ss1);
    ss2 = rga::wave_sum(ss2);
    if (lane < 3) {
      const float sd = lane == 0 ? sd0 : (lane == 1 ? sd1 : sd2);
      const float ss = lane == 0 ? ss0 : (lane == 1 ? ss1 : ss2);
      const float alb = lane == 0 ? A.alb[0] : (lane == 1 ? A.alb[1] : A.alb[2]);
      o_col = srgb(alb * (1.f / kPi) * sd + A.tint * ss);
    }
    og = g;
    wait_all();
    wave_fence();
    if (!more) break;
    A = An;
    g = gn;
    cur ^= 1;
  }
  if (lane < 3) color[(size_t)lane * n + og] = o_col;
}

// ---- BF16X3 form: the contraction on MFMA -----------------------------------
// A wave owns 16 Gaussians (MFMA rows) and walks the light directions 32 at
// a time (the MFMA reduction dimension).  Lane l evaluates the BRDF weights of
// Gaussian l % 16 for the 8 directions 8 (l / 16) .. + 7 of the step -- exactly
// its slots of the A operand -- on VALU, splits each weight into bf16 hi + lo,
// and the contraction with B = [E_hi | E_lo] (columns 0-2 and 3-5) runs on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation:
//   S_c = A_hi E_hi + A_hi E_lo + A_lo E_hi + A_lo E_lo (columns c and c+3).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMWaves = 4;
constexpr int kMThreads = kMWaves * 64;

// LDS: dir x,y,z | E r,g,b | view (int) [K each], then B [16 cols][K] bf16
// B operand of the shading contraction in LDS, [6 columns][K] bf16:
// columns 0-2 the high parts of E (r, g, b), 3-5 the low parts.  The other
// ten columns of the 16-wide MFMA operand are zero and never stored.
__device__ inline void build_btab(const float* tab, int K, __bf16* bt) {
  for (int i = threadIdx.x; i < 6 * K; i += blockDim.x) {
    const int col = i / K, k = i - col * K;
    float v = 0.f;
    const float4 er = rad_of(tab, K, k);
    const int cc = col < 3 ? col : col - 3;
    const float e = cc == 0 ? er.x : (cc == 1 ? er.y : er.z);
    v = col < 3 ? (float)(__bf16)e : e - (float)(__bf16)e;
    bt[i] = (__bf16)v;
  }
}

// 8 consecutive k of column `col` of the B operand (zero for col >= 6).
__device__ inline bf16x8 btab_load(const __bf16* bt, int K, int col, int kb) {
  const bf16x8 b = *reinterpret_cast<const bf16x8*>(bt + (size_t)min(col, 5) * K + kb);
  const bf16x8 z = {};
  return col < 6 ? b : z;
}

// visibility bytes of 8 consecutive directions k..k+7 (k % 8 == 0, same
// texel row) for one count row: identity view map (view = k), two texels
// per view (view = k / 2), or the table's view indices
__device__ inline void vis8(const uint8_t* row, const float* tab, int k, int ratio, float* c) {
  if (ratio == 1) {
    const uint2 w = *reinterpret_cast<const uint2*>(row + k);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      c[i] = (float)((w.x >> (8 * i)) & 0xFFu);
      c[4 + i] = (float)((w.y >> (8 * i)) & 0xFFu);
    }
  } else if (ratio == 2) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(row + (k >> 1));
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = (float)((w >> (8 * (i >> 1))) & 0xFFu);
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = (float)row[__float_as_int(dir_of(tab, k + i).w)];
  }
}

// Slots kb .. kb+7 of one lane (8 texels of one row, consecutive in the
// texel order too): the interpolated visibility of each and the mask of
// the live ones (front-facing, n.w_k > 0, visibility > 0).
__device__ inline uint32_t live8(const ShadeArgs& a, const GaussCtx& G, const float* tab,
                                 const uint8_t* r0, const uint8_t* r1, const uint8_t* r2, int kb,
                                 int ratio, bool on, float (&vv)[8]) {
  const int kv = ratio ? slot_k(kb, a.we, a.patch) : kb;
  float c0[8], c1[8], c2[8];
  vis8(r0, tab, kv, ratio, c0);
  vis8(r1, tab, kv, ratio, c1);
  vis8(r2, tab, kv, ratio, c2);
  uint32_t lm = 0u;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float4 dv = dir_of(tab, kb + i);
    const float ci = fmaf(G.nn[2], dv.z, fmaf(G.nn[1], dv.y, G.nn[0] * dv.x));
    vv[i] = fmaf(G.u2, c2[i], fmaf(G.u1, c1[i], G.u0 * c0[i]));
    if (on && ci > 0.f && vv[i] > 0.f) lm |= 1u << i;
  }
  return lm;
}

__global__ void __launch_bounds__(kMThreads)
shade_fwd_mfma_kernel(ShadeArgs a, int ratio, float* __restrict__ color,
                      uint8_t* __restrict__ front) {
  extern __shared__ __align__(16) float tab[];
  const int K = a.K, n = a.n, V = a.V;
  __bf16* bt = reinterpret_cast<__bf16*>(tab + 8 * K);
  float* stage = reinterpret_cast<float*>(bt + 6 * K) + (threadIdx.x >> 6) * 512;
  build_table(a, tab);
  __syncthreads();
  build_btab(tab, K, bt);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, kg = lane >> 4;
  const int ntiles = (n + 15) / 16;
  for (int tile = blockIdx.x * kMWaves + wave; tile < ntiles; tile += gridDim.x * kMWaves) {
    const int g = tile * 16 + row;
    const bool have = g < n;
    Attr A;
    attr_load<false>(a, have ? g : n - 1, A);
    GaussCtx G;
    gauss_setup<false>(a, A, nullptr, G);
    const bool on = have && G.front;
    const uint8_t* r0 = a.count + (size_t)A.vidx[0] * V;
    const uint8_t* r1 = a.count + (size_t)A.vidx[1] * V;
    const uint8_t* r2 = a.count + (size_t)A.vidx[2] * V;
    f32x4 accD = {0.f, 0.f, 0.f, 0.f}, accS = {0.f, 0.f, 0.f, 0.f};
    // the tape: this Gaussian's live pairs so far (the same in the four
    // lanes of its row), written step by step in (step, lane group, i) order
    int tcount = 0;
    uint2* const trow = (a.tape && on) ? a.tape + (size_t)g * K : nullptr;
    for (int k0 = 0; k0 < K; k0 += 32) {
      const int kb = k0 + 8 * kg;
      float vv[8];
      const uint32_t lm = live8(a, G, tab, r0, r1, r2, kb, ratio, on, vv);
      // a step with no live pair in the tile adds nothing
      if (__ballot(lm != 0u) == 0ull) continue;
      if (a.tape) {
        // this lane's pairs follow those of the row's lanes with smaller kg
        const int p = __popc(lm);
        const int p0 = __shfl(p, row), p1 = __shfl(p, row + 16), p2 = __shfl(p, row + 32),
                  p3 = __shfl(p, row + 48);
        int pos = tcount + (kg > 0 ? p0 : 0) + (kg > 1 ? p1 : 0) + (kg > 2 ? p2 : 0);
        if (trow) {
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if ((lm >> i) & 1u)
              trow[pos++] = make_uint2((uint32_t)slot_k(kb + i, a.we, a.patch),
                                       __float_as_uint(vv[i]));
        }
        tcount += p0 + p1 + p2 + p3;
      }
      bf16x8 dh, dl, sh, sl;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = kb + i;
        float Wd = 0.f, Ws = 0.f;
        if ((lm >> i) & 1u) {
          Pair P;
          pair_eval(G, tab, K, k, vv[i], P);
          Wd = P.Wd;
          Ws = P.Ws;
        }
        const __bf16 hd = (__bf16)Wd, hs = (__bf16)Ws;
        dh[i] = hd;
        dl[i] = (__bf16)(Wd - (float)hd);
        sh[i] = hs;
        sl[i] = (__bf16)(Ws - (float)hs);
      }
      const bf16x8 b = btab_load(bt, K, row, kb);
      accD = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dh, b, accD, 0, 0, 0);
      accD = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dl, b, accD, 0, 0, 0);
      accS = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sh, b, accS, 0, 0, 0);
      accS = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sl, b, accS, 0, 0, 0);
    }
    if (a.tape_n && have && kg == 0) a.tape_n[g] = tcount;
    // D[row 4 kg + i][col] -> stage; then one lane per (Gaussian, channel)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      stage[(4 * kg + i) * 16 + row] = accD[i];
      stage[256 + (4 * kg + i) * 16 + row] = accS[i];
    }
    wave_fence();
    if (lane < 48) {
      const int gr = lane / 3, c = lane - 3 * gr;
      const int gg = tile * 16 + gr;
      if (gg < n) {
        const float sd = stage[gr * 16 + c] + stage[gr * 16 + 3 + c];
        const float ss = stage[256 + gr * 16 + c] + stage[256 + gr * 16 + 3 + c];
        // this Gaussian's inputs (lane gr of the tile holds them)
        const float alb = a.albedo[(size_t)c * n + gg];
        const float tnt = a.tint[gg];
        const float m0 = a.nrm[gg], m1 = a.nrm[n + gg], m2 = a.nrm[2 * n + gg];
        const float w0 = a.cam[0] - a.x[gg], w1 = a.cam[1] - a.x[n + gg],
                    w2 = a.cam[2] - a.x[2 * n + gg];
        const bool fr = fmaf(m2, w2, fmaf(m1, w1, m0 * w0)) > 0.f;
        color[(size_t)c * n + gg] = fr ? srgb(alb * (1.f / kPi) * sd + tnt * ss) : 0.f;
        if (c == 0) front[gg] = fr ? 1 : 0;
      }
    }
    wave_fence();
  }
}

// ---- adjoint ------------------------------------------------------------
struct BwdAcc {
  float gn[3], gw[3], gco, gga, sd[3], ts;
};

// Chain rule through one live pair's weights: upstream gWd = dL/dW_d and
// gWs = dL/dW_s give the pair's share of dL/dn^, dL/dw_o, dL/d(n.w_o) and
// dL/dgamma.  Uses the logarithmic derivatives of D (in n.h and alpha), F
// (through dF/d(o.h)) and G1.  Only the part of dL/dw_o orthogonal to w_o
// reaches x, so the w_o terms are taken along h = h~/|h~|: n.h changes by
// (n - (n.h) h)/|h~| and o.h = |h~|/2 by h/2 (up to multiples of w_o).  The
// same derivative taken through o.w_k (d(n.h)/d(o.w_k) = -(n.h~)/|h~|^3)
// is of size 1/|h~|^2 near w_k = -w_o, almost all of it along w_o, and the
// projection onto the tangent plane then cancels it in FP32.
__device__ inline void pair_grads(const GaussCtx& G, const Pair& P, float v, float gWd, float gWs,
                                  BwdAcc& acc) {
  const float one_m_a2 = 1.f - G.a2;
  const float dlnD_dnh = 4.f * P.nh * one_m_a2 * P.hd;
  const float dlnD_da = 2.f * G.ialpha - 4.f * G.alpha * P.nh * P.nh * P.hd;
  // dF/d(o.h); gs dlnF/d(o.h) = gWs (W_s / F) dF/d(o.h) needs no 1/F
  const float dF_doh = 0.96f * P.e2 * 0.69314718f * (-2.f * 5.55473f * P.oh - 6.98316f);
  const float gs = gWs * P.Ws;
  const float gsF = gWs * P.W0F * P.G1i * dF_doh;
  const float gnh = gs * dlnD_dnh * P.invh;          // dL/d(n.h~) through D
  const float gci = gWd * v + gWs * P.W0 * G.kG * (P.ideni * P.ideni) + gnh;
  const float gco = gnh - gs * (1.f - G.kG) * G.Go;
  // dL/dw_o = gco n + ghh h~ (modulo w_o)
  const float ghh = fmaf(-gnh, P.nh, 0.5f * gsF) * P.invh;
  const float dlnG_dk = -(1.f - P.ci) * P.ideni - (1.f - G.co) * G.Go;
  const float gga = gs * (dlnD_da * 2.f * G.gamma + dlnG_dk * (G.gamma + 1.f) * 0.25f);
  acc.gn[0] = fmaf(gci, P.d[0], acc.gn[0]);
  acc.gn[1] = fmaf(gci, P.d[1], acc.gn[1]);
  acc.gn[2] = fmaf(gci, P.d[2], acc.gn[2]);
  acc.gw[0] = fmaf(ghh, P.d[0] + G.wo[0], acc.gw[0]);
  acc.gw[1] = fmaf(ghh, P.d[1] + G.wo[1], acc.gw[1]);
  acc.gw[2] = fmaf(ghh, P.d[2] + G.wo[2], acc.gw[2]);
  acc.gco += gco;
  acc.gga += gga;
}

__device__ inline void pair_bwd(const GaussCtx& G, const float* tab, float* denv_lds, int K, int k,
                                float v, const float* qd, const float* dLo, float tint,
                                const float* aop, BwdAcc& acc) {
  Pair P;
  pair_eval(G, tab, K, k, v, P);
  // upstream weights of W_d and W_s
  const float gWd = fmaf(qd[2], P.E[2], fmaf(qd[1], P.E[1], qd[0] * P.E[0]));
  const float sE = fmaf(dLo[2], P.E[2], fmaf(dLo[1], P.E[1], dLo[0] * P.E[0]));
  const float gWs = tint * sE;
  acc.sd[0] = fmaf(P.Wd, P.E[0], acc.sd[0]);
  acc.sd[1] = fmaf(P.Wd, P.E[1], acc.sd[1]);
  acc.sd[2] = fmaf(P.Wd, P.E[2], acc.sd[2]);
  acc.ts = fmaf(P.Ws, sE, acc.ts);
  // environment: dL/d(L_k,c A_k) = dLo_c (a_c/pi W_d + p W_s); the area
  // factor is applied when the per-workgroup sums are reduced
  rga::lds_add3(&denv_lds[3 * k], dLo[0] * fmaf(aop[0], P.Wd, tint * P.Ws),
                dLo[1] * fmaf(aop[1], P.Wd, tint * P.Ws), dLo[2] * fmaf(aop[2], P.Wd, tint * P.Ws));
  pair_grads(G, P, v, gWd, gWs, acc);
}

// BF16X3 adjoint.  Same tiling (16 Gaussians x 32 directions per step).  On
// MFMA: the per-Gaussian sums S_d = W_d E and S_s = W_s E (for the albedo and
// tint gradients, 16x16x32 as in the forward), and the environment gradient
// dE[k][c] = sum_g W_d[g][k] Qd[g][c] + W_s[g][k] Qs[g][c] with
// Qd = dL/dL_o a / pi, Qs = dL/dL_o p -- a reduction over Gaussians, so W is
// transposed through LDS and fed to v_mfma_f32_32x32x16_bf16 (A = W^T,
// 32 directions x 16 Gaussians; B = [Q_hi | Q_lo]).  The direction-dependent
// derivative terms of the BRDF weights stay on VALU in FP32.
typedef float f32x16 __attribute__((ext_vector_type(16)));

__global__ void __launch_bounds__(kMThreads)
shade_bwd_mfma_kernel(ShadeArgs a, int ratio, const float* __restrict__ color,
                      const float* __restrict__ dcolor, float* __restrict__ dx,
                      float* __restrict__ dn, float* __restrict__ dalbedo,
                      float* __restrict__ drough, float* __restrict__ dtint,
                      float* __restrict__ denv_part) {
  extern __shared__ __align__(16) float tab[];
  const int K = a.K, n = a.n, V = a.V;
  __bf16* bt = reinterpret_cast<__bf16*>(tab + 8 * K);
  float* denv_lds = reinterpret_cast<float*>(bt + 6 * K);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // per-wave scratch: W^T stage (4 x [32 k][16 g] bf16 = 4 KB), Q (16 x 6 f32),
  // per-Gaussian sums (2 x 256 f32)
  char* wbase = reinterpret_cast<char*>(denv_lds + 3 * K) + (size_t)wave * (4096 + 384 + 2048);
  __bf16* wt = reinterpret_cast<__bf16*>(wbase);
  float* qst = reinterpret_cast<float*>(wbase + 4096);
  float* stage = reinterpret_cast<float*>(wbase + 4096 + 384);
  build_table(a, tab);
  for (int i = threadIdx.x; i < 3 * K; i += blockDim.x) denv_lds[i] = 0.f;
  __syncthreads();
  build_btab(tab, K, bt);
  __syncthreads();
  const int row = lane & 15, kg = lane >> 4;
  const int ntiles = (n + 15) / 16;
  for (int tile = blockIdx.x * kMWaves + wave; tile < ntiles; tile += gridDim.x * kMWaves) {
    const int g = tile * 16 + row;
    const bool have = g < n;
    const int gc = have ? g : n - 1;
    Attr A;
    attr_load<false>(a, gc, A);
    GaussCtx G;
    gauss_setup<false>(a, A, nullptr, G);
    const bool on = have && G.front;
    float dLo[3], aop[3], qd[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float col = color[(size_t)c * n + gc];
      const float dc = on ? dcolor[(size_t)c * n + gc] : 0.f;
      dLo[c] = srgb_adjoint(col, dc);
      aop[c] = A.alb[c] * (1.f / kPi);
      qd[c] = dLo[c] * aop[c];
    }
    const float tint = A.tint;
    // B operand of the environment contraction: Q of the tile's 16 Gaussians
    if (kg == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        qst[row * 6 + c] = qd[c];
        qst[row * 6 + 3 + c] = dLo[c] * tint;
      }
    }
    wave_fence();
    bf16x8 bqd, bqs;   // B [16 g][32 cols]: lane holds col lane % 32, g = 8 (lane / 32) + i
    {
      const int col = lane & 31, g0 = 8 * (lane >> 5);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        float vd = 0.f, vs = 0.f;
        if (col < 6) {
          const float qdv = qst[(g0 + i) * 6 + (col % 3)];
          const float qsv = qst[(g0 + i) * 6 + 3 + (col % 3)];
          vd = col < 3 ? (float)(__bf16)qdv : qdv - (float)(__bf16)qdv;
          vs = col < 3 ? (float)(__bf16)qsv : qsv - (float)(__bf16)qsv;
        }
        bqd[i] = (__bf16)vd;
        bqs[i] = (__bf16)vs;
      }
    }
    const uint8_t* r0 = a.count + (size_t)A.vidx[0] * V;
    const uint8_t* r1 = a.count + (size_t)A.vidx[1] * V;
    const uint8_t* r2 = a.count + (size_t)A.vidx[2] * V;
    f32x4 accD = {0.f, 0.f, 0.f, 0.f}, accS = {0.f, 0.f, 0.f, 0.f};
    BwdAcc acc = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, 0.f, 0.f, {0.f, 0.f, 0.f}, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
      const int kb = k0 + 8 * kg;
      float vv[8];
      const uint32_t lm = live8(a, G, tab, r0, r1, r2, kb, ratio, on, vv);
      // a step with no live pair in the tile adds nothing (W = 0)
      if (__ballot(lm != 0u) == 0ull) continue;
      bf16x8 dh, dl, sh, sl;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = kb + i;
        float Wd = 0.f, Ws = 0.f;
        if ((lm >> i) & 1u) {
          Pair P;
          pair_eval(G, tab, K, k, vv[i], P);
          Wd = P.Wd;
          Ws = P.Ws;
          const float gWd = fmaf(qd[2], P.E[2], fmaf(qd[1], P.E[1], qd[0] * P.E[0]));
          const float sE = fmaf(dLo[2], P.E[2], fmaf(dLo[1], P.E[1], dLo[0] * P.E[0]));
          const float gWs = tint * sE;
          pair_grads(G, P, vv[i], gWd, gWs, acc);
        }
        const __bf16 hd = (__bf16)Wd, hs = (__bf16)Ws;
        dh[i] = hd;
        dl[i] = (__bf16)(Wd - (float)hd);
        sh[i] = hs;
        sl[i] = (__bf16)(Ws - (float)hs);
        // W^T stage [k local][g]
        const int kl = 8 * kg + i;
        wt[0 * 512 + kl * 16 + row] = dh[i];
        wt[1 * 512 + kl * 16 + row] = dl[i];
        wt[2 * 512 + kl * 16 + row] = sh[i];
        wt[3 * 512 + kl * 16 + row] = sl[i];
      }
      const bf16x8 b = btab_load(bt, K, row, kb);
      accD = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dh, b, accD, 0, 0, 0);
      accD = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dl, b, accD, 0, 0, 0);
      accS = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sh, b, accS, 0, 0, 0);
      accS = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sl, b, accS, 0, 0, 0);
      wave_fence();
      // environment: A = W^T [32 k][16 g]; lane holds k = lane % 32, g = 8 (lane / 32) + i
      const int kr = lane & 31, gq = 8 * (lane >> 5);
      const bf16x8 adh = *reinterpret_cast<const bf16x8*>(wt + 0 * 512 + kr * 16 + gq);
      const bf16x8 adl = *reinterpret_cast<const bf16x8*>(wt + 1 * 512 + kr * 16 + gq);
      const bf16x8 ash = *reinterpret_cast<const bf16x8*>(wt + 2 * 512 + kr * 16 + gq);
      const bf16x8 asl = *reinterpret_cast<const bf16x8*>(wt + 3 * 512 + kr * 16 + gq);
      f32x16 de;
#pragma unroll
      for (int i = 0; i < 16; ++i) de[i] = 0.f;
      de = __builtin_amdgcn_mfma_f32_32x32x16_bf16(adh, bqd, de, 0, 0, 0);
      de = __builtin_amdgcn_mfma_f32_32x32x16_bf16(adl, bqd, de, 0, 0, 0);
      de = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ash, bqs, de, 0, 0, 0);
      de = __builtin_amdgcn_mfma_f32_32x32x16_bf16(asl, bqs, de, 0, 0, 0);
      // D[k][col]: lane holds col = lane % 32, rows 8 (i / 4) + 4 (lane / 32) + i % 4
      const int col = lane & 31;
      if (col < 6) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int kk = k0 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
          atomicAdd(&denv_lds[3 * kk + (col % 3)], de[i]);
        }
      }
      wave_fence();
    }
    // per-Gaussian sums from the forward-style MFMA: D[row 4 kg + i][col]
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      stage[(4 * kg + i) * 16 + row] = accD[i];
      stage[256 + (4 * kg + i) * 16 + row] = accS[i];
    }
    // VALU partial sums of the four lanes of each Gaussian row
    float r8[8] = {acc.gn[0], acc.gn[1], acc.gn[2], acc.gw[0], acc.gw[1], acc.gw[2], acc.gco, acc.gga};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      r8[q] += __shfl_xor(r8[q], 16, 64);
      r8[q] += __shfl_xor(r8[q], 32, 64);
    }
    wave_fence();
    if (kg == 0 && have) {
      if (!G.front) {
        for (int c = 0; c < 3; ++c) {
          dn[(size_t)c * n + g] = 0.f;
          dalbedo[(size_t)c * n + g] = 0.f;
        }
        drough[g] = 0.f;
        dtint[g] = 0.f;
      } else {
        const float gco = r8[6];
        float gn3[3] = {r8[0] + gco * G.wo[0], r8[1] + gco * G.wo[1], r8[2] + gco * G.wo[2]};
        float gw[3] = {r8[3] + gco * G.nn[0], r8[4] + gco * G.nn[1], r8[5] + gco * G.nn[2]};
        const float pn = gn3[0] * G.nn[0] + gn3[1] * G.nn[1] + gn3[2] * G.nn[2];
        const float pw = gw[0] * G.wo[0] + gw[1] * G.wo[1] + gw[2] * G.wo[2];
        float ts = 0.f;
        for (int c = 0; c < 3; ++c) {
          const float sd = stage[row * 16 + c] + stage[row * 16 + 3 + c];
          const float ss = stage[256 + row * 16 + c] + stage[256 + row * 16 + 3 + c];
          dn[(size_t)c * n + g] = (gn3[c] - G.nn[c] * pn) * G.inn;
          dx[(size_t)c * n + g] += -(gw[c] - G.wo[c] * pw) * G.iwo;
          dalbedo[(size_t)c * n + g] = dLo[c] * sd * (1.f / kPi);
          ts = fmaf(dLo[c], ss, ts);
        }
        drough[g] = r8[7];
        dtint[g] = ts;
      }
    }
    wave_fence();
  }
  __syncthreads();
  // LDS sums are in slot order; the partials in texel order
  float* out = denv_part + (size_t)blockIdx.x * 3 * K;
  for (int i = threadIdx.x; i < 3 * K; i += blockDim.x) {
    const int sl = i / 3, c = i - 3 * sl;
    out[3 * slot_k(sl, a.we, a.patch) + c] = denv_lds[i];
  }
}

// (up to 512 views: two workgroups per CU, four waves per SIMD, at most
// 128 VGPRs).  With TAPE the live pairs of each Gaussian are read from the
// forward's tape, in the order and 64-pair groups the walk would produce
// them (so the sums are the same), instead of testing every direction: no
// count rows, no ring.
template <int NQ, bool TAPE>
__global__ void __launch_bounds__(kThreads, NQ <= 2 ? 4 : 2)
shade_bwd_kernel(ShadeArgs a, const float* __restrict__ color, const float* __restrict__ dcolor,
                 float* __restrict__ dx, float* __restrict__ dn, float* __restrict__ dalbedo,
                 float* __restrict__ drough, float* __restrict__ dtint,
                 float* __restrict__ denv_part /*[grid][K][3]*/) {
  extern __shared__ __align__(16) float tab[];
  __shared__ int qk[kWaves][kRing];
  __shared__ float qv[kWaves][kRing];
  const int K = a.K, n = a.n, V = a.V;
  float* denv_lds = tab + 8 * K;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint8_t* rows0 = TAPE ? nullptr : reinterpret_cast<uint8_t*>(tab + 11 * K) + (size_t)wave * 6 * V;
  build_table(a, tab);
  for (int i = threadIdx.x; i < 3 * K; i += blockDim.x) denv_lds[i] = 0.f;
  __syncthreads();
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  RowPlan<NQ> plan;
  row_plan<NQ>(V, lane, plan);
  const Walk walk = wave_walk(n, wave);
  const int nblk = (walk_count(walk) + 63) / 64;
  // Lane c < 3 handles channel c of the per-Gaussian inputs and outputs.
  const int ch = min(lane, 2);
  Cand C;
  int b = -1;
  uint64_t fm = 0ull;
  // next block with a front-facing Gaussian; a back-facing one gets zero
  // gradients (dx, accumulated, is left as it is)
  auto advance = [&]() {
    while (fm == 0ull && b + 1 < nblk) {
      ++b;
      cand_load(a, walk, b, lane, C);
      if (C.g >= 0 && !C.front) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          dn[(size_t)c * n + C.g] = 0.f;
          dalbedo[(size_t)c * n + C.g] = 0.f;
        }
        drough[C.g] = 0.f;
        dtint[C.g] = 0.f;
      }
      fm = __ballot(C.front);
    }
  };
  advance();
  if (fm != 0ull) {
    Attr A;
    int g = cand_take(a, C, __builtin_ctzll(fm), A);
    fm &= fm - 1;
    // TAPE: the Gaussian's live count and first 64 pairs (lane < K keeps
    // the read inside the Gaussian's row of the tape)
    int tl = 0;
    uint2 tw = make_uint2(0u, 0u);
    if constexpr (TAPE) {
      tl = a.tape_n[g];
      if (lane < K) tw = a.tape[(size_t)g * K + lane];
    } else {
      rows_copy(a, plan, A.vidx, rows0);
    }
    float pcol = color[(size_t)ch * n + g], pdc = dcolor[(size_t)ch * n + g];
    wait_all();
    int cur = 0;
    int og = -1;   // Gaussian whose outputs are pending
    float o_dn = 0.f, o_dalb = 0.f, o_dx = 0.f, o_rough = 0.f, o_tint = 0.f;
    for (;;) {
      if (og >= 0) {
        if (lane < 3) {
          dn[(size_t)lane * n + og] = o_dn;
          dalbedo[(size_t)lane * n + og] = o_dalb;
          dx[(size_t)lane * n + og] = o_dx;
        }
        if (lane == 0) {
          drough[og] = o_rough;
          dtint[og] = o_tint;
        }
      }
      const float col = pcol, dcol = pdc;
      const float dx_in = dx[(size_t)ch * n + g];
      advance();
      const bool more = fm != 0ull;
      Attr An;
      int gn = -1;
      int tln = 0;
      uint2 twn = make_uint2(0u, 0u);
      if (more) {
        gn = cand_take(a, C, __builtin_ctzll(fm), An);
        fm &= fm - 1;
        if constexpr (TAPE) {
          tln = a.tape_n[gn];
          if (lane < K) twn = a.tape[(size_t)gn * K + lane];
        } else {
          rows_copy(a, plan, An.vidx, rows0 + (cur ^ 1) * 3 * V);
        }
        pcol = color[(size_t)ch * n + gn];
        pdc = dcolor[(size_t)ch * n + gn];
      }
      GaussCtx G;
      gauss_setup<true>(a, A, TAPE ? nullptr : rows0 + cur * 3 * V, G);
      // dL/dL_o: lane c < 3 takes channel c, every lane reads the three
      float dLo[3], aop[3], qd[3];
      {
        const float d = srgb_adjoint(col, dcol);
#pragma unroll
        for (int q = 0; q < 3; ++q)
          dLo[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), q));
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        aop[c] = A.alb[c] * (1.f / kPi);
        qd[c] = dLo[c] * aop[c];
      }
      const float tint = A.tint;
      BwdAcc acc = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, 0.f, 0.f, {0.f, 0.f, 0.f}, 0.f};
      if constexpr (TAPE) {
        // 64 pairs at a time, the next group's read issued before this one
        uint2 w = tw;
        for (int base = 0; base < tl; base += 64) {
          uint2 wn2 = make_uint2(0u, 0u);
          if (base + 64 < tl && base + 64 + lane < K) wn2 = a.tape[(size_t)g * K + base + 64 + lane];
          if (base + lane < tl)
            pair_bwd(G, tab, denv_lds, K, (int)w.x, __uint_as_float(w.y), qd, dLo, tint, aop, acc);
          w = wn2;
        }
      } else {
        live_walk(G, tab, K, V, qk[wave], qv[wave], lane, lt, [&](int k, float v, bool on, int) {
          if (on) pair_bwd(G, tab, denv_lds, K, k, v, qd, dLo, tint, aop, acc);
        });
      }
      // per-Gaussian sums of the twelve partials over the wave: four slots
      // of three values (lane swaps and DPP), slot s summed in row s
      float r[12];
      {
        float v4[4][3] = {{acc.gn[0], acc.gn[1], acc.gn[2]},
                          {acc.gw[0], acc.gw[1], acc.gw[2]},
                          {acc.gco, acc.gga, acc.ts},
                          {acc.sd[0], acc.sd[1], acc.sd[2]}};
        float o3[3];
        rga::slot_sums4<3>(v4, o3);
#pragma unroll
        for (int sl = 0; sl < 4; ++sl)
#pragma unroll
          for (int q = 0; q < 3; ++q)
            r[3 * sl + q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(o3[q]), 16 * sl));
      }
      // r: gn 0-2, gw 3-5, gco 6, gga 7, ts 8, sd 9-11
      {
        const float gco = r[6];
        float gn3[3] = {r[0] + gco * G.wo[0], r[1] + gco * G.wo[1], r[2] + gco * G.wo[2]};
        float gw[3] = {r[3] + gco * G.nn[0], r[4] + gco * G.nn[1], r[5] + gco * G.nn[2]};
        const float pn = gn3[0] * G.nn[0] + gn3[1] * G.nn[1] + gn3[2] * G.nn[2];
        const float pw = gw[0] * G.wo[0] + gw[1] * G.wo[1] + gw[2] * G.wo[2];
        const int c = ch;
        const float gnc = c == 0 ? gn3[0] : (c == 1 ? gn3[1] : gn3[2]);
        const float gwc = c == 0 ? gw[0] : (c == 1 ? gw[1] : gw[2]);
        const float nnc = c == 0 ? G.nn[0] : (c == 1 ? G.nn[1] : G.nn[2]);
        const float woc = c == 0 ? G.wo[0] : (c == 1 ? G.wo[1] : G.wo[2]);
        const float dlc = c == 0 ? dLo[0] : (c == 1 ? dLo[1] : dLo[2]);
        const float sdc = c == 0 ? r[9] : (c == 1 ? r[10] : r[11]);
        o_dn = (gnc - nnc * pn) * G.inn;
        // w_o = (cam - x)/|cam - x|: d/dx = -(I - w w^T)/|cam - x|
        o_dx = dx_in - (gwc - woc * pw) * G.iwo;
        o_dalb = dlc * sdc * (1.f / kPi);
        o_rough = r[7];
        o_tint = r[8];
      }
      og = g;
      wait_all();
      wave_fence();
      if (!more) break;
      A = An;
      g = gn;
      tl = tln;
      tw = twn;
      cur ^= 1;
    }
    if (lane < 3) {
      dn[(size_t)lane * n + og] = o_dn;
      dalbedo[(size_t)lane * n + og] = o_dalb;
      dx[(size_t)lane * n + og] = o_dx;
    }
    if (lane == 0) {
      drough[og] = o_rough;
      dtint[og] = o_tint;
    }
  }
  __syncthreads();
  float* out = denv_part + (size_t)blockIdx.x * 3 * K;
  for (int i = threadIdx.x; i < 3 * K; i += blockDim.x) out[i] = denv_lds[i];
}

// denv[k][c] = area_k * sum over workgroups.  Each block owns 64 outputs;
// its 1024 threads split the partials into 16 interleaved groups and the
// groups are added in a fixed tree order (deterministic).
__global__ void __launch_bounds__(1024)
denv_reduce_kernel(int K, int he, int we, int parts, const float* __restrict__ part,
                   float* __restrict__ denv) {
  __shared__ float red[16][64];
  const int o = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + o;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  if (i < 3 * K) {
    int p = grp;
    for (; p + 48 < parts; p += 64) {
      s0 += part[(size_t)p * 3 * K + i];
      s1 += part[(size_t)(p + 16) * 3 * K + i];
      s2 += part[(size_t)(p + 32) * 3 * K + i];
      s3 += part[(size_t)(p + 48) * 3 * K + i];
    }
    for (; p < parts; p += 16) s0 += part[(size_t)p * 3 * K + i];
  }
  red[grp][o] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  for (int h = 8; h > 0; h >>= 1) {
    if (grp < h) red[grp][o] += red[grp + h][o];
    __syncthreads();
  }
  if (grp == 0 && i < 3 * K) {
    const int k = i / 3, r = k / we;
    const float dth = kPi / (float)he;
    const float area = (2.f * kPi / (float)we) * 2.f * sinf(0.5f * dth) * sinf(((float)r + 0.5f) * dth);
    denv[i] = red[0][o] * area;
  }
}

template <int NQ>
void set_lds_limits_nq() {
  const void* ks[] = {reinterpret_cast<const void*>(shade_fwd_kernel<NQ>),
                      reinterpret_cast<const void*>(shade_bwd_kernel<NQ, false>),
                      reinterpret_cast<const void*>(shade_bwd_kernel<NQ, true>)};
  for (const void* k : ks) hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 152 * 1024);
}

void set_lds_limits() {
  static bool done = false;
  if (done) return;
  set_lds_limits_nq<2>();
  set_lds_limits_nq<6>();
  done = true;
}

// LDS of the FP32 kernels (dynamic part, at most 152 KB beside the static
// 8 KB of the rings): the direction table (8 K floats; the adjoint adds 3 K
// for the environment gradient) and each wave's double buffer of three
// count rows (6 V bytes).
inline size_t fp32_lds(int K, int V, bool adjoint) {
  return (size_t)(adjoint ? 11 : 8) * K * sizeof(float) + (size_t)kWaves * 6 * V;
}

// Persistent grid: as many workgroups as the device holds at once (every
// workgroup resident, so the static division of the Gaussians over the
// waves is also the division of the work), from the occupancy of the exact
// kernel at its LDS size; never more than one wave per Gaussian.
int grid_for(const void* kernel, int n, size_t lds) {
  set_lds_limits();
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
      ncu = 256;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  int grid = ncu * per_cu;
  const int need = (int)rga::ceil_div(n, kWaves);
  return grid < need ? grid : (need > 0 ? need : 1);
}

// The FP32 kernel instance for the number of 1024-byte pieces of a
// Gaussian's three count rows.
// (The adjoint that reads a tape copies no rows: one instance serves every
// view count.)
const void* fp32_kernel(bool adjoint, int nq, bool tape = false) {
  if (adjoint && tape) return reinterpret_cast<const void*>(shade_bwd_kernel<2, true>);
  if (nq <= 2)
    return adjoint ? reinterpret_cast<const void*>(shade_bwd_kernel<2, false>)
                   : reinterpret_cast<const void*>(shade_fwd_kernel<2>);
  return adjoint ? reinterpret_cast<const void*>(shade_bwd_kernel<6, false>)
                 : reinterpret_cast<const void*>(shade_fwd_kernel<6>);
}

int check_args(const char* fn, int n, const float* x, const float* nrm, const float* albedo,
               const float* rough, const float* tint, const int32_t* vidx, const float* vw,
               const uint8_t* count, int nv, int kv, int he, int we, int hv, int wv,
               const float* env, const float* cam_pos, int precision) {
  if (n < 0) return rga::fail(RGA_EINVAL, "%s: n < 0", fn);
  if (he < 1 || we < 1 || hv < 1 || wv < 1 || he % hv || we % wv)
    return rga::fail(RGA_EINVAL, "%s: view grid %dx%d must divide the map %dx%d", fn, hv, wv, he, we);
  if ((int64_t)he * we > 3584)
    return rga::fail(RGA_EUNSUPPORTED, "%s: at most 3584 light directions (LDS table)", fn);
  if (nv < 1 || kv < 1) return rga::fail(RGA_EINVAL, "%s: nv, kv >= 1", fn);
  if ((hv * wv) % 16 != 0 || hv * wv > 2048)
    return rga::fail(RGA_EUNSUPPORTED, "%s: the view count must be a multiple of 16, at most 2048", fn);
  if (count && !rga::aligned16(count))
    return rga::fail(RGA_EINVAL, "%s: count must be 16-byte aligned", fn);
  if (!cam_pos || !env) return rga::fail(RGA_EINVAL, "%s: null env or cam_pos", fn);
  if (precision != RGA_FP32 && precision != RGA_BF16X3)
    return rga::fail(RGA_EINVAL, "%s: unknown precision %d", fn, precision);
  if (n > 0 && (!x || !nrm || !albedo || !rough || !tint || !vidx || !vw || !count))
    return rga::fail(RGA_EINVAL, "%s: null input", fn);
  return RGA_OK;
}

ShadeArgs make_args(int n, const float* x, const float* nrm, const float* albedo,
                    const float* rough, const float* tint, const int32_t* vidx, const float* vw,
                    const uint8_t* count, int nv, int kv, int he, int we, int hv, int wv,
                    const float* env, const float* cam_pos) {
  ShadeArgs a;
  a.n = n;
  a.nv = nv;
  a.V = hv * wv;
  a.kv = kv;
  a.he = he;
  a.we = we;
  a.hv = hv;
  a.wv = wv;
  a.K = he * we;
  for (int i = 0; i < 3; ++i) a.cam[i] = cam_pos[i];
  a.x = x;
  a.nrm = nrm;
  a.albedo = albedo;
  a.rough = rough;
  a.tint = tint;
  a.vw = vw;
  a.env = env;
  a.vidx = vidx;
  a.count = count;
  a.patch = 0;
  a.tape_n = nullptr;
  a.tape = nullptr;
  return a;
}

}  // namespace

// The live-pair tape: [n] int32 counts (256-byte aligned block), then
// [n][K] (direction, visibility bits) pairs.
extern "C" size_t shade_tape_bytes(int n, int he, int we) {
  if (n < 0 || he < 1 || we < 1) return 0;
  return rga::align_up((size_t)4 * (n > 0 ? n : 1), 256) + (size_t)8 * n * he * we;
}

namespace {
int attach_tape(const char* fn, ShadeArgs& a, const void* tape, size_t tape_bytes) {
  if (!tape) return RGA_OK;
  if (!rga::aligned16(tape)) return rga::fail(RGA_EINVAL, "%s: tape must be 16-byte aligned", fn);
  if (tape_bytes < shade_tape_bytes(a.n, a.he, a.we))
    return rga::fail(RGA_ECAPACITY, "%s: tape %zu < %zu bytes", fn, tape_bytes,
                     shade_tape_bytes(a.n, a.he, a.we));
  char* t = static_cast<char*>(const_cast<void*>(tape));
  a.tape_n = reinterpret_cast<int32_t*>(t);
  a.tape = reinterpret_cast<uint2*>(t + rga::align_up((size_t)4 * (a.n > 0 ? a.n : 1), 256));
  return RGA_OK;
}
}  // namespace

extern "C" int shade_gaussians(void* stream, int n, const float* x, const float* nrm,
                               const float* albedo, const float* rough, const float* tint,
                               const int32_t* vidx, const float* vw, const uint8_t* count, int nv,
                               int kv, int he, int we, int hv, int wv, const float* env,
                               const float* cam_pos, int precision, float* color,
                               uint8_t* front, void* tape, size_t tape_bytes) {
  int rc = check_args("shade_gaussians", n, x, nrm, albedo, rough, tint, vidx, vw, count, nv, kv,
                      he, we, hv, wv, env, cam_pos, precision);
  if (rc) return rc;
  if (n == 0) return RGA_OK;
  if (!color || !front) return rga::fail(RGA_EINVAL, "shade_gaussians: null output");
  ShadeArgs a = make_args(n, x, nrm, albedo, rough, tint, vidx, vw, count, nv, kv, he, we, hv, wv,
                          env, cam_pos);
  rc = attach_tape("shade_gaussians", a, tape, tape_bytes);
  if (rc) return rc;
  if (precision == RGA_BF16X3) {
    if (a.K % 32 != 0)
      return rga::fail(RGA_EUNSUPPORTED, "shade_gaussians: BF16X3 needs a multiple of 32 directions");
    const int ratio = (hv == he && we == wv) ? 1 : ((hv == he && we == 2 * wv && we % 8 == 0) ? 2 : 0);
    a.patch = (he % 4 == 0 && we % 8 == 0) ? 1 : 0;
    const size_t lds = (size_t)8 * a.K * sizeof(float) + (size_t)6 * a.K * 2 + kMWaves * 512 * 4;
    static bool mattr = false;
    if (!mattr) {
      hipFuncSetAttribute(reinterpret_cast<const void*>(shade_fwd_mfma_kernel),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
      mattr = true;
    }
    if (lds > 150 * 1024) return rga::fail(RGA_EUNSUPPORTED, "shade_gaussians: too many directions");
    int ncu = 0, dev = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
      ncu = 256;
    const int per_cu = lds <= 40 * 1024 ? 4 : (lds <= 76 * 1024 ? 2 : 1);
    const int tiles = (int)rga::ceil_div(n, 16);
    int grid = ncu * per_cu;
    const int need = (int)rga::ceil_div(tiles, kMWaves);
    if (grid > need) grid = need;
    hipStream_t s = static_cast<hipStream_t>(stream);
    RGA_LAUNCH("shade_fwd_bf16x3", shade_fwd_mfma_kernel, dim3(grid), dim3(kMThreads), lds, s, a,
               ratio, color, front);
    RGA_CHECK_LAUNCH("shade_gaussians");
    return RGA_OK;
  }
  const size_t lds = fp32_lds(a.K, a.V, false);
  if (lds > 152 * 1024)
    return rga::fail(RGA_EUNSUPPORTED, "shade_gaussians: %d directions and %d views need %zu B of LDS",
                     a.K, a.V, lds);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nq = (int)rga::ceil_div(3 * a.V, 1024);
  const void* kern = fp32_kernel(false, nq);
  const dim3 grid(grid_for(kern, n, lds));
  {
    rga::TimedLaunch tl("shade_fwd", s);
    void* args[] = {&a, &color, &front};
    if (hipLaunchKernel(kern, grid, dim3(kThreads), args, lds, s) != hipSuccess)
      return rga::fail(RGA_EHIP, "shade_gaussians: launch failed");
  }
  RGA_CHECK_LAUNCH("shade_gaussians");
  return RGA_OK;
}

extern "C" size_t shade_gaussians_workspace(int n, int he, int we) {
  if (n < 0 || he < 1 || we < 1) return 0;
  const size_t K = (size_t)he * we;
  // at most 4 workgroups per CU on up to 512 CUs
  return 4 * 512 * 3 * K * sizeof(float);
}

extern "C" int shade_gaussians_backward(void* stream, int n, const float* x, const float* nrm,
                                        const float* albedo, const float* rough, const float* tint,
                                        const int32_t* vidx, const float* vw, const uint8_t* count,
                                        int nv, int kv, int he, int we, int hv, int wv,
                                        const float* env, const float* cam_pos, int precision,
                                        const float* color, const uint8_t* front,
                                        const float* dcolor, float* dx, float* dn,
                                        float* dalbedo, float* drough, float* dtint, float* denv,
                                        void* ws, size_t ws_bytes, const void* tape,
                                        size_t tape_bytes) {
  (void)front;
  int rc = check_args("shade_gaussians_backward", n, x, nrm, albedo, rough, tint, vidx, vw, count,
                      nv, kv, he, we, hv, wv, env, cam_pos, precision);
  if (rc) return rc;
  if (!denv) return rga::fail(RGA_EINVAL, "shade_gaussians_backward: null denv");
  if (n > 0 && (!color || !dcolor || !dx || !dn || !dalbedo || !drough || !dtint))
    return rga::fail(RGA_EINVAL, "shade_gaussians_backward: null pointer");
  ShadeArgs a = make_args(n, x, nrm, albedo, rough, tint, vidx, vw, count, nv, kv, he, we, hv, wv,
                          env, cam_pos);
  rc = attach_tape("shade_gaussians_backward", a, tape, tape_bytes);
  if (rc) return rc;
  // given a tape (of either form's forward), the adjoint replays its live
  // pairs in FP32; the MFMA adjoint is the BF16X3 form's without one
  if (precision == RGA_BF16X3 && !a.tape) {
    if (a.K % 32 != 0)
      return rga::fail(RGA_EUNSUPPORTED, "shade_gaussians_backward: BF16X3 needs a multiple of 32 directions");
    const int ratio = (hv == he && we == wv) ? 1 : ((hv == he && we == 2 * wv && we % 8 == 0) ? 2 : 0);
    a.patch = (he % 4 == 0 && we % 8 == 0) ? 1 : 0;
    const size_t lds = (size_t)11 * a.K * sizeof(float) + (size_t)6 * a.K * 2 +
                       (size_t)kMWaves * (4096 + 384 + 2048);
    if (lds > 150 * 1024)
      return rga::fail(RGA_EUNSUPPORTED, "shade_gaussians_backward: too many directions");
    static bool mattr = false;
    if (!mattr) {
      hipFuncSetAttribute(reinterpret_cast<const void*>(shade_bwd_mfma_kernel),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
      mattr = true;
    }
    int ncu = 0, dev = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
      ncu = 256;
    const int per_cu = lds <= 40 * 1024 ? 4 : (lds <= 76 * 1024 ? 2 : 1);
    int grid = ncu * per_cu;
    const int need = (int)rga::ceil_div(rga::ceil_div(n, 16), kMWaves);
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    if (!ws || ws_bytes < (size_t)grid * 3 * a.K * sizeof(float))
      return rga::fail(RGA_ECAPACITY, "shade_gaussians_backward: workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* part = static_cast<float*>(ws);
    if (n > 0)
      RGA_LAUNCH("shade_bwd_bf16x3", shade_bwd_mfma_kernel, dim3(grid), dim3(kMThreads), lds, s, a,
                 ratio, color, dcolor, dx, dn, dalbedo, drough, dtint, part);
    RGA_LAUNCH("shade_denv", denv_reduce_kernel, dim3(rga::ceil_div(3 * a.K, 64)), dim3(1024), 0, s,
               a.K, he, we, n > 0 ? grid : 0, part, denv);
    RGA_CHECK_LAUNCH("shade_gaussians_backward");
    return RGA_OK;
  }
  const bool taped = a.tape != nullptr;
  // with a tape: the direction table and the environment sums only
  const size_t lds = taped ? (size_t)11 * a.K * sizeof(float) : fp32_lds(a.K, a.V, true);
  if (lds > 152 * 1024)
    return rga::fail(RGA_EUNSUPPORTED,
                     "shade_gaussians_backward: %d directions and %d views need %zu B of LDS", a.K,
                     a.V, lds);
  const int nq = (int)rga::ceil_div(3 * a.V, 1024);
  const void* kern = fp32_kernel(true, nq, taped);
  const int grid = grid_for(kern, n, lds);
  if (!ws || ws_bytes < (size_t)grid * 3 * a.K * sizeof(float))
    return rga::fail(RGA_ECAPACITY, "shade_gaussians_backward: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* part = static_cast<float*>(ws);
  if (n > 0) {
    rga::TimedLaunch tl("shade_bwd", s);
    void* args[] = {&a, &color, &dcolor, &dx, &dn, &dalbedo, &drough, &dtint, &part};
    if (hipLaunchKernel(kern, dim3(grid), dim3(kThreads), args, lds, s) != hipSuccess)
      return rga::fail(RGA_EHIP, "shade_gaussians_backward: launch failed");
  }
  RGA_LAUNCH("shade_denv", denv_reduce_kernel, dim3(rga::ceil_div(3 * a.K, 64)), dim3(1024), 0, s,
             a.K, he, we, n > 0 ? grid : 0, part, denv);
  RGA_CHECK_LAUNCH("shade_gaussians_backward");
  return RGA_OK;
}
