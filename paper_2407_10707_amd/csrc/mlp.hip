// The pose-dependent vertex displacement dx = d(x, theta) (Sec. 3.1,
// attribute paragraph; Sec. 3.5, implementation details): four hidden layers
// of width 256 with ReLU and a linear output of 3, the coordinates encoded by
// random Fourier features gamma(x) = [sin(2 pi B x), cos(2 pi B x)] (B is
// 64 x 3) and the pose theta (72) appended to every vertex's input.
//
// Every layer is a dense product over the vertices, so it runs on MFMA
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation) in a split form that keeps
// FP32 accuracy: each operand is a bf16 high part plus a bf16 low part and
// a product is taken as hi.hi + lo.hi + hi.lo (the lo.lo term is below FP32
// rounding).
//
//   pack      weights -> bf16 hi/lo operands in the exact per-lane order of
//             the MFMA B operand (one 16-byte load per lane and step), once
//             in forward order and once transposed for the adjoint; the pose
//             is folded into the first layer's bias (b_1 + W_1[:, 128:] theta)
//   forward   one workgroup per 32 vertices, all layers in one kernel: the
//             activations stay in LDS (two buffers), each wave computes 64
//             of a layer's columns with the weights streaming from L2; the
//             hidden activations are kept for the adjoint
//   backward  the same shape: dz_5 = ddx, dh = dz W (transposed pack),
//             dz = dh where h > 0; every dz is kept
//   wgrad     dW_l = sum over vertices of dz_l h_{l-1}^T: a workgroup per
//             (layer, chunk of vertices) for the four large layers (the
//             inputs staged through LDS once per workgroup), a small tiled
//             kernel for the output layer; partial sums per chunk (no
//             atomics), then a fixed-order sum over the chunks; the Fourier
//             features of the first layer are recomputed from x; dW_1's pose
//             columns are db_1 theta^T and dtheta = W_1[:, 128:]^T db_1
#include "common.h"

#include <algorithm>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kFreqs = RGA_MLP_FREQS;     // 64
constexpr int kPose = RGA_MLP_POSE;       // 72
constexpr int kWidth = RGA_MLP_WIDTH;     // 256
constexpr int kIn1 = 2 * kFreqs + kPose;  // 200
constexpr int kLayers = 5;
constexpr int kParams = RGA_MLP_PARAMS;
constexpr int kAS = kWidth + 4;           // LDS row stride of the activations (floats)
constexpr int kMaxChunks = 51;   // five layer workgroups per chunk: 255 fit the 256 CUs at once
constexpr int kWaves = 4;

// parameter layout: W_1 [256][200], b_1, W_2 [256][256], b_2, W_3, b_3, W_4, b_4, W_5 [3][256], b_5
__host__ __device__ constexpr int n_out(int l) { return l < 4 ? kWidth : 3; }
__host__ __device__ constexpr int n_in(int l) { return l == 0 ? kIn1 : kWidth; }
__host__ __device__ constexpr int w_off(int l) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += n_out(i) * n_in(i) + n_out(i);
  return o;
}
__host__ __device__ constexpr int b_off(int l) { return w_off(l) + n_out(l) * n_in(l); }
static_assert(w_off(kLayers) == kParams, "parameter count");

// forward operand of layer l: reduction over its MFMA inputs (the 128
// Fourier features for l = 0), columns = outputs padded to 16
__host__ __device__ constexpr int f_k(int l) { return l == 0 ? 2 * kFreqs : kWidth; }
__host__ __device__ constexpr int f_n(int l) { return l < 4 ? kWidth : 16; }
__host__ __device__ constexpr int f_off(int l) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += f_k(i) * f_n(i);
  return o;
}
constexpr int kFwdElems = f_off(kLayers);
// transposed operand of layer l = 1..4: reduction over its outputs (padded
// to 32), columns = its 256 inputs
__host__ __device__ constexpr int t_k(int l) { return l < 4 ? kWidth : 32; }
__host__ __device__ constexpr int t_off(int l) {
  int o = kFwdElems;
  for (int i = 1; i < l; ++i) o += t_k(i) * kWidth;
  return o;
}
constexpr int kPackElems = t_off(kLayers);   // per hi and lo

struct MlpLayout {
  int nvp, chunks, chunk_len;
  size_t pack, bias, h, dz, part, total;
};

MlpLayout mlp_layout(int nv) {
  MlpLayout L{};
  L.nvp = (int)rga::align_up((size_t)(nv > 0 ? nv : 1), 32);
  L.chunks = std::max(1, std::min(kMaxChunks, L.nvp / 256));
  L.chunk_len = (int)rga::align_up((size_t)rga::ceil_div(L.nvp, L.chunks), 32);
  const size_t V = (size_t)L.nvp;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t a = o;
    o = rga::align_up(o + bytes, 256);
    return a;
  };
  L.pack = take((size_t)2 * kPackElems * 2);
  L.bias = take((size_t)kLayers * kWidth * 4);
  L.h = take((size_t)4 * kWidth * V * 4);
  L.dz = take(((size_t)4 * kWidth + 16) * V * 4);
  L.part = take((size_t)L.chunks * kParams * 4);
  L.total = o;
  return L;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 8 floats -> bf16 high parts and bf16 low parts (the remainders)
__device__ inline void split8(const float* v, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)v[e];
    hi[e] = h;
    lo[e] = (__bf16)(v[e] - (float)h);
  }
}

__device__ inline f32x4 mfma3(const bf16x8& ah, const bf16x8& al, const bf16x8& bh,
                              const bf16x8& bl, f32x4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
  return acc;
}

__device__ inline void load8(const float* p, float* v) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

// Fragment order of an operand with KS reduction steps of 32: element
// ((ct * KS + ks) * 64 + lane) * 8 + e holds column ct * 16 + lane % 16 and
// reduction index ks * 32 + 8 (lane / 16) + e.
__global__ void __launch_bounds__(256)
mlp_pack_kernel(const float* __restrict__ P, const float* __restrict__ theta,
                __bf16* __restrict__ hi, __bf16* __restrict__ lo, float* __restrict__ bias) {
  const int groups = kPackElems / 8;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < groups + kLayers * kWidth;
       i += gridDim.x * blockDim.x) {
    if (i < groups) {
      const int e0 = 8 * i;
      float v[8];
      if (e0 < kFwdElems) {
        int l = 0;
        while (l + 1 < kLayers && e0 >= f_off(l + 1)) ++l;
        const int KS = f_k(l) / 32, frag = (e0 - f_off(l)) / 8;
        const int lane = frag & 63, t = frag >> 6, ks = t % KS, ct = t / KS;
        const int n = ct * 16 + (lane & 15), kb = ks * 32 + 8 * (lane >> 4);
        for (int e = 0; e < 8; ++e)
          v[e] = n < n_out(l) ? P[w_off(l) + n * n_in(l) + kb + e] : 0.f;
      } else {
        int l = 1;
        while (l + 1 < kLayers && e0 >= t_off(l + 1)) ++l;
        const int KS = t_k(l) / 32, frag = (e0 - t_off(l)) / 8;
        const int lane = frag & 63, t = frag >> 6, ks = t % KS, ct = t / KS;
        const int k = ct * 16 + (lane & 15), nb = ks * 32 + 8 * (lane >> 4);
        for (int e = 0; e < 8; ++e)
          v[e] = nb + e < n_out(l) ? P[w_off(l) + (nb + e) * n_in(l) + k] : 0.f;
      }
      bf16x8 h, l8;
      split8(v, h, l8);
      *reinterpret_cast<bf16x8*>(hi + e0) = h;
      *reinterpret_cast<bf16x8*>(lo + e0) = l8;
    } else {
      const int j = i - groups, l = j / kWidth, n = j % kWidth;
      float b = 0.f;
      if (l == 0) {
        b = P[b_off(0) + n];
        for (int t = 0; t < kPose; ++t) b = fmaf(P[w_off(0) + n * kIn1 + 2 * kFreqs + t], theta[t], b);
      } else if (n < n_out(l)) {
        b = P[b_off(l) + n];
      }
      bias[j] = b;
    }
  }
}

// gamma(x): sin and cos of 2 pi (B_j . x), with the 2 folded into the
// argument of sinpi / cospi
__device__ inline float fourier_arg(const float* __restrict__ freqs, int j, float x0, float x1,
                                    float x2) {
  const float a = fmaf(freqs[3 * j + 2], x2, fmaf(freqs[3 * j + 1], x1, freqs[3 * j] * x0));
  return 2.f * a;
}

// One layer's product for a workgroup's 32 rows: wave w takes the NQ
// column tiles from `ct0`; A comes from the LDS activations (two row tiles),
// the operand fragments from global memory, those of the next reduction
// step loaded before the products of the current one.
template <int NQ>
__device__ inline void layer_mm(const float (*Ain)[kAS], const bf16x8* __restrict__ bh,
                                const bf16x8* __restrict__ bl, int fo, int KS, int ct0,
                                f32x4 (&acc)[2][NQ]) {
  const int lane = threadIdx.x & 63, row = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[rt][q] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 ch[NQ], cl[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int fi = fo + ((ct0 + q) * KS) * 64 + lane;
    ch[q] = bh[fi];
    cl[q] = bl[fi];
  }
  for (int ks = 0; ks < KS; ++ks) {
    bf16x8 nh[NQ], nl[NQ];
    if (ks + 1 < KS) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int fi = fo + ((ct0 + q) * KS + ks + 1) * 64 + lane;
        nh[q] = bh[fi];
        nl[q] = bl[fi];
      }
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      float av[8];
      load8(&Ain[rt * 16 + row][ks * 32 + 8 * g], av);
      bf16x8 ah, al;
      split8(av, ah, al);
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[rt][q] = mfma3(ah, al, ch[q], cl[q], acc[rt][q]);
    }
    if (ks + 1 < KS) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        ch[q] = nh[q];
        cl[q] = nl[q];
      }
    }
  }
}

constexpr int kRows = 32;                // vertices per workgroup

__global__ void __launch_bounds__(256)
mlp_forward_kernel(int nv, int nvp, const float* __restrict__ x, const float* __restrict__ freqs,
                   const __bf16* __restrict__ phi, const __bf16* __restrict__ plo,
                   const float* __restrict__ bias, float* __restrict__ H, float* __restrict__ out) {
  __shared__ __align__(16) float act[2][kRows][kAS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, g = lane >> 4;
  const int r0 = blockIdx.x * kRows;     // < nvp by the grid
  // Fourier features: lane = frequency, rows wave, wave + 4, ...
  for (int r = wave; r < kRows; r += kWaves) {
    const int v = r0 + r;
    const bool in = v < nv;
    const float x0 = in ? x[v] : 0.f, x1 = in ? x[nv + v] : 0.f, x2 = in ? x[2 * nv + v] : 0.f;
    const float f = fourier_arg(freqs, lane, x0, x1, x2);
    act[0][r][lane] = sinpif(f);
    act[0][r][kFreqs + lane] = cospif(f);
  }
  __syncthreads();
  const bf16x8* bh = reinterpret_cast<const bf16x8*>(phi);
  const bf16x8* bl = reinterpret_cast<const bf16x8*>(plo);
  int cur = 0;
  for (int l = 0; l < kLayers - 1; ++l) {
    f32x4 acc[2][4];
    layer_mm<4>(act[cur], bh, bl, f_off(l) / 8, f_k(l) / 32, 4 * wave, acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = (4 * wave + q) * 16 + row;
      const float bn = bias[l * kWidth + n];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        float hv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = rt * 16 + 4 * g + i;
          const float h = fmaxf(acc[rt][q][i] + bn, 0.f);
          act[cur ^ 1][r][n] = h;
          hv[i] = r0 + r < nv ? h : 0.f;
        }
        *reinterpret_cast<float4*>(H + ((size_t)l * kWidth + n) * nvp + r0 + rt * 16 + 4 * g) =
            make_float4(hv[0], hv[1], hv[2], hv[3]);
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  if (wave == 0) {                       // the output layer: one 16-column tile
    f32x4 acc[2][1];
    layer_mm<1>(act[cur], bh, bl, f_off(kLayers - 1) / 8, f_k(kLayers - 1) / 32, 0, acc);
    if (row < 3)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int v = r0 + rt * 16 + 4 * g + i;
          if (v < nv) out[(size_t)row * nv + v] = acc[rt][0][i] + bias[(kLayers - 1) * kWidth + row];
        }
  }
}

__global__ void __launch_bounds__(256)
mlp_backward_kernel(int nv, int nvp, const float* __restrict__ ddx, const __bf16* __restrict__ phi,
                    const __bf16* __restrict__ plo, const float* __restrict__ H,
                    float* __restrict__ dZ) {
  __shared__ __align__(16) float act[2][kRows][kAS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, g = lane >> 4;
  const int r0 = blockIdx.x * kRows;
  float* dZ5 = dZ + (size_t)4 * kWidth * nvp;
  // dz_5 = ddx, as 32 reduction columns (3 used)
  for (int t = threadIdx.x; t < kRows * 32; t += blockDim.x) {
    const int r = t >> 5, c = t & 31, v = r0 + r;
    const float d = (c < 3 && v < nv) ? ddx[(size_t)c * nv + v] : 0.f;
    act[0][r][c] = d;
    if (c < 16) dZ5[(size_t)c * nvp + v] = d;
  }
  __syncthreads();
  const bf16x8* bh = reinterpret_cast<const bf16x8*>(phi);
  const bf16x8* bl = reinterpret_cast<const bf16x8*>(plo);
  int cur = 0;
  for (int l = kLayers - 1; l >= 1; --l) {
    f32x4 acc[2][4];
    layer_mm<4>(act[cur], bh, bl, t_off(l) / 8, t_k(l) / 32, 4 * wave, acc);
    // dz of hidden layer l - 1 (the input of layer l): dh where h > 0
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = (4 * wave + q) * 16 + row;
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const size_t o = ((size_t)(l - 1) * kWidth + n) * nvp + r0 + rt * 16 + 4 * g;
        const float4 h = *reinterpret_cast<const float4*>(H + o);
        const float hv[4] = {h.x, h.y, h.z, h.w};
        float dv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          dv[i] = hv[i] > 0.f ? acc[rt][q][i] : 0.f;
          act[cur ^ 1][rt * 16 + 4 * g + i][n] = dv[i];
        }
        *reinterpret_cast<float4*>(dZ + o) = make_float4(dv[0], dv[1], dv[2], dv[3]);
      }
    }
    __syncthreads();
    cur ^= 1;
  }
}

// dW_l of one layer over one chunk of vertices, the whole layer per
// workgroup so that every operand row is read once per chunk (a workgroup
// per 64 x 128 tile re-reads dz twice and h four times); blockIdx.x = the
// layer, so all five run side by side: the first layer's Fourier columns
// (256 x 128, features recomputed from x once per chunk step instead of
// once per tile), the hidden layers (256 x 256, h_{l-1} from the forward)
// and the output layer (3 x 256, its dz padded to 16 rows).  Eight waves,
// each RT row tiles x NCT column tiles of 16 x 16.  Both operands of a
// 32-vertex step are split into bf16 hi / lo fragments in LDS (A = dz
// rows, B = the layer's inputs), double-buffered: each thread loads its
// share of the next step into registers before this step's MFMAs and
// splits and stores it after them, so the loads' latency is spent under
// the products.  The db sums come from the same loads.
constexpr int kLayerThreads = 512;
constexpr int kLayerWaves = kLayerThreads / 64;
constexpr int kFragA = 16 * 64;   // A fragments per step buffer (256 rows)
constexpr int kFragB = 16 * 64;   // B fragments per step buffer (256 columns)

struct WgradLds {
  bf16x8 a[2][2][kFragA];   // [buffer][hi, lo][row tile * 64 + lane]
  bf16x8 b[2][2][kFragB];   // [buffer][hi, lo][column tile * 64 + lane]
};

template <bool FIRST, int NRT, int RT, int NCT>
__device__ inline void wgrad_layer(int l, int nv, int nvp, int chunk_len, const float* x,
                                   const float* freqs, const float* H, const float* dZ,
                                   float* part, WgradLds& S) {
  constexpr int NQ = FIRST ? 2 * kFreqs / 16 : kWidth / 16;   // the layer's input column tiles
  constexpr int NRG = kLayerWaves * NCT / NQ;                  // row groups of waves
  static_assert(NRG * RT == NRT, "the waves cover the layer's rows");
  constexpr int FA = NRT * 64, FB = NQ * 64;                   // fragments per step
  constexpr int PA = (FA + kLayerThreads - 1) / kLayerThreads;  // per thread
  constexpr int PB = FIRST ? 0 : FB / kLayerThreads;            // loaded per thread (B)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, g = lane >> 4;
  const int c = blockIdx.y;
  const int n0 = 16 * RT * (wave % NRG), q0 = NCT * (wave / NRG);
  const int nrows = l < 4 ? kWidth : 16;
  const float* dz = dZ + (size_t)l * kWidth * nvp;
  const float* hin = H + (size_t)(FIRST ? 0 : l - 1) * kWidth * nvp;
  const int v0 = c * chunk_len, v1 = min(nvp, v0 + chunk_len);
  // fragment f = 64 t + L of either operand: row (or column) 16 t + L % 16,
  // vertices vb + 8 (L / 16) .. + 7 (the MFMA operand order)
  float ra[PA][8], rb[PB > 0 ? PB : 1][8];
  float dsum[PA];
#pragma unroll
  for (int p = 0; p < PA; ++p) dsum[p] = 0.f;
  auto load = [&](int vb) {
#pragma unroll
    for (int p = 0; p < PA; ++p) {
      const int f = threadIdx.x + p * kLayerThreads;
      const int n = 16 * (f >> 6) + (f & 15), va = vb + 8 * ((f & 63) >> 4);
      if (f < FA && n < nrows) {
        load8(dz + (size_t)n * nvp + va, ra[p]);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) ra[p][e] = 0.f;
      }
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      const int f = threadIdx.x + p * kLayerThreads;
      const int col = 16 * (f >> 6) + (f & 15), va = vb + 8 * ((f & 63) >> 4);
      load8(hin + (size_t)col * nvp + va, rb[p]);
    }
  };
  auto store = [&](int buf, int vb) {
#pragma unroll
    for (int p = 0; p < PA; ++p) {
      const int f = threadIdx.x + p * kLayerThreads;
      if (f < FA) {
        bf16x8 h, lo;
        split8(ra[p], h, lo);
        S.a[buf][0][f] = h;
        S.a[buf][1][f] = lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) dsum[p] += ra[p][e];
      }
    }
    if constexpr (FIRST) {
      for (int f = threadIdx.x; f < FB; f += kLayerThreads) {
        const int col = 16 * (f >> 6) + (f & 15), va = vb + 8 * ((f & 63) >> 4);
        float b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int v = va + e;
          const bool in = v < nv;
          const float x0 = in ? x[v] : 0.f, x1 = in ? x[nv + v] : 0.f, x2 = in ? x[2 * nv + v] : 0.f;
          const float fa = fourier_arg(freqs, col & (kFreqs - 1), x0, x1, x2);
          b[e] = col < kFreqs ? sinpif(fa) : cospif(fa);
        }
        bf16x8 h, lo;
        split8(b, h, lo);
        S.b[buf][0][f] = h;
        S.b[buf][1][f] = lo;
      }
    } else {
#pragma unroll
      for (int p = 0; p < PB; ++p) {
        const int f = threadIdx.x + p * kLayerThreads;
        bf16x8 h, lo;
        split8(rb[p], h, lo);
        S.b[buf][0][f] = h;
        S.b[buf][1][f] = lo;
      }
    }
  };
  f32x4 acc[RT][NCT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int j = 0; j < NCT; ++j) acc[rt][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  int buf = 0;
  if (v0 < v1) {
    load(v0);
    store(0, v0);
  }
  __syncthreads();
  for (int vb = v0; vb < v1; vb += 32) {
    const bool more = vb + 32 < v1;
    if (more) load(vb + 32);
    bf16x8 ah[RT], al[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int f = (n0 / 16 + rt) * 64 + lane;
      ah[rt] = S.a[buf][0][f];
      al[rt] = S.a[buf][1][f];
    }
#pragma unroll
    for (int j = 0; j < NCT; ++j) {
      const bf16x8 bh = S.b[buf][0][(q0 + j) * 64 + lane];
      const bf16x8 bl = S.b[buf][1][(q0 + j) * 64 + lane];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt][j] = mfma3(ah[rt], al[rt], bh, bl, acc[rt][j]);
    }
    // the other buffer's readers all passed the barrier that ended the
    // previous step
    if (more) store(buf ^ 1, vb + 32);
    __syncthreads();
    buf ^= 1;
  }
  float* pc = part + (size_t)c * kParams;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int j = 0; j < NCT; ++j) {
      const int k = 16 * (q0 + j) + row;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int n = n0 + 16 * rt + 4 * g + i;
        if (n < n_out(l)) pc[w_off(l) + n * n_in(l) + k] = acc[rt][j][i];
      }
    }
  // db: fragment f's thread summed row 16 (f >> 6) + f % 16 over its
  // vertex quarter (f % 64) / 16; the four quarters are lanes L, L ^ 16,
  // L ^ 32, L ^ 48 of one wave
#pragma unroll
  for (int p = 0; p < PA; ++p) {
    float d = dsum[p];
    d += __shfl_xor(d, 16);
    d += __shfl_xor(d, 32);
    const int f = threadIdx.x + p * kLayerThreads;
    const int n = 16 * (f >> 6) + (f & 15);
    if (f < FA && lane < 16 && n < n_out(l)) pc[b_off(l) + n] = d;
  }
}

__global__ void __launch_bounds__(kLayerThreads)
mlp_wgrad_layer_kernel(int nv, int nvp, int chunk_len, const float* __restrict__ x,
                       const float* __restrict__ freqs, const float* __restrict__ H,
                       const float* __restrict__ dZ, float* __restrict__ part) {
  __shared__ WgradLds S;
  const int l = blockIdx.x;
  if (l == 0)
    wgrad_layer<true, 16, 4, 4>(l, nv, nvp, chunk_len, x, freqs, H, dZ, part, S);
  else if (l < 4)
    wgrad_layer<false, 16, 4, 8>(l, nv, nvp, chunk_len, x, freqs, H, dZ, part, S);
  else
    wgrad_layer<false, 1, 1, 2>(l, nv, nvp, chunk_len, x, freqs, H, dZ, part, S);
}

// dparams = sum over the chunks (fixed order); W_1's pose columns are
// db_1 theta^T (the pose is shared by every vertex)
__global__ void __launch_bounds__(256)
mlp_reduce_kernel(int chunks, const float* __restrict__ theta, const float* __restrict__ part,
                  float* __restrict__ dP) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const int k = p % kIn1;
  if (p < b_off(0) && k >= 2 * kFreqs) {
    const int n = p / kIn1;
    float db = 0.f;
    for (int c = 0; c < chunks; ++c) db += part[(size_t)c * kParams + b_off(0) + n];
    dP[p] = db * theta[k - 2 * kFreqs];
  } else {
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(size_t)c * kParams + p];
    dP[p] = s;
  }
}

// dtheta = W_1[:, 128:]^T db_1 (db_1 summed over the chunks first; the
// 256-term products in four fixed quarters, then added in order)
constexpr int kDthThreads = 320;
__global__ void __launch_bounds__(kDthThreads)
mlp_dtheta_kernel(int chunks, const float* __restrict__ P, const float* __restrict__ part,
                  float* __restrict__ dtheta) {
  __shared__ float db[kWidth];
  __shared__ float quarter[4][kPose];
  const int t = threadIdx.x;
  if (t < kWidth) {
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(size_t)c * kParams + b_off(0) + t];
    db[t] = s;
  }
  __syncthreads();
  if (t < 4 * kPose) {
    const int k = t % kPose, q = t / kPose;
    float a = 0.f;
    for (int n = 64 * q; n < 64 * q + 64; ++n)
      a = fmaf(P[w_off(0) + n * kIn1 + 2 * kFreqs + k], db[n], a);
    quarter[q][k] = a;
  }
  __syncthreads();
  if (t < kPose) dtheta[t] = ((quarter[0][t] + quarter[1][t]) + quarter[2][t]) + quarter[3][t];
}

}  // namespace

extern "C" size_t mlp_workspace(int nv) {
  if (nv < 0) return 0;
  return mlp_layout(nv).total;
}

extern "C" int mlp_forward(void* stream, int nv, const float* x, const float* freqs,
                           const float* theta, const float* params, void* ws, size_t ws_bytes,
                           float* dx) {
  if (nv < 0 || nv > (1 << 26)) return rga::fail(RGA_EINVAL, "mlp_forward: nv in 0..2^26");
  if (!freqs || !theta || !params || !ws || (nv > 0 && (!x || !dx)))
    return rga::fail(RGA_EINVAL, "mlp_forward: null pointer");
  const MlpLayout L = mlp_layout(nv);
  if (ws_bytes < L.total) return rga::fail(RGA_ECAPACITY, "mlp_forward: workspace too small");
  if (!rga::aligned16(ws)) return rga::fail(RGA_EINVAL, "mlp_forward: workspace not 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  __bf16* hi = at<__bf16>(ws, L.pack);
  __bf16* lo = hi + kPackElems;
  RGA_LAUNCH("mlp_pack", mlp_pack_kernel, dim3(256), dim3(256), 0, s, params, theta, hi, lo,
             at<float>(ws, L.bias));
  // with no vertices the kernel still clears the kept activations of the
  // padding rows, which the adjoint reads
  RGA_LAUNCH("mlp_fwd", mlp_forward_kernel, dim3(L.nvp / kRows), dim3(64 * kWaves), 0, s, nv, L.nvp, x, freqs, hi, lo, at<float>(ws, L.bias),
               at<float>(ws, L.h), dx);
  RGA_CHECK_LAUNCH("mlp_forward");
  return RGA_OK;
}

extern "C" int mlp_backward(void* stream, int nv, const float* x, const float* freqs,
                            const float* theta, const float* params, const float* ddx, void* ws,
                            size_t ws_bytes, float* dparams, float* dtheta) {
  if (nv < 0 || nv > (1 << 26)) return rga::fail(RGA_EINVAL, "mlp_backward: nv in 0..2^26");
  if (!freqs || !theta || !params || !ws || !dparams || !dtheta || (nv > 0 && (!x || !ddx)))
    return rga::fail(RGA_EINVAL, "mlp_backward: null pointer");
  const MlpLayout L = mlp_layout(nv);
  if (ws_bytes < L.total) return rga::fail(RGA_ECAPACITY, "mlp_backward: workspace too small");
  if (!rga::aligned16(ws)) return rga::fail(RGA_EINVAL, "mlp_backward: workspace not 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const __bf16* hi = at<__bf16>(ws, L.pack);
  const __bf16* lo = hi + kPackElems;
  float* part = at<float>(ws, L.part);
  // with no vertices every partial sum is zero: the backward and the
  // weight-gradient kernels still run over the (zero) padding rows
  RGA_LAUNCH("mlp_bwd", mlp_backward_kernel, dim3(L.nvp / kRows), dim3(64 * kWaves), 0, s, nv, L.nvp, ddx, hi, lo, at<float>(ws, L.h),
             at<float>(ws, L.dz));
  RGA_LAUNCH("mlp_wgrad", mlp_wgrad_layer_kernel, dim3(kLayers, L.chunks), dim3(kLayerThreads), 0,
             s, nv, L.nvp, L.chunk_len, x, freqs, at<float>(ws, L.h), at<float>(ws, L.dz), part);
  RGA_LAUNCH("mlp_reduce", mlp_reduce_kernel, dim3(rga::ceil_div(kParams, 256)), dim3(256), 0, s,
             L.chunks, theta, part, dparams);
  RGA_LAUNCH("mlp_dtheta", mlp_dtheta_kernel, dim3(1), dim3(kDthThreads), 0, s, L.chunks, params,
             part, dtheta);
  RGA_CHECK_LAUNCH("mlp_backward");
  return RGA_OK;
}
