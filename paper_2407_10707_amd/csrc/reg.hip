// Regularisers of the training loss (Sec. 3.3): material smoothness over
// the K_v nearest vertices, mesh distance of each Gaussian to its K_g
// nearest vertices, displacement length, and the Gaussian scale hinge, with
// the gradients of their weighted sum.
//
//   vertex    one thread per vertex i: sum over k in S_v(i) and the five
//             materials of |m_i - m_k| (sign(m_i - m_k) added to i's gradient
//             in registers and subtracted from k's with a float atomic),
//             |dx_i| and dx_i / |dx_i|
//   gaussian  one thread per Gaussian: sum over its K_g vertices of
//             |x_g - x_k| and the unit vectors, the scale hinge
//             max(0, exp(l) - s_0) and exp(l) where it is active
//   final     fixed-order sum of the per-workgroup sums
// A zero difference or length contributes a zero gradient; neighbour
// indices are clamped to 0..nv-1.
#include "common.h"

namespace {

constexpr int kBlock = 256;

__device__ inline float block_sum(float v, float* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kBlock)
reg_zero_kernel(float* __restrict__ p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.f;
}

__global__ void __launch_bounds__(kBlock)
reg_vertex_kernel(int nv, int kv, const float* __restrict__ mat, const int32_t* __restrict__ knn,
                  const float* __restrict__ disp, float ls, float ld, float* __restrict__ dmat,
                  float* __restrict__ ddisp, float* __restrict__ part, int accumulate) {
  __shared__ float red[kBlock];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float sm = 0.f, dl = 0.f;
  if (i < nv) {
    float mi[5], gi[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 5; ++a) mi[a] = mat[(size_t)a * nv + i];
    for (int t = 0; t < kv; ++t) {
      const int k = rga::clampi(knn[(size_t)i * kv + t], 0, nv - 1);
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        const float d = mi[a] - mat[(size_t)a * nv + k];
        sm += fabsf(d);
        const float sg = d > 0.f ? ls : (d < 0.f ? -ls : 0.f);
        gi[a] += sg;
        if (sg != 0.f) atomicAdd(&dmat[(size_t)a * nv + k], -sg);
      }
    }
#pragma unroll
    for (int a = 0; a < 5; ++a) atomicAdd(&dmat[(size_t)a * nv + i], gi[a]);
    const float x = disp[i], y = disp[nv + i], z = disp[2 * nv + i];
    const float len = sqrtf(fmaf(z, z, fmaf(y, y, x * x)));
    dl = len;
    const float s = len > 0.f ? ld / len : 0.f;
    ddisp[i] = accumulate ? ddisp[i] + s * x : s * x;
    ddisp[nv + i] = accumulate ? ddisp[nv + i] + s * y : s * y;
    ddisp[2 * nv + i] = accumulate ? ddisp[2 * nv + i] + s * z : s * z;
  }
  const float a = block_sum(sm, red);
  const float b = block_sum(dl, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = b;
  }
}

__global__ void __launch_bounds__(kBlock)
reg_gauss_kernel(int n, int nv, int kg, const float* __restrict__ xg,
                 const float* __restrict__ verts, const int32_t* __restrict__ vidx,
                 const float* __restrict__ log_s, float s0, float lm, float lsc,
                 float* __restrict__ dxg, float* __restrict__ dlogs, float* __restrict__ part,
                 int accumulate) {
  __shared__ float red[kBlock];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float md = 0.f, sc = 0.f;
  if (i < n) {
    const float px = xg[i], py = xg[n + i], pz = xg[2 * n + i];
    float gx = 0.f, gy = 0.f, gz = 0.f;
    for (int t = 0; t < kg; ++t) {
      const int k = rga::clampi(vidx[(size_t)t * n + i], 0, nv - 1);
      const float dx = px - verts[k], dy = py - verts[nv + k], dz = pz - verts[2 * nv + k];
      const float len = sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
      md += len;
      if (len > 0.f) {
        const float s = lm / len;
        gx = fmaf(s, dx, gx);
        gy = fmaf(s, dy, gy);
        gz = fmaf(s, dz, gz);
      }
    }
    dxg[i] = accumulate ? dxg[i] + gx : gx;
    dxg[n + i] = accumulate ? dxg[n + i] + gy : gy;
    dxg[2 * n + i] = accumulate ? dxg[2 * n + i] + gz : gz;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float e = expf(log_s[(size_t)c * n + i]);
      const bool on = e > s0;
      sc += on ? e - s0 : 0.f;
      const float gl = on ? lsc * e : 0.f;
      float* o = dlogs + (size_t)c * n + i;
      *o = accumulate ? *o + gl : gl;
    }
  }
  const float a = block_sum(md, red);
  const float b = block_sum(sc, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = b;
  }
}

// terms: smooth, mdist, disp, scale, weighted total
__global__ void __launch_bounds__(kBlock)
reg_final_kernel(int nbv, int nbg, const float* __restrict__ pv, const float* __restrict__ pg,
                 float ls, float lm, float ld, float lsc, float* __restrict__ terms,
                 float* __restrict__ loss_accum) {
  __shared__ float red[kBlock];
  float v[4] = {0.f, 0.f, 0.f, 0.f};
  for (int b = threadIdx.x; b < nbv; b += blockDim.x) {
    v[0] += pv[b];
    v[2] += pv[nbv + b];
  }
  for (int b = threadIdx.x; b < nbg; b += blockDim.x) {
    v[1] += pg[b];
    v[3] += pg[nbg + b];
  }
  float t[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) t[q] = block_sum(v[q], red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) terms[q] = t[q];
    const float tot = ls * t[0] + lm * t[1] + ld * t[2] + lsc * t[3];
    terms[4] = tot;
    if (loss_accum) *loss_accum += tot;
  }
}

int blocks(int count) { return (int)rga::ceil_div(count > 0 ? count : 1, kBlock); }

}  // namespace

extern "C" size_t regularisers_workspace(int nv, int n) {
  if (nv < 0 || n < 0) return 0;
  return (size_t)2 * (blocks(nv) + blocks(n)) * 4;
}

extern "C" int regularisers(void* stream, int nv, int n, int kv, int kg, const float* mat,
                            const int32_t* knn_v, const float* xg, const float* verts,
                            const int32_t* vidx, const float* disp, const float* log_s, float s0,
                            float lam_smooth, float lam_mdist, float lam_disp, float lam_scale,
                            float* terms, float* dmat, float* dxg, float* ddisp, float* dlogs,
                            int accumulate, float* loss_accum, void* ws, size_t ws_bytes) {
  if (nv < 1 || n < 0 || kv < 1 || kg < 1 || kv > nv || kg > nv)
    return rga::fail(RGA_EINVAL, "regularisers: nv >= 1, n >= 0, 1 <= kv, kg <= nv");
  if (!mat || !knn_v || !verts || !disp || !terms || !dmat || !ddisp || !ws ||
      (n > 0 && (!xg || !vidx || !log_s || !dxg || !dlogs)))
    return rga::fail(RGA_EINVAL, "regularisers: null pointer");
  if (ws_bytes < regularisers_workspace(nv, n))
    return rga::fail(RGA_ECAPACITY, "regularisers: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nbv = blocks(nv), nbg = blocks(n);
  float* pv = static_cast<float*>(ws);
  float* pg = pv + 2 * nbv;
  if (!accumulate)
    RGA_LAUNCH("reg_zero", reg_zero_kernel, dim3(blocks(5 * nv)), dim3(kBlock), 0, s, dmat, 5 * nv);
  RGA_LAUNCH("reg_vertex", reg_vertex_kernel, dim3(nbv), dim3(kBlock), 0, s, nv, kv, mat, knn_v,
             disp, lam_smooth, lam_disp, dmat, ddisp, pv, accumulate);
  RGA_LAUNCH("reg_gauss", reg_gauss_kernel, dim3(nbg), dim3(kBlock), 0, s, n, nv, kg, xg, verts,
             vidx, log_s, s0, lam_mdist, lam_scale, dxg, dlogs, pg, accumulate);
  RGA_LAUNCH("reg_final", reg_final_kernel, dim3(1), dim3(kBlock), 0, s, nbv, nbg, pv, pg,
             lam_smooth, lam_mdist, lam_disp, lam_scale, terms, loss_accum);
  RGA_CHECK_LAUNCH("regularisers");
  return RGA_OK;
}
