// Forward linear blend skinning and its adjoint (Sec. 3.1, deformation).
//
// One thread per point; the joint table ([J][3][4], <= 12 KB) is staged in
// LDS once per workgroup, SoA planes are read and written fully coalesced.
// HBM-bound: 72 B in, 60 B out per point with normal and A.
#include "common.h"

namespace {

constexpr int kMaxJoints = 256;
constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock)
lbs_fwd_kernel(int n, int J, const float* __restrict__ skin, const int32_t* __restrict__ jidx,
               const float* __restrict__ jw, const float* __restrict__ x,
               const float* __restrict__ nrm, float* __restrict__ x_out,
               float* __restrict__ n_out, float* __restrict__ A_out) {
  __shared__ float S[kMaxJoints * 12];
  for (int k = threadIdx.x; k < J * 12; k += blockDim.x) S[k] = skin[k];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float p0 = x[i], p1 = x[n + i], p2 = x[2 * n + i];
  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
  float Aa[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float w = jw[j * n + i];
    const float* Sj = S + 12 * rga::clampi(jidx[j * n + i], 0, J - 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float d0 = Sj[4 * a + 0] - (a == 0 ? 1.f : 0.f);
      const float d1 = Sj[4 * a + 1] - (a == 1 ? 1.f : 0.f);
      const float d2 = Sj[4 * a + 2] - (a == 2 ? 1.f : 0.f);
      const float pa = fmaf(d2, p2, fmaf(d1, p1, fmaf(d0, p0, Sj[4 * a + 3])));
      if (a == 0) acc0 = fmaf(w, pa, acc0);
      if (a == 1) acc1 = fmaf(w, pa, acc1);
      if (a == 2) acc2 = fmaf(w, pa, acc2);
      Aa[3 * a + 0] = fmaf(w, d0, Aa[3 * a + 0]);
      Aa[3 * a + 1] = fmaf(w, d1, Aa[3 * a + 1]);
      Aa[3 * a + 2] = fmaf(w, d2, Aa[3 * a + 2]);
    }
  }
  x_out[i] = p0 + acc0;
  x_out[n + i] = p1 + acc1;
  x_out[2 * n + i] = p2 + acc2;
  float A[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) A[3 * a + b] = (a == b ? 1.f : 0.f) + Aa[3 * a + b];
  if (A_out) {
#pragma unroll
    for (int k = 0; k < 9; ++k) A_out[k * n + i] = A[k];
  }
  if (nrm && n_out) {
    const float m0 = nrm[i], m1 = nrm[n + i], m2 = nrm[2 * n + i];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      n_out[a * n + i] = fmaf(A[3 * a + 2], m2, fmaf(A[3 * a + 1], m1, A[3 * a + 0] * m0));
  }
}

__global__ void __launch_bounds__(kBlock)
lbs_bwd_kernel(int n, int J, const float* __restrict__ skin, const int32_t* __restrict__ jidx,
               const float* __restrict__ jw, const float* __restrict__ dx_out,
               const float* __restrict__ dn_out, float* __restrict__ dx, float* __restrict__ dn) {
  __shared__ float S[kMaxJoints * 12];
  for (int k = threadIdx.x; k < J * 12; k += blockDim.x) S[k] = skin[k];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float A[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float w = jw[j * n + i];
    const float* Sj = S + 12 * rga::clampi(jidx[j * n + i], 0, J - 1);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) A[3 * a + b] = fmaf(w, Sj[4 * a + b] - (a == b ? 1.f : 0.f), A[3 * a + b]);
  }
  const float g0 = dx_out[i], g1 = dx_out[n + i], g2 = dx_out[2 * n + i];
#pragma unroll
  for (int b = 0; b < 3; ++b) dx[b * n + i] = fmaf(A[6 + b], g2, fmaf(A[3 + b], g1, A[b] * g0));
  if (dn_out && dn) {
    const float h0 = dn_out[i], h1 = dn_out[n + i], h2 = dn_out[2 * n + i];
#pragma unroll
    for (int b = 0; b < 3; ++b) dn[b * n + i] = fmaf(A[6 + b], h2, fmaf(A[3 + b], h1, A[b] * h0));
  }
}

}  // namespace

namespace {

// Pose gradient: dS_j[r][c] = sum_i w_ij (dx'_i[r] (x_i, 1)[c] + dn'_i[r] (n_i, 0)[c]),
// w_ij the summed weights of joint j in Gaussian i's slots.  Workgroups over
// (chunk of Gaussians, joint); per-workgroup sums, then a fixed-order sum
// over the chunks (no atomics: every joint is shared by many Gaussians).
constexpr int kPoseChunk = 2048;

__global__ void __launch_bounds__(kBlock)
lbs_pose_grad_kernel(int n, const int32_t* __restrict__ jidx, const float* __restrict__ jw,
                     const float* __restrict__ x, const float* __restrict__ nrm,
                     const float* __restrict__ dxo, const float* __restrict__ dno,
                     float* __restrict__ part) {
  __shared__ float red[12][kBlock];
  const int j = blockIdx.y, c = blockIdx.x;
  const int i0 = c * kPoseChunk, i1 = min(n, i0 + kPoseChunk);
  float acc[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) acc[q] = 0.f;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    float w = 0.f;
#pragma unroll
    for (int sl = 0; sl < 4; ++sl)
      if (jidx[(size_t)sl * n + i] == j) w += jw[(size_t)sl * n + i];
    if (w == 0.f) continue;
    const float xv[3] = {x[i], x[n + i], x[2 * n + i]};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const float g = w * dxo[(size_t)r * n + i];
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[4 * r + q] = fmaf(g, xv[q], acc[4 * r + q]);
      acc[4 * r + 3] += g;
    }
    if (dno) {
      const float nv[3] = {nrm[i], nrm[n + i], nrm[2 * n + i]};
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const float g = w * dno[(size_t)r * n + i];
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[4 * r + q] = fmaf(g, nv[q], acc[4 * r + q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 12; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
#pragma unroll
      for (int q = 0; q < 12; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 12)
    part[((size_t)c * gridDim.y + j) * 12 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(kBlock)
lbs_pose_grad_final(int n_joints, int chunks, const float* __restrict__ part,
                    float* __restrict__ dskin) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 12 * n_joints) return;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += part[(size_t)c * n_joints * 12 + t];
  dskin[t] = s;
}

int pose_chunks(int n) { return (int)rga::ceil_div(n > 0 ? n : 1, kPoseChunk); }

}  // namespace

extern "C" size_t lbs_skin_pose_grad_workspace(int n, int n_joints) {
  if (n < 0 || n_joints < 1 || n_joints > kMaxJoints) return 0;
  return (size_t)pose_chunks(n) * n_joints * 12 * 4;
}

extern "C" int lbs_skin_pose_grad(void* stream, int n, int n_joints, const int32_t* jidx,
                                  const float* jw, const float* x, const float* nrm,
                                  const float* dx_out, const float* dn_out, float* dskin,
                                  void* ws, size_t ws_bytes) {
  if (n < 0) return rga::fail(RGA_EINVAL, "lbs_skin_pose_grad: n < 0");
  if (n_joints < 1 || n_joints > kMaxJoints)
    return rga::fail(RGA_EINVAL, "lbs_skin_pose_grad: n_joints must be in 1..%d", kMaxJoints);
  if (!dskin || !ws || (n > 0 && (!jidx || !jw || !x || !dx_out)))
    return rga::fail(RGA_EINVAL, "lbs_skin_pose_grad: null pointer");
  if ((dn_out == nullptr) != (nrm == nullptr))
    return rga::fail(RGA_EINVAL, "lbs_skin_pose_grad: nrm and dn_out must both be set or both NULL");
  if (ws_bytes < lbs_skin_pose_grad_workspace(n, n_joints))
    return rga::fail(RGA_ECAPACITY, "lbs_skin_pose_grad: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int chunks = pose_chunks(n);
  float* part = static_cast<float*>(ws);
  RGA_LAUNCH("lbs_pose_grad", lbs_pose_grad_kernel, dim3(chunks, n_joints), dim3(kBlock), 0, s, n,
             jidx, jw, x, nrm, dx_out, dn_out, part);
  RGA_LAUNCH("lbs_pose_grad_final", lbs_pose_grad_final, dim3(rga::ceil_div(12 * n_joints, kBlock)),
             dim3(kBlock), 0, s, n_joints, chunks, part, dskin);
  RGA_CHECK_LAUNCH("lbs_skin_pose_grad");
  return RGA_OK;
}

extern "C" int lbs_skin(void* stream, int n, int n_joints, const float* skin, const int32_t* jidx,
                        const float* jw, const float* x, const float* nrm, float* x_out,
                        float* n_out, float* A_out) {
  if (n < 0) return rga::fail(RGA_EINVAL, "lbs_skin: n < 0");
  if (n_joints < 1 || n_joints > kMaxJoints)
    return rga::fail(RGA_EINVAL, "lbs_skin: n_joints must be in 1..%d", kMaxJoints);
  if (n == 0) return RGA_OK;
  if (!skin || !jidx || !jw || !x || !x_out) return rga::fail(RGA_EINVAL, "lbs_skin: null pointer");
  if (n_out && !nrm) return rga::fail(RGA_EINVAL, "lbs_skin: n_out requires nrm");
  hipStream_t s = static_cast<hipStream_t>(stream);
  RGA_LAUNCH("lbs_fwd", lbs_fwd_kernel, dim3(rga::ceil_div(n, kBlock)), dim3(kBlock), 0, s, n,
             n_joints, skin, jidx, jw, x, nrm, x_out, n_out, A_out);
  RGA_CHECK_LAUNCH("lbs_skin");
  return RGA_OK;
}

extern "C" int lbs_skin_backward(void* stream, int n, int n_joints, const float* skin,
                                 const int32_t* jidx, const float* jw, const float* dx_out,
                                 const float* dn_out, float* dx, float* dn) {
  if (n < 0) return rga::fail(RGA_EINVAL, "lbs_skin_backward: n < 0");
  if (n_joints < 1 || n_joints > kMaxJoints)
    return rga::fail(RGA_EINVAL, "lbs_skin_backward: n_joints must be in 1..%d", kMaxJoints);
  if (n == 0) return RGA_OK;
  if (!skin || !jidx || !jw || !dx_out || !dx)
    return rga::fail(RGA_EINVAL, "lbs_skin_backward: null pointer");
  if ((dn_out == nullptr) != (dn == nullptr))
    return rga::fail(RGA_EINVAL, "lbs_skin_backward: dn_out and dn must both be set or both NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  RGA_LAUNCH("lbs_bwd", lbs_bwd_kernel, dim3(rga::ceil_div(n, kBlock)), dim3(kBlock), 0, s, n,
             n_joints, skin, jidx, jw, dx_out, dn_out, dx, dn);
  RGA_CHECK_LAUNCH("lbs_skin_backward");
  return RGA_OK;
}
