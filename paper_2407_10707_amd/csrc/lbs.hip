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
               const float* __restrict__ disp, const float* __restrict__ nrm,
               float* __restrict__ x_out, float* __restrict__ n_out, float* __restrict__ A_out) {
  __shared__ float S[kMaxJoints * 12];
  for (int k = threadIdx.x; k < J * 12; k += blockDim.x) S[k] = skin[k];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // the optional displacement is added first (x + dx rounded to FP32)
  const float p0 = disp ? x[i] + disp[i] : x[i];
  const float p1 = disp ? x[n + i] + disp[n + i] : x[n + i];
  const float p2 = disp ? x[2 * n + i] + disp[2 * n + i] : x[2 * n + i];
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

// Pose gradient: dS_j[r][c] = sum_i w_ij (dx'_i[r] (x_i, 1)[c] + dn'_i[r] (n_i, 0)[c]
// + dA_i[r][c] for c < 3),
// w_ij the summed weights of joint j in Gaussian i's slots.  Workgroups over
// (chunk of Gaussians, joint); per-workgroup sums, then a fixed-order sum
// over the chunks (no atomics: every joint is shared by many Gaussians).
constexpr int kPoseChunk = 2048;

__global__ void __launch_bounds__(kBlock)
lbs_pose_grad_kernel(int n, const int32_t* __restrict__ jidx, const float* __restrict__ jw,
                     const float* __restrict__ x, const float* __restrict__ disp,
                     const float* __restrict__ nrm, const float* __restrict__ dxo,
                     const float* __restrict__ dno, const float* __restrict__ dA,
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
    const float xv[3] = {disp ? x[i] + disp[i] : x[i], disp ? x[n + i] + disp[n + i] : x[n + i],
                         disp ? x[2 * n + i] + disp[2 * n + i] : x[2 * n + i]};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const float g = w * dxo[(size_t)r * n + i];
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[4 * r + q] = fmaf(g, xv[q], acc[4 * r + q]);
      acc[4 * r + 3] += g;
    }
    if (dA)
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[4 * r + q] = fmaf(w, dA[(size_t)(3 * r + q) * n + i], acc[4 * r + q]);
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

namespace {

// ---- pose -> skinning matrices (forward kinematics of the axis-angle pose)
// R_j = exp([theta_j]x) = I + a K + b K^2 (a = sin t / t, b = (1 - cos t) / t^2,
// series near t = 0), G_j = G_p R_j, P_j = P_p + G_p (J_j - J_p), a root
// (parent outside 0..j-1) has G = R, P = J; skin_j = [G_j | P_j - G_j J_j].
// One workgroup: the Rodrigues matrices in parallel, the chain in joint order
// by one thread, the rows written in parallel.
__device__ inline void rodrigues(const float* th, float* R, float& a, float& b, float& ap,
                                 float& bp) {
  const float t2 = fmaf(th[2], th[2], fmaf(th[1], th[1], th[0] * th[0]));
  const float t = sqrtf(t2);
  if (t2 < 1e-12f) {
    a = 1.f - t2 / 6.f;
    b = 0.5f - t2 / 24.f;
  } else {
    const float h = sinf(0.5f * t);      // 1 - cos t = 2 sin^2(t/2), no cancellation
    a = sinf(t) / t;
    b = 2.f * h * h / t2;
  }
  // (da/dt) / t and (db/dt) / t: Taylor series below t = 0.5 (the closed
  // forms cancel there), the closed forms above
  if (t2 < 0.25f) {
    ap = -1.f / 3.f + t2 * (1.f / 30.f + t2 * (-1.f / 840.f + t2 * (1.f / 45360.f)));
    bp = -1.f / 12.f + t2 * (1.f / 180.f + t2 * (-1.f / 6720.f + t2 * (1.f / 453600.f)));
  } else {
    const float sn = sinf(t), cs = cosf(t);
    ap = (t * cs - sn) / (t2 * t);
    bp = (t * sn - 2.f * (1.f - cs)) / (t2 * t2);
  }
  const float K[9] = {0.f, -th[2], th[1], th[2], 0.f, -th[0], -th[1], th[0], 0.f};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      float k2 = 0.f;
      for (int m = 0; m < 3; ++m) k2 = fmaf(K[3 * r + m], K[3 * m + c], k2);
      R[3 * r + c] = (r == c ? 1.f : 0.f) + a * K[3 * r + c] + b * k2;
    }
}

__device__ inline void mat3_mul(const float* A, const float* B, float* C) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      float v = 0.f;
      for (int m = 0; m < 3; ++m) v = fmaf(A[3 * r + m], B[3 * m + c], v);
      C[3 * r + c] = v;
    }
}

__device__ inline int parent_of(const int32_t* parents, int j) {
  const int p = parents[j];
  return (p >= 0 && p < j) ? p : -1;
}

struct Chain {
  float R[kMaxJoints][9], G[kMaxJoints][9], P[kMaxJoints][3];
};

__device__ void forward_chain(int J, const float* theta, const float* joints,
                              const int32_t* parents, Chain& ch) {
  for (int j = threadIdx.x; j < J; j += blockDim.x) {
    float a, b, ap, bp;
    rodrigues(theta + 3 * j, ch.R[j], a, b, ap, bp);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 0; j < J; ++j) {
      const int p = parent_of(parents, j);
      if (p < 0) {
        for (int q = 0; q < 9; ++q) ch.G[j][q] = ch.R[j][q];
        for (int q = 0; q < 3; ++q) ch.P[j][q] = joints[3 * j + q];
      } else {
        mat3_mul(ch.G[p], ch.R[j], ch.G[j]);
        for (int r = 0; r < 3; ++r) {
          float v = ch.P[p][r];
          for (int m = 0; m < 3; ++m)
            v = fmaf(ch.G[p][3 * r + m], joints[3 * j + m] - joints[3 * p + m], v);
          ch.P[j][r] = v;
        }
      }
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kBlock)
pose_skin_kernel(int J, const float* __restrict__ theta, const float* __restrict__ joints,
                 const int32_t* __restrict__ parents, float* __restrict__ skin) {
  __shared__ Chain ch;
  forward_chain(J, theta, joints, parents, ch);
  for (int j = threadIdx.x; j < J; j += blockDim.x)
    for (int r = 0; r < 3; ++r) {
      float t = ch.P[j][r];
      for (int m = 0; m < 3; ++m) t = fmaf(-ch.G[j][3 * r + m], joints[3 * j + m], t);
      for (int c = 0; c < 3; ++c) skin[12 * j + 4 * r + c] = ch.G[j][3 * r + c];
      skin[12 * j + 4 * r + 3] = t;
    }
}

// Adjoint: dG_j = dS_j[:, :3] - dt_j J_j^T, dP_j = dt_j; in reverse joint
// order dG_p += dG_j R_j^T + dP_j (J_j - J_p)^T, dP_p += dP_j, dR_j = G_p^T dG_j
// (dR_j = dG_j at a root); then dtheta_j from dR_j through Rodrigues.
__global__ void __launch_bounds__(kBlock)
pose_skin_bwd_kernel(int J, const float* __restrict__ theta, const float* __restrict__ joints,
                     const int32_t* __restrict__ parents, const float* __restrict__ dskin,
                     float* __restrict__ dtheta, int accumulate) {
  __shared__ Chain ch;
  __shared__ float dG[kMaxJoints][9], dP[kMaxJoints][3], dR[kMaxJoints][9];
  forward_chain(J, theta, joints, parents, ch);
  for (int j = threadIdx.x; j < J; j += blockDim.x)
    for (int r = 0; r < 3; ++r) {
      const float dt = dskin[12 * j + 4 * r + 3];
      dP[j][r] = dt;
      for (int c = 0; c < 3; ++c) dG[j][3 * r + c] = dskin[12 * j + 4 * r + c] - dt * joints[3 * j + c];
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = J - 1; j >= 0; --j) {
      const int p = parent_of(parents, j);
      if (p < 0) {
        for (int q = 0; q < 9; ++q) dR[j][q] = dG[j][q];
        continue;
      }
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          float vR = 0.f, vG = 0.f;
          for (int m = 0; m < 3; ++m) {
            vR = fmaf(ch.G[p][3 * m + r], dG[j][3 * m + c], vR);       // G_p^T dG_j
            vG = fmaf(dG[j][3 * r + m], ch.R[j][3 * c + m], vG);       // dG_j R_j^T
          }
          dR[j][3 * r + c] = vR;
          dG[p][3 * r + c] += vG + dP[j][r] * (joints[3 * j + c] - joints[3 * p + c]);
        }
      for (int r = 0; r < 3; ++r) dP[p][r] += dP[j][r];
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < J; j += blockDim.x) {
    const float* th = theta + 3 * j;
    float R[9], a, b, ap, bp;
    rodrigues(th, R, a, b, ap, bp);
    const float* D = dR[j];
    const float K[9] = {0.f, -th[2], th[1], th[2], 0.f, -th[0], -th[1], th[0], 0.f};
    float K2[9];
    mat3_mul(K, K, K2);
    float dK = 0.f, dK2 = 0.f;
    for (int q = 0; q < 9; ++q) {
      dK = fmaf(D[q], K[q], dK);
      dK2 = fmaf(D[q], K2[q], dK2);
    }
    for (int k = 0; k < 3; ++k) {
      float E[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (k == 0) { E[5] = -1.f; E[7] = 1.f; }
      if (k == 1) { E[2] = 1.f; E[6] = -1.f; }
      if (k == 2) { E[1] = -1.f; E[3] = 1.f; }
      float EK[9], KE[9];
      mat3_mul(E, K, EK);
      mat3_mul(K, E, KE);
      float dE = 0.f, dS = 0.f;
      for (int q = 0; q < 9; ++q) {
        dE = fmaf(D[q], E[q], dE);
        dS = fmaf(D[q], EK[q] + KE[q], dS);
      }
      const float v = ap * th[k] * dK + a * dE + bp * th[k] * dK2 + b * dS;
      dtheta[3 * j + k] = accumulate ? dtheta[3 * j + k] + v : v;
    }
  }
}

}  // namespace

extern "C" int pose_to_skin(void* stream, int n_joints, const float* theta, const float* joints,
                            const int32_t* parents, float* skin) {
  if (n_joints < 1 || n_joints > kMaxJoints)
    return rga::fail(RGA_EINVAL, "pose_to_skin: n_joints must be in 1..%d", kMaxJoints);
  if (!theta || !joints || !parents || !skin) return rga::fail(RGA_EINVAL, "pose_to_skin: null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  RGA_LAUNCH("pose_skin", pose_skin_kernel, dim3(1), dim3(kBlock), 0, s, n_joints, theta, joints,
             parents, skin);
  RGA_CHECK_LAUNCH("pose_to_skin");
  return RGA_OK;
}

extern "C" int pose_to_skin_backward(void* stream, int n_joints, const float* theta,
                                     const float* joints, const int32_t* parents,
                                     const float* dskin, float* dtheta, int accumulate) {
  if (n_joints < 1 || n_joints > kMaxJoints)
    return rga::fail(RGA_EINVAL, "pose_to_skin_backward: n_joints must be in 1..%d", kMaxJoints);
  if (!theta || !joints || !parents || !dskin || !dtheta)
    return rga::fail(RGA_EINVAL, "pose_to_skin_backward: null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  RGA_LAUNCH("pose_skin_bwd", pose_skin_bwd_kernel, dim3(1), dim3(kBlock), 0, s, n_joints, theta,
             joints, parents, dskin, dtheta, accumulate);
  RGA_CHECK_LAUNCH("pose_to_skin_backward");
  return RGA_OK;
}

extern "C" size_t lbs_skin_pose_grad_workspace(int n, int n_joints) {
  if (n < 0 || n_joints < 1 || n_joints > kMaxJoints) return 0;
  return (size_t)pose_chunks(n) * n_joints * 12 * 4;
}

extern "C" int lbs_skin_pose_grad(void* stream, int n, int n_joints, const int32_t* jidx,
                                  const float* jw, const float* x, const float* disp,
                                  const float* nrm, const float* dx_out, const float* dn_out,
                                  const float* dA, float* dskin, void* ws, size_t ws_bytes) {
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
             jidx, jw, x, disp, nrm, dx_out, dn_out, dA, part);
  RGA_LAUNCH("lbs_pose_grad_final", lbs_pose_grad_final, dim3(rga::ceil_div(12 * n_joints, kBlock)),
             dim3(kBlock), 0, s, n_joints, chunks, part, dskin);
  RGA_CHECK_LAUNCH("lbs_skin_pose_grad");
  return RGA_OK;
}

extern "C" int lbs_skin(void* stream, int n, int n_joints, const float* skin, const int32_t* jidx,
                        const float* jw, const float* x, const float* disp, const float* nrm,
                        float* x_out, float* n_out, float* A_out) {
  if (n < 0) return rga::fail(RGA_EINVAL, "lbs_skin: n < 0");
  if (n_joints < 1 || n_joints > kMaxJoints)
    return rga::fail(RGA_EINVAL, "lbs_skin: n_joints must be in 1..%d", kMaxJoints);
  if (n == 0) return RGA_OK;
  if (!skin || !jidx || !jw || !x || !x_out) return rga::fail(RGA_EINVAL, "lbs_skin: null pointer");
  if (n_out && !nrm) return rga::fail(RGA_EINVAL, "lbs_skin: n_out requires nrm");
  hipStream_t s = static_cast<hipStream_t>(stream);
  RGA_LAUNCH("lbs_fwd", lbs_fwd_kernel, dim3(rga::ceil_div(n, kBlock)), dim3(kBlock), 0, s, n,
             n_joints, skin, jidx, jw, x, disp, nrm, x_out, n_out, A_out);
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
