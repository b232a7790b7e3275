// Image loss of the training section (Sec. 3.3, image-loss equation):
// L = (1 - lambda) L_1 + lambda (1 - mean SSIM), SSIM with an 11 x 11
// Gaussian window (std 1.5), C1 = 0.01^2, C2 = 0.03^2, every channel filtered
// on its own with zero padding.
//
// With mu = G * x, E_xx = G * x^2, E_xy = G * (x y) (G the separable window)
// and sigma_x^2 = E_xx - mu_x^2, sigma_xy = E_xy - mu_x mu_y, the SSIM of a
// pixel p depends on x through (mu_x, E_xx, E_xy) only, so
//   dS/dx_q = (G * a)_q + 2 x_q (G * b)_q + y_q (G * c)_q
// with a = dS/dmu_x (through the sigmas as well), b = dS/dE_xx and
// c = dS/dE_xy per pixel (G is symmetric, so its adjoint is itself).
//
//   forward   per 32 x 32 tile and channel: x and y with a 5-pixel halo in
//             LDS, the five horizontal sums, the five vertical sums, the
//             SSIM, the (a, b, c) maps for the adjoint, per-tile sums of
//             SSIM and |x - y|
//   adjoint   per tile: (a, b, c) with halo in LDS, the same two passes,
//             then the image gradient with the L1 term
//   final     fixed-order sum of the tile sums -> the loss
#include "common.h"

#include <cmath>

namespace {

constexpr int kT = 32;                 // output tile (pixels per side)
constexpr int kR = 5;                  // window radius
constexpr int kS = kT + 2 * kR;        // tile with halo: 42
constexpr float kC1 = 0.0001f;
constexpr float kC2 = 0.0009f;

struct Window {
  float g[2 * kR + 1];
};

Window window() {
  Window w{};
  double s = 0.0, v[2 * kR + 1];
  for (int i = 0; i <= 2 * kR; ++i) {
    const double t = i - kR;
    v[i] = std::exp(-t * t / (2.0 * 1.5 * 1.5));
    s += v[i];
  }
  for (int i = 0; i <= 2 * kR; ++i) w.g[i] = (float)(v[i] / s);
  return w;
}

// Loads `n` maps of a tile with halo (zero outside the image) into LDS.
template <int N>
__device__ inline void load_halo(const float* const (&src)[N], int H, int W, int y0, int x0,
                                 float (*dst)[kS][kS]) {
  for (int i = threadIdx.x; i < kS * kS; i += blockDim.x) {
    const int r = i / kS, c = i - r * kS;
    const int yy = y0 - kR + r, xx = x0 - kR + c;
    const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
#pragma unroll
    for (int m = 0; m < N; ++m) dst[m][r][c] = in ? src[m][(size_t)yy * W + xx] : 0.f;
  }
}

__global__ void __launch_bounds__(256)
ssim_fwd_kernel(int H, int W, Window win, const float* __restrict__ img,
                const float* __restrict__ tgt, float* __restrict__ abc, float* __restrict__ part) {
  __shared__ float in[2][kS][kS];
  __shared__ float hs[5][kS][kT];
  __shared__ float red[2][256];
  const int ch = blockIdx.z, x0 = blockIdx.x * kT, y0 = blockIdx.y * kT;
  const size_t HW = (size_t)H * W;
  const float* x = img + ch * HW;
  const float* y = tgt + ch * HW;
  {
    const float* const src[2] = {x, y};
    load_halo<2>(src, H, W, y0, x0, in);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kS * kT; i += blockDim.x) {
    const int r = i / kT, c = i - r * kT;
    float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j <= 2 * kR; ++j) {
      const float a = in[0][r][c + j], b = in[1][r][c + j], gj = win.g[j];
      s[0] = fmaf(gj, a, s[0]);
      s[1] = fmaf(gj, b, s[1]);
      s[2] = fmaf(gj, a * a, s[2]);
      s[3] = fmaf(gj, b * b, s[3]);
      s[4] = fmaf(gj, a * b, s[4]);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) hs[q][r][c] = s[q];
  }
  __syncthreads();
  float ssum = 0.f, lsum = 0.f;
  for (int i = threadIdx.x; i < kT * kT; i += blockDim.x) {
    const int r = i / kT, c = i - r * kT;
    const int yy = y0 + r, xx = x0 + c;
    if (yy >= H || xx >= W) continue;
    float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j <= 2 * kR; ++j) {
      const float gj = win.g[j];
#pragma unroll
      for (int q = 0; q < 5; ++q) m[q] = fmaf(gj, hs[q][r + j][c], m[q]);
    }
    const float mx = m[0], my = m[1];
    const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
    const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
    const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
    const float iB = 1.f / (B1 * B2);
    const float S = A1 * A2 * iB;
    // dS/dmu_x holding the sigmas, dS/dsigma_x^2, dS/dsigma_xy
    const float dmu = 2.f * my * A2 * iB - 2.f * mx * S / B1;
    const float dsx = -S / B2;
    const float dsxy = 2.f * A1 * iB;
    const size_t p = (size_t)yy * W + xx;
    abc[ch * HW + p] = dmu - 2.f * mx * dsx - my * dsxy;     // a
    abc[(gridDim.z + ch) * HW + p] = dsx;                     // b
    abc[(2 * gridDim.z + ch) * HW + p] = dsxy;                // c
    ssum += S;
    lsum += fabsf(in[0][r + kR][c + kR] - in[1][r + kR][c + kR]);
  }
  red[0][threadIdx.x] = ssum;
  red[1][threadIdx.x] = lsum;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int b = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const int nb = gridDim.x * gridDim.y * gridDim.z;
    part[b] = red[0][0];
    part[nb + b] = red[1][0];
  }
}

__global__ void __launch_bounds__(256)
ssim_bwd_kernel(int H, int W, Window win, float ks, float kl, const float* __restrict__ img,
                const float* __restrict__ tgt, const float* __restrict__ abc,
                float* __restrict__ dimg) {
  __shared__ float in[3][kS][kS];
  __shared__ float hs[3][kS][kT];
  const int ch = blockIdx.z, x0 = blockIdx.x * kT, y0 = blockIdx.y * kT;
  const size_t HW = (size_t)H * W;
  {
    const float* const src[3] = {abc + ch * HW, abc + (gridDim.z + ch) * HW,
                                 abc + (2 * gridDim.z + ch) * HW};
    load_halo<3>(src, H, W, y0, x0, in);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kS * kT; i += blockDim.x) {
    const int r = i / kT, c = i - r * kT;
    float s[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j <= 2 * kR; ++j)
#pragma unroll
      for (int q = 0; q < 3; ++q) s[q] = fmaf(win.g[j], in[q][r][c + j], s[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q) hs[q][r][c] = s[q];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kT * kT; i += blockDim.x) {
    const int r = i / kT, c = i - r * kT;
    const int yy = y0 + r, xx = x0 + c;
    if (yy >= H || xx >= W) continue;
    float m[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j <= 2 * kR; ++j)
#pragma unroll
      for (int q = 0; q < 3; ++q) m[q] = fmaf(win.g[j], hs[q][r + j][c], m[q]);
    const size_t p = ch * HW + (size_t)yy * W + xx;
    const float xv = img[p], yv = tgt[p];
    const float dS = m[0] + 2.f * xv * m[1] + yv * m[2];
    const float sg = xv > yv ? 1.f : (xv < yv ? -1.f : 0.f);
    dimg[p] = fmaf(ks, dS, kl * sg);
  }
}

__global__ void __launch_bounds__(256)
ssim_final_kernel(int nb, float inv, float lam, const float* __restrict__ part,
                  float* __restrict__ loss) {
  __shared__ float red[2][256];
  float s = 0.f, l = 0.f;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    s += part[b];
    l += part[nb + b];
  }
  red[0][threadIdx.x] = s;
  red[1][threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    loss[0] = (1.f - lam) * red[1][0] * inv + lam * (1.f - red[0][0] * inv);
}

size_t tiles(int C, int H, int W) {
  return (size_t)rga::ceil_div(W, kT) * rga::ceil_div(H, kT) * C;
}

}  // namespace

extern "C" size_t image_loss_workspace(int C, int H, int W) {
  if (C < 1 || H < 1 || W < 1) return 0;
  return rga::align_up((size_t)3 * C * H * W * 4, 256) + 2 * tiles(C, H, W) * 4;
}

extern "C" int image_loss(void* stream, int C, int H, int W, const float* image,
                          const float* target, float lambda, float* loss, float* dimage, void* ws,
                          size_t ws_bytes) {
  if (C < 1 || H < 1 || W < 1 || C > 65535 || H > (1 << 20) || W > (1 << 20))
    return rga::fail(RGA_EINVAL, "image_loss: C in 1..65535, H and W in 1..2^20");
  if (!(lambda >= 0.f && lambda <= 1.f)) return rga::fail(RGA_EINVAL, "image_loss: lambda in [0, 1]");
  if (!image || !target || !loss || !ws) return rga::fail(RGA_EINVAL, "image_loss: null pointer");
  if (ws_bytes < image_loss_workspace(C, H, W))
    return rga::fail(RGA_ECAPACITY, "image_loss: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  static const Window win = window();
  float* abc = static_cast<float*>(ws);
  float* part = reinterpret_cast<float*>(static_cast<char*>(ws) +
                                         rga::align_up((size_t)3 * C * H * W * 4, 256));
  const dim3 grid(rga::ceil_div(W, kT), rga::ceil_div(H, kT), C);
  const int nb = (int)tiles(C, H, W);
  const double count = (double)C * H * W;
  RGA_LAUNCH("ssim_fwd", ssim_fwd_kernel, grid, dim3(256), 0, s, H, W, win, image, target, abc,
             part);
  RGA_LAUNCH("ssim_final", ssim_final_kernel, dim3(1), dim3(256), 0, s, nb, (float)(1.0 / count),
             lambda, part, loss);
  if (dimage)
    RGA_LAUNCH("ssim_bwd", ssim_bwd_kernel, grid, dim3(256), 0, s, H, W, win,
               (float)(-lambda / count), (float)((1.0 - lambda) / count), image, target, abc,
               dimage);
  RGA_CHECK_LAUNCH("image_loss");
  return RGA_OK;
}
