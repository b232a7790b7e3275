// L1 term of the image loss (Sec. 3.3): mean |I - I_target| and its gradient.
// Deterministic two-stage reduction (per-block partials, then one block).
#include "common.h"

namespace {

constexpr int kBlock = 256;
constexpr int kGrid = 1024;

__global__ void __launch_bounds__(kBlock)
l1_partial_kernel(int64_t count, const float* __restrict__ img, const float* __restrict__ tgt,
                  float* __restrict__ dimg, float inv_count, float* __restrict__ part) {
  __shared__ float red[kBlock];
  float s = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * kBlock) {
    const float d = img[i] - tgt[i];
    s += fabsf(d);
    if (dimg) dimg[i] = d > 0.f ? inv_count : (d < 0.f ? -inv_count : 0.f);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kBlock)
l1_final_kernel(int parts, const float* __restrict__ part, float inv_count, float* __restrict__ loss) {
  __shared__ float red[kBlock];
  float s = 0.f;
  for (int i = threadIdx.x; i < parts; i += kBlock) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] * inv_count;
}

}  // namespace

extern "C" size_t l1_loss_workspace(int64_t count) {
  (void)count;
  return kGrid * sizeof(float);
}

extern "C" int l1_loss(void* stream, int64_t count, const float* image, const float* target,
                       float* loss, float* dimage, void* ws, size_t ws_bytes) {
  if (count < 1) return rga::fail(RGA_EINVAL, "l1_loss: count >= 1");
  if (!image || !target || !loss || !ws) return rga::fail(RGA_EINVAL, "l1_loss: null pointer");
  if (ws_bytes < kGrid * sizeof(float)) return rga::fail(RGA_ECAPACITY, "l1_loss: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int grid = (int)(rga::ceil_div(count, kBlock) < kGrid ? rga::ceil_div(count, kBlock) : kGrid);
  const float inv = (float)(1.0 / (double)count);
  float* part = static_cast<float*>(ws);
  RGA_LAUNCH("l1_partial", l1_partial_kernel, dim3(grid), dim3(kBlock), 0, s, count, image, target,
             dimage, inv, part);
  RGA_LAUNCH("l1_final", l1_final_kernel, dim3(1), dim3(kBlock), 0, s, grid, part, inv, loss);
  RGA_CHECK_LAUNCH("l1_loss");
  return RGA_OK;
}
