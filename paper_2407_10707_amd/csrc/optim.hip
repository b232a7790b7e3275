// The optimiser of the training loop: Adam (Kingma and Ba), as 3DGS trains,
// one fused pass per parameter tensor (parameter, gradient and both moments
// read once and written once: 28 bytes per value, HBM-bound).
#include "common.h"

#include <cmath>

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock)
adam_kernel(int64_t count, float* __restrict__ p, const float* __restrict__ g,
            float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2, float eps,
            float ic1, float ic2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * ic1) / (sqrtf(vi * ic2) + eps);
  }
}

}  // namespace

extern "C" int adam_step(void* stream, int64_t count, float* param, const float* grad, float* m,
                         float* v, float lr, float beta1, float beta2, float eps, int step) {
  if (count < 0 || step < 1) return rga::fail(RGA_EINVAL, "adam_step: count >= 0, step >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
    return rga::fail(RGA_EINVAL, "adam_step: betas in [0, 1), eps > 0");
  if (count == 0) return RGA_OK;
  if (!param || !grad || !m || !v) return rga::fail(RGA_EINVAL, "adam_step: null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // bias corrections 1 / (1 - beta^t), formed in double on the host
  const float ic1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
  const float ic2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
  const int64_t blocks = std::min<int64_t>(rga::ceil_div(count, kBlock), 2048);
  RGA_LAUNCH("adam", adam_kernel, dim3(blocks), dim3(kBlock), 0, s, count, param, grad, m, v, lr,
             beta1, beta2, eps, ic1, ic2);
  RGA_CHECK_LAUNCH("adam_step");
  return RGA_OK;
}
