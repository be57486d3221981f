// measure.hip -- the chip's FP32 multiply-add rate as the render kernel can
// issue it: non-packed v_fma_f32 (packed FP32 is disabled for all device code
// of the library), the measured peak the render kernel's FP32 roofline is
// also reported against.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tr_internal.h"

namespace {

constexpr int kChains = 16;    // independent FMA chains per lane
constexpr int kBlock = 256;    // threads per block (4 waves)

// Every lane runs kChains independent chains x <- x a + b for `iters` rounds:
// 2 kChains iters flops per lane, none of them foldable (a, b are arguments).
// One float per thread is stored so that the chains stay live.
__global__ __launch_bounds__(kBlock) void k_fma_rate(float *out, int32_t iters, float a, float b) {
  float x[kChains];
  const float s = (float)(blockIdx.x * kBlock + threadIdx.x) * 0x1p-24f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = s + (float)c;
  // iters is a multiple of 8: 128 FMAs per loop branch
#pragma unroll 8
  for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(x[c], a, b);
  }
  float acc = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc += x[c];
  out[blockIdx.x * kBlock + threadIdx.x] = acc;
}

}  // namespace

namespace trh {

hipError_t measure_fma_rate(hipStream_t st, int32_t n_cus, double *tflops) {
  const int32_t blocks = n_cus * 8;  // 32 waves per compute unit
  const int32_t iters = 4096;
  float *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void **)&out, sizeof(float) * (size_t)blocks * kBlock);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  double best = 0.0;
  for (int rep = 0; rep < 6 && e == hipSuccess; ++rep) {  // the first is a warm-up
    e = hipEventRecord(e0, st);
    if (e == hipSuccess) {
      k_fma_rate<<<blocks, kBlock, 0, st>>>(out, iters, 0.999f, 1e-3f);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && rep > 0 && ms > 0.0f) {
      const double flops = 2.0 * kChains * (double)iters * (double)blocks * kBlock;
      best = std::max(best, flops / (ms * 1e-3) / 1e12);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  *tflops = best;
  return e;
}

}  // namespace trh
