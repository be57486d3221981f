// frame_out.hip -- 8-bit output of a rendered frame (the paper's "Image I/O"
// phase, Table 5, moved onto the GPU): every float value v becomes
// floor(min(max(v, 0), 1) * 255 + 1/2), NaN becoming 0.
//
// A streaming kernel, bound by HBM: 4 bytes read and 1 byte written per
// value.  Each thread converts four float4 groups placed 256 groups apart, so
// every load and store instruction of a wave covers one contiguous span
// (1 KiB of input, 256 B of output); the data is touched once, so it is read
// and written non-temporally.  The rounding is exact: a float times 255 is
// exact in double, so the conversion runs in FP64 (two FP64 ops per value
// are far below the memory time).
//
// Also here: the mean over an antialiased frame's sample planes, another
// streaming pass (A * 4 bytes read and 4 written per value).
#include "tr_internal.h"

namespace {

typedef float vf4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kPerThread = 4;                     // float4 groups per thread
constexpr int kGroups = kThreads * kPerThread;    // float4 groups per block

__device__ __forceinline__ uint32_t q8(float x) {
  double v = (double)x;
  v = v > 0.0 ? v : 0.0;  // also NaN
  v = v < 1.0 ? v : 1.0;
  return (uint32_t)floor(v * 255.0 + 0.5);
}

// n4 float4 groups of a 16-byte aligned input to 4-byte words of the output.
__global__ __launch_bounds__(kThreads) void k_quantize_vec(const vf4 *__restrict__ in,
                                                           uint32_t *__restrict__ out, int64_t n4) {
  const int64_t base = (int64_t)blockIdx.x * kGroups + threadIdx.x;
  vf4 v[kPerThread];
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    const int64_t i = base + (int64_t)j * kThreads;
    if (i < n4) v[j] = __builtin_nontemporal_load(&in[i]);
  }
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    const int64_t i = base + (int64_t)j * kThreads;
    if (i < n4) {
      const uint32_t w = q8(v[j].x) | (q8(v[j].y) << 8) | (q8(v[j].z) << 16) | (q8(v[j].w) << 24);
      __builtin_nontemporal_store(w, &out[i]);
    }
  }
}

// Any alignment and the values past the last whole group: one value per thread.
__global__ __launch_bounds__(kThreads) void k_quantize_scalar(const float *__restrict__ in,
                                                              uint8_t *__restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) out[i] = (uint8_t)q8(in[i]);
}

// Mean of an antialiased pixel's samples: sample 0 is already in rgb, samples
// 1..n_planes in the planes; the sum runs in sample order, so the result
// does not depend on how the samples were scheduled.
__global__ __launch_bounds__(kThreads) void k_aa_mean(float *rgb, const float *planes,
                                                      int32_t n_planes, int64_t n, float count) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    float sum = rgb[i];
    const float *p = planes + i;
    for (int32_t a = 0; a < n_planes; ++a, p += n) sum += *p;
    rgb[i] = sum / count;
  }
}

}  // namespace

namespace trh {

hipError_t launch_aa_mean(float *rgb, const float *planes, int32_t n_planes, int64_t n,
                          hipStream_t st) {
  if (n <= 0 || n_planes <= 0) return hipSuccess;
  int64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;  // grid-stride beyond 2M threads
  k_aa_mean<<<(unsigned)blocks, kThreads, 0, st>>>(rgb, planes, n_planes, n, (float)(n_planes + 1));
  return hipGetLastError();
}

hipError_t launch_quantize_rgb8(const float *in, int64_t n, uint8_t *out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const bool aligned = ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 4 == 0);
  int64_t done = 0;
  if (aligned) {
    const int64_t n4 = n / 4;
    if (n4 > 0) {
      const int64_t blocks = (n4 + kGroups - 1) / kGroups;
      k_quantize_vec<<<(unsigned)blocks, kThreads, 0, st>>>((const vf4 *)in, (uint32_t *)out, n4);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    done = n4 * 4;
  }
  const int64_t rest = n - done;
  if (rest > 0) {
    const int64_t blocks = (rest + kThreads - 1) / kThreads;
    k_quantize_scalar<<<(unsigned)blocks, kThreads, 0, st>>>(in + done, out + done, rest);
  }
  return hipGetLastError();
}

}  // namespace trh
