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
// streaming pass (A * 4 bytes read and 4 written per value), and the
// run-length Targa file of an 8-bit image (see k_tga_rows).
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

// ---- Targa file, run-length true colour (the packet rule is written out
// with the host-side declaration).  One wave per image row; each lane takes
// kTgaPx adjacent pixels, so a step covers 64 * kTgaPx pixels and issues all
// its byte loads at once.  A pixel's role follows from its neighbours alone:
// it belongs to a run when it equals a neighbour; a segment (a maximal run
// of one colour, or a maximal stretch of pixels in no run) starts where the
// role changes or a run changes colour; packets are the 128-pixel pieces of
// segments.  A pixel's segment starts at the last start at or before it: in
// its own lane, else the last one of the lower lanes (a max scan), else the
// segment still open from the previous step.  A run packet's 4 bytes belong
// to its last pixel, a raw packet's header byte to its first, so a pixel's
// byte position is the exclusive prefix sum of these sizes along the row.
// Pass 1 sums each row, a scan turns the sums into row offsets, pass 2
// recomputes the roles and writes.  The file is 18 header bytes, the rows,
// 26 footer bytes.

constexpr int kTgaHead = 18, kTgaFoot = 26;
constexpr int kTgaPx = 8;  // pixels per lane per step
__constant__ char kTgaSig[18] = "TRUEVISION-XFILE.";  // footer signature (with its zero)

__device__ __forceinline__ uint32_t px3(const uint8_t *row, int32_t x) {
  const uint8_t *p = row + 3 * (int64_t)x;
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
}

template <bool WRITE>
__global__ __launch_bounds__(64) void k_tga_rows(const uint8_t *__restrict__ rgb, int32_t W,
                                                 int64_t *__restrict__ row_bytes,
                                                 const int64_t *__restrict__ row_off,
                                                 uint8_t *__restrict__ out) {
  const int32_t y = blockIdx.x;
  const int32_t lane = threadIdx.x;
  const uint8_t *row = rgb + (int64_t)y * W * 3;
  const int64_t base = WRITE ? row_off[y] : 0;
  int64_t done = 0;      // bytes of the row before this step's pixels
  int32_t open_seg = 0;  // first pixel of the segment still open at the step's start
  for (int32_t x0 = 0; x0 < W; x0 += 64 * kTgaPx) {
    const int32_t xb = x0 + kTgaPx * lane;  // this lane's first pixel
    // the lane's pixels and two neighbours on each side
    uint32_t w[kTgaPx + 4];
    bool has[kTgaPx + 4];
#pragma unroll
    for (int k = 0; k < kTgaPx + 4; ++k) {
      const int32_t x = xb - 2 + k;
      has[k] = x >= 0 && x < W;
      w[k] = has[k] ? px3(row, x) : 0u;
    }
    bool run[kTgaPx], start[kTgaPx], end[kTgaPx];
    int32_t last_start = -1;
#pragma unroll
    for (int j = 0; j < kTgaPx; ++j) {
      const bool valid = has[j + 2];
      const bool eq_l = valid && has[j + 1] && w[j + 2] == w[j + 1];
      const bool eq_r = valid && has[j + 3] && w[j + 2] == w[j + 3];
      run[j] = eq_l || eq_r;
      const bool run_l = has[j + 1] && (eq_l || (has[j] && w[j + 1] == w[j]));  // pixel before
      const bool run_r = has[j + 3] && (eq_r || (has[j + 4] && w[j + 3] == w[j + 4]));  // after
      start[j] = valid && (!has[j + 1] || run[j] != run_l || (run[j] && !eq_l));
      end[j] = valid && (!has[j + 3] || run[j] != run_r || (run_r && !eq_r));  // next one starts
      if (start[j]) last_start = xb + j;
    }
    // last segment start of the lanes below (exclusive max scan) and of the wave
    int32_t m = last_start;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t v = __shfl_up(m, d);
      if (lane >= d) m = max(m, v);
    }
    int32_t below = __shfl_up(m, 1);
    if (lane == 0) below = -1;
    const int32_t wave_last = __shfl(m, 63);
    const int32_t seg_before = below >= 0 ? below : open_seg;
    int32_t kk[kTgaPx], bytes[kTgaPx];
    int32_t seg_in = -1, lane_sum = 0;
#pragma unroll
    for (int j = 0; j < kTgaPx; ++j) {
      if (start[j]) seg_in = xb + j;
      const int32_t seg = seg_in >= 0 ? seg_in : seg_before;
      kk[j] = (xb + j - seg) & 127;  // position in its packet
      const bool first = kk[j] == 0, last = kk[j] == 127 || end[j];
      bytes[j] = !has[j + 2] ? 0 : (run[j] ? (last ? 4 : 0) : (first ? 4 : 3));
      lane_sum += bytes[j];
    }
    int32_t incl = lane_sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t v = __shfl_up(incl, d);
      if (lane >= d) incl += v;
    }
    if (WRITE) {
      int64_t pos = base + done + (incl - lane_sum);
#pragma unroll
      for (int j = 0; j < kTgaPx; ++j) {
        if (has[j + 2]) {
          const uint32_t p0 = w[j + 2];
          const uint8_t r = (uint8_t)(p0 & 255u), g = (uint8_t)((p0 >> 8) & 255u),
                        b = (uint8_t)(p0 >> 16);
          const bool first = kk[j] == 0, last = kk[j] == 127 || end[j];
          if (run[j]) {
            if (last) {
              out[pos] = (uint8_t)(0x80 | kk[j]);
              out[pos + 1] = b;
              out[pos + 2] = g;
              out[pos + 3] = r;
            }
          } else {
            const int64_t q = pos + (first ? 1 : 0);
            out[q] = b;
            out[q + 1] = g;
            out[q + 2] = r;
            // the header sits before the packet's first pixel: 1 + 3 kk bytes back
            if (last) out[first ? pos : pos - 1 - 3 * (int64_t)kk[j]] = (uint8_t)kk[j];
          }
        }
        pos += bytes[j];
      }
    }
    done += __shfl(incl, 63);
    if (wave_last >= 0) open_seg = wave_last;
  }
  if (!WRITE && lane == 0) row_bytes[y] = done;
}

// Row offsets (exclusive sum of row sizes, after the header) and the file
// size, in one workgroup: each thread sums a contiguous block of rows, the
// block sums are scanned in LDS, then each thread writes its rows' offsets.
__global__ __launch_bounds__(1024) void k_tga_offsets(const int64_t *__restrict__ row_bytes,
                                                      int32_t H, int64_t *__restrict__ row_off,
                                                      int64_t *__restrict__ total) {
  __shared__ int64_t part[1024];
  const int32_t t = threadIdx.x;
  const int32_t per = (H + 1023) / 1024;
  const int32_t b = min(H, t * per), e = min(H, b + per);
  int64_t s = 0;
  for (int32_t i = b; i < e; ++i) s += row_bytes[i];
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t at = kTgaHead + (t ? part[t - 1] : 0);
  for (int32_t i = b; i < e; ++i) {
    row_off[i] = at;
    at += row_bytes[i];
  }
  if (t == 1023) *total = kTgaHead + part[1023] + kTgaFoot;
}

// Header (no image id or colour map, type 10, width, height, 24 bits, rows
// top first) and footer (no extension or developer area, the signature).
__global__ __launch_bounds__(64) void k_tga_frame(int32_t W, int32_t H,
                                                  const int64_t *__restrict__ total,
                                                  uint8_t *__restrict__ out) {
  const int32_t t = threadIdx.x;
  if (t < kTgaHead) {
    uint8_t v = 0;
    switch (t) {
      case 2: v = 10; break;
      case 12: v = (uint8_t)(W & 255); break;
      case 13: v = (uint8_t)(W >> 8); break;
      case 14: v = (uint8_t)(H & 255); break;
      case 15: v = (uint8_t)(H >> 8); break;
      case 16: v = 24; break;
      case 17: v = 0x20; break;
      default: break;
    }
    out[t] = v;
  } else if (t < kTgaHead + kTgaFoot) {
    const int32_t k = t - kTgaHead;  // footer byte
    out[*total - kTgaFoot + k] = k < 8 ? (uint8_t)0 : (uint8_t)kTgaSig[k - 8];
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

namespace trh {

hipError_t launch_tga_sizes(const uint8_t *rgb, int32_t W, int32_t H, int64_t *row_bytes,
                            int64_t *row_off, int64_t *total, hipStream_t st) {
  k_tga_rows<false><<<(unsigned)H, 64, 0, st>>>(rgb, W, row_bytes, nullptr, nullptr);
  k_tga_offsets<<<1, 1024, 0, st>>>(row_bytes, H, row_off, total);
  return hipGetLastError();
}

hipError_t launch_tga_write(const uint8_t *rgb, int32_t W, int32_t H, const int64_t *row_off,
                            const int64_t *total, uint8_t *out, hipStream_t st) {
  k_tga_rows<true><<<(unsigned)H, 64, 0, st>>>(rgb, W, nullptr, row_off, out);
  k_tga_frame<<<1, 64, 0, st>>>(W, H, total, out);
  return hipGetLastError();
}

}  // namespace trh
