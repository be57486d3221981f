// tr_internal.h -- host-side internals shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/tr.h"
#include "tr_device.h"

namespace trh {

// Uniform-grid parameters, computed on the host from the device bounds.
struct GridParams {
  double lo[3], hi[3], h[3], inv[3];
  double delta;
  int32_t res[3];
  int64_t n_cells;
};

// Inputs of the count / scatter kernels.
struct BuildArgs {
  int32_t n_s, n_c, n_t;
  const double4 *sph64, *cylA64, *cylB64;
  const double4 *triA64, *triB64, *triC64;
  double lo[3], h[3], inv[3], delta;
  int32_t res[3];
};

// ---- grid build launchers (grid_build.hip) ----
// albedo = (r, g, b, opacity); sop / cop / top may be null (opaque)
struct PackArgs {
  int64_t n_s, n_c, n_t;
  const double *sc, *sr, *ca, *cb, *cr, *tv0, *tv1, *tv2;
  const float *srgb, *sop, *crgb, *cop, *trgb, *top;
  double4 *sph64, *cylA64, *cylW64, *cylB64, *triA64, *triB64, *triC64;
  float4 *albedo;
};
hipError_t launch_pack(const PackArgs &p, hipStream_t st);
// FP32 copies with positions relative to origin (the centre of the grid box);
// also maxes the scene's bounding radius about origin (FP64 bits) into
// *rmax64, which must be zero on entry
hipError_t launch_pack32(const BuildArgs &a, const double4 *cylW64, const double origin[3],
                         float4 *sph32, float4 *cylA32, float4 *cylW32, float4 *triV32,
                         float4 *triE1_32, float4 *triE2_32, unsigned long long *rmax64,
                         hipStream_t st);
// bounds: out6 = (lo xyz, hi xyz); scratch >= bounds_scratch_doubles(N) doubles
int64_t bounds_scratch_doubles(int64_t n_prims);
hipError_t launch_bounds(const BuildArgs &a, double *scratch, double *out6, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);
// per-cell counts (count zeroed) and their 64-bit total added to *total64 (zeroed)
hipError_t launch_count(const BuildArgs &a, uint32_t *count, unsigned long long *total64,
                        hipStream_t st);
// exclusive scan of n+1 entries in place (data[n] must be 0 on entry)
int64_t scan_scratch_u32(int64_t n);
hipError_t launch_scan(uint32_t *data, int64_t n_plus_1, uint32_t *scratch, hipStream_t st);
hipError_t launch_scatter(const BuildArgs &a, const uint32_t *cell_begin, uint32_t *cursor,
                          uint32_t *refs, hipStream_t st);
// empty-space distance field + per-cell traversal words (d0, d1: n_cells bytes each)
// Empty-space distances, walk lists (wsz: n_cells + 1 scratch words, scanned
// in place with scan_scratch) and the per-cell traversal records.
// cap: largest stored distance, 1..32 (1 = no jumps); anything else = 32
hipError_t launch_cellinfo(const uint32_t *cell_begin, const uint32_t *refs, const int32_t res[3],
                           int32_t cap, uint8_t *d0, uint8_t *d1, uint32_t *wsz,
                           uint32_t *scan_scratch, uint32_t *wrefs, trd::CellInfo *info,
                           hipStream_t st);
hipError_t launch_sort_cells(const uint32_t *cell_begin, int64_t n_cells, uint32_t *refs,
                             hipStream_t st);

// Linear BVH over all primitives (n >= 2): 4 float4 per internal node (see
// k_bvh_pack); node 0 is the root.  Scratch sizes: keys, vals, keys2, vals2,
// parent_l: n; flags (the sort's digit counts): bvh_sort_counts(n); left,
// right, parent_i, arrivals, height: n - 1; ibox: 6 (n - 1) doubles;
// scan_scratch: scan_scratch_u32(bvh_sort_counts(n)).
// launch_bvh_tree sorts, builds the hierarchy and leaves each internal
// node's depth (links from the root) in height[] and the largest depth in
// flags[0]; launch_bvh_boxes then computes the boxes level by level from
// that depth up and packs the records.
struct BvhScratch {
  uint32_t *keys, *vals, *keys2, *vals2, *flags, *scan_scratch, *arrivals;
  int32_t *left, *right, *parent_i, *parent_l, *height;
  double *ibox;
};
// Entries of the BVH walk's per-lane traversal stack.  A walk that visits a
// node at depth d holds at most d deferred siblings, so a tree of depth
// <= kBvhStack never overflows it; deeper trees are refused before launch.
constexpr int kBvhStack = 48;
int64_t bvh_sort_counts(int64_t n);
hipError_t launch_bvh_tree(const BuildArgs &a, const double lo[3], const double hi[3],
                           BvhScratch &w, hipStream_t st);
hipError_t launch_bvh_boxes(const BuildArgs &a, const BvhScratch &w, int32_t max_depth,
                            double margin, const double origin[3], float4 *nodes, hipStream_t st);

// ---- frame output (frame_out.hip) ----
// values -> bytes, floor(clamp(v, 0, 1) * 255 + 1/2); any alignment
hipError_t launch_quantize_rgb8(const float *in, int64_t n, uint8_t *out, hipStream_t st);
// Run-length Targa file of an 8-bit RGB image [H][W][3] (1 <= W, H <= 65535):
// sizes computes row_bytes[H], row_off[H] (absolute file offsets of the rows)
// and *total (the file size); write then fills out[0, *total), which must
// hold *total bytes.
hipError_t launch_tga_sizes(const uint8_t *rgb, int32_t W, int32_t H, int64_t *row_bytes,
                            int64_t *row_off, int64_t *total, hipStream_t st);
hipError_t launch_tga_write(const uint8_t *rgb, int32_t W, int32_t H, const int64_t *row_off,
                            const int64_t *total, uint8_t *out, hipStream_t st);
// rgb[i] = (rgb[i] + planes[0][i] + ... + planes[n_planes - 1][i]) / (n_planes + 1),
// summed in that order; planes are n floats apart
hipError_t launch_aa_mean(float *rgb, const float *planes, int32_t n_planes, int64_t n,
                          hipStream_t st);

// ---- render launchers ----
hipError_t launch_render_plain_f64(const trd::JobDev &job, uint64_t *stats, hipStream_t st);

struct WaveLaunch {
  const trd::JobDev *jobs;   // device array
  int32_t n_jobs;
  int64_t n_tiles;           // total tiles in the queue
  uint32_t *tile_counter;    // device, trd::kQueueWords words zeroed before the launch
  uint64_t *stats;           // device or null
  int32_t tile_w, banks, refill_below, count_ops;
  int32_t stripe;            // tiles per tile-queue stripe (a power of two)
  int32_t n_waves;           // persistent waves launched
  int32_t resolve;
  int32_t trans;             // some job composites transparent layers
  int32_t tri;               // some job's scene has triangles
  int32_t bvh;               // walk the scenes' BVHs instead of their grids
};
hipError_t launch_render_wave(const WaveLaunch &L, hipStream_t st);
hipError_t launch_zero_counter(uint32_t *p, hipStream_t st);
// write one job table entry (device memory) from the host's job, by a kernel
hipError_t launch_put_job(const trd::JobDev &J, trd::JobDev *dst, hipStream_t st);

// FP32 FMA rate (TFLOP/s) of non-packed v_fma_f32 over the whole device
hipError_t measure_fma_rate(hipStream_t st, int32_t n_cus, double *tflops);

hipError_t launch_debug_philox(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out,
                               hipStream_t st);
hipError_t launch_debug_ao_dirs(int64_t n, const float *nrm, const uint32_t *pix,
                                const uint32_t *smp, uint32_t view, uint32_t k0, uint32_t k1,
                                float *w, hipStream_t st);

}  // namespace trh
