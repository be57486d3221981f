// grid_build.hip -- GPU build of the uniform grid (the "Preprocess" phase of
// the paper's Table 5): FP64 scene packing, bounds reduction, per-cell
// counting, exclusive prefix scan, scatter of primitive references, and an
// in-cell sort that makes the reference order deterministic.
//
// Compiled with -ffp-contract=off: the cell lists must equal, bit for bit,
// those of the grid definition (primitive boxes widened by delta, spheres
// kept only where their centre lies within r of the widened cell box).
#include "tr_internal.h"

namespace {

using namespace trd;

constexpr int kBlock = 256;

__device__ __forceinline__ void prim_box(const trh::BuildArgs &a, int64_t k, double lo[3],
                                         double hi[3]) {
  if (k < a.n_s) {
    const double4 s = a.sph64[k];
    lo[0] = s.x - s.w; lo[1] = s.y - s.w; lo[2] = s.z - s.w;
    hi[0] = s.x + s.w; hi[1] = s.y + s.w; hi[2] = s.z + s.w;
  } else if (k >= (int64_t)a.n_s + a.n_c) {  // triangle: min/max of its vertices
    const int64_t m = k - a.n_s - a.n_c;
    const double4 A = a.triA64[m], B = a.triB64[m], C = a.triC64[m];
    const double av[3] = {A.x, A.y, A.z}, bv[3] = {B.x, B.y, B.z}, cv[3] = {C.x, C.y, C.z};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double mn = av[q], mx = av[q];
      mn = bv[q] < mn ? bv[q] : mn;
      mx = bv[q] > mx ? bv[q] : mx;
      mn = cv[q] < mn ? cv[q] : mn;
      mx = cv[q] > mx ? cv[q] : mx;
      lo[q] = mn;
      hi[q] = mx;
    }
  } else {
    const int64_t m = k - a.n_s;
    const double4 A = a.cylA64[m], B = a.cylB64[m];
    const double av[3] = {A.x, A.y, A.z}, bv[3] = {B.x, B.y, B.z};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double mn = av[q] < bv[q] ? av[q] : bv[q];
      const double mx = av[q] < bv[q] ? bv[q] : av[q];
      lo[q] = mn - A.w;
      hi[q] = mx + A.w;
    }
  }
}

__device__ __forceinline__ int32_t cell_coord(const trh::BuildArgs &a, int q, double x) {
  const double f = floor((x - a.lo[q]) * a.inv[q]);
  if (!(f >= 0.0)) return 0;
  if (f > (double)(a.res[q] - 1)) return a.res[q] - 1;
  return (int32_t)f;
}

__device__ __forceinline__ bool sphere_in_cell(const trh::BuildArgs &a, const double4 s,
                                               int32_t ix, int32_t iy, int32_t iz) {
  const int32_t idx[3] = {ix, iy, iz};
  const double c[3] = {s.x, s.y, s.z};
  double d2 = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double cl = (a.lo[q] + (double)idx[q] * a.h[q]) - a.delta;
    const double ch = (a.lo[q] + (double)(idx[q] + 1) * a.h[q]) + a.delta;
    double e = 0.0;
    if (c[q] < cl) e = cl - c[q];
    else if (c[q] > ch) e = c[q] - ch;
    d2 = d2 + e * e;
  }
  return d2 <= s.w * s.w;
}

// Visit every cell primitive k is listed in.  kLanes lanes share a primitive:
// lane g takes the cells of its box whose linear index (x fastest) is g, g +
// kLanes, ...  A protein-sized scene has only tens of thousands of primitives,
// too few for one thread each to fill the chip.
constexpr int kLanes = 16;

template <class F>
__device__ __forceinline__ void for_prim_cells(const trh::BuildArgs &a, int64_t k, int g,
                                               F &&visit) {
  double lo[3], hi[3];
  prim_box(a, k, lo, hi);
  int32_t c0[3], n[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    c0[q] = cell_coord(a, q, lo[q] - a.delta);
    n[q] = cell_coord(a, q, hi[q] + a.delta) - c0[q] + 1;
  }
  const bool sph = k < a.n_s;
  double4 s = make_double4(0, 0, 0, 0);
  if (sph) s = a.sph64[k];
  // first cell of this lane, then steps of kLanes along x with carries
  int32_t ix = g, iy = 0, iz = 0;
  while (ix >= n[0]) { ix -= n[0]; ++iy; }
  while (iy >= n[1]) { iy -= n[1]; ++iz; }
  while (iz < n[2]) {
    const int32_t x = c0[0] + ix, y = c0[1] + iy, z = c0[2] + iz;
    if (!sph || sphere_in_cell(a, s, x, y, z))
      visit((uint32_t)(((int64_t)z * a.res[1] + y) * a.res[0] + x));
    ix += kLanes;
    while (ix >= n[0]) {
      ix -= n[0];
      if (++iy == n[1]) { iy = 0; ++iz; }
    }
  }
}

__global__ void k_pack(const trh::PackArgs P) {
  const int64_t n_s = P.n_s, n_c = P.n_c;
  const double *sc = P.sc, *sr = P.sr, *ca = P.ca, *cb = P.cb, *cr = P.cr;
  const float *srgb = P.srgb, *sop = P.sop, *crgb = P.crgb, *cop = P.cop;
  double4 *sph64 = P.sph64, *cylA64 = P.cylA64, *cylW64 = P.cylW64, *cylB64 = P.cylB64;
  float4 *albedo = P.albedo;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_s + n_c && k < n_s + n_c + P.n_t) {
    const int64_t m = k - n_s - n_c;
    P.triA64[m] = make_double4(P.tv0[3 * m], P.tv0[3 * m + 1], P.tv0[3 * m + 2], 0.0);
    P.triB64[m] = make_double4(P.tv1[3 * m], P.tv1[3 * m + 1], P.tv1[3 * m + 2], 0.0);
    P.triC64[m] = make_double4(P.tv2[3 * m], P.tv2[3 * m + 1], P.tv2[3 * m + 2], 0.0);
    albedo[k] = make_float4(P.trgb[3 * m], P.trgb[3 * m + 1], P.trgb[3 * m + 2],
                            P.top ? P.top[m] : 1.0f);
  }
  if (k < n_s) {
    sph64[k] = make_double4(sc[3 * k], sc[3 * k + 1], sc[3 * k + 2], sr[k]);
    albedo[k] = make_float4(srgb[3 * k], srgb[3 * k + 1], srgb[3 * k + 2], sop ? sop[k] : 1.0f);
  } else if (k < n_s + n_c) {
    const int64_t m = k - n_s;
    const double a[3] = {ca[3 * m], ca[3 * m + 1], ca[3 * m + 2]};
    const double b[3] = {cb[3 * m], cb[3 * m + 1], cb[3 * m + 2]};
    const double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double L = sqrt((ab[0] * ab[0] + ab[1] * ab[1]) + ab[2] * ab[2]);
    cylA64[m] = make_double4(a[0], a[1], a[2], cr[m]);
    cylW64[m] = make_double4(ab[0] / L, ab[1] / L, ab[2] / L, L);
    cylB64[m] = make_double4(b[0], b[1], b[2], 0.0);
    albedo[k] = make_float4(crgb[3 * m], crgb[3 * m + 1], crgb[3 * m + 2], cop ? cop[m] : 1.0f);
  }
}

// FP32 copies for the wavefront walk, with positions relative to the centre of
// the grid box (the FP32 frame: the smallest magnitudes, so the least rounding,
// wherever the scene sits).  Spheres and cylinders carry their squared radius
// (squared in FP64, then rounded), which is all the FP32 tests use.
//
// The same pass takes the scene's bounding radius about that centre: the
// largest distance from it of any point of any primitive (a sphere's centre
// distance plus its radius, a cylinder's farther end plus its radius, a
// triangle's farthest vertex), in FP64, as the bit pattern of a non-negative
// double (whose order is the integer order of its bits) maxed into *rmax64
// (zero on entry): one atomic per wave.
__device__ __forceinline__ double dist3(double x, double y, double z) {
  return sqrt((x * x + y * y) + z * z);
}

__global__ void k_pack32(const trh::BuildArgs a, const double4 *cylW64, double ox, double oy,
                         double oz, float4 *sph32, float4 *cylA32, float4 *cylW32, float4 *triV32,
                         float4 *triE1_32, float4 *triE2_32, unsigned long long *rmax64) {
  const int64_t n_s = a.n_s, n_c = a.n_c;
  const double4 *sph64 = a.sph64, *cylA64 = a.cylA64, *cylB64 = a.cylB64;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double ext = 0.0;  // this primitive's farthest point from the centre
  if (k >= n_s + n_c && k < n_s + n_c + a.n_t) {
    // triangle: v0 in the FP32 frame, its edges (differences taken in FP64),
    // and |e1 x e2| (the scale of the determinant) in v0's fourth word
    const int64_t m = k - n_s - n_c;
    const double4 A = a.triA64[m], B = a.triB64[m], C = a.triC64[m];
    const double e1[3] = {B.x - A.x, B.y - A.y, B.z - A.z};
    const double e2[3] = {C.x - A.x, C.y - A.y, C.z - A.z};
    const double nx = e1[1] * e2[2] - e1[2] * e2[1];
    const double ny = e1[2] * e2[0] - e1[0] * e2[2];
    const double nz = e1[0] * e2[1] - e1[1] * e2[0];
    triV32[m] = make_float4((float)(A.x - ox), (float)(A.y - oy), (float)(A.z - oz),
                            (float)sqrt((nx * nx + ny * ny) + nz * nz));
    ext = fmax(dist3(A.x - ox, A.y - oy, A.z - oz),
               fmax(dist3(B.x - ox, B.y - oy, B.z - oz), dist3(C.x - ox, C.y - oy, C.z - oz)));
    triE1_32[m] = make_float4((float)e1[0], (float)e1[1], (float)e1[2], 0.0f);
    triE2_32[m] = make_float4((float)e2[0], (float)e2[1], (float)e2[2], 0.0f);
  }
  if (k < n_s) {
    const double4 s = sph64[k];
    sph32[k] = make_float4((float)(s.x - ox), (float)(s.y - oy), (float)(s.z - oz), (float)(s.w * s.w));
    ext = dist3(s.x - ox, s.y - oy, s.z - oz) + s.w;
  } else if (k < n_s + n_c) {
    const int64_t m = k - n_s;
    const double4 a = cylA64[m], w = cylW64[m];
    cylA32[m] = make_float4((float)(a.x - ox), (float)(a.y - oy), (float)(a.z - oz), (float)(a.w * a.w));
    cylW32[m] = make_float4((float)w.x, (float)w.y, (float)w.z, (float)w.w);
    const double4 b = cylB64[m];
    // The bounding sphere of the (open) cylinder, after the spheres: centre
    // the axis midpoint, squared radius (L/2)^2 + rho^2, padded by 2^-9 and
    // rounded up, so the cylinder stays inside the FP32 sphere by a margin
    // far above the FP32 rounding of the test against it.
    const double hl = 0.5 * w.w;
    const float bb = (float)((hl * hl + a.w * a.w) * (1.0 + 0x1p-9));
    sph32[k] = make_float4((float)(0.5 * (a.x + b.x) - ox), (float)(0.5 * (a.y + b.y) - oy),
                           (float)(0.5 * (a.z + b.z) - oz), nextafterf(bb, INFINITY));
    ext = fmax(dist3(a.x - ox, a.y - oy, a.z - oz), dist3(b.x - ox, b.y - oy, b.z - oz)) + a.w;
  }
  // every lane gets here (no early return): the wave's maximum, one atomic
  for (int off = 32; off > 0; off >>= 1) ext = fmax(ext, __shfl_xor(ext, off, 64));
  if ((threadIdx.x & 63) == 0 && ext > 0.0)
    atomicMax(rmax64, (unsigned long long)__double_as_longlong(ext));
}

// Per-block min/max of primitive boxes -> scratch[block*6 .. +6].
__global__ __launch_bounds__(kBlock) void k_bounds_partial(const trh::BuildArgs a, double *part) {
  __shared__ double red[6][kBlock];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  const int64_t N = (int64_t)a.n_s + a.n_c + a.n_t;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < N;
       k += (int64_t)gridDim.x * kBlock) {
    double bl[3], bh[3];
    prim_box(a, k, bl, bh);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      lo[q] = bl[q] < lo[q] ? bl[q] : lo[q];
      hi[q] = bh[q] > hi[q] ? bh[q] : hi[q];
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    red[q][threadIdx.x] = lo[q];
    red[3 + q][threadIdx.x] = hi[q];
  }
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double x = red[q][threadIdx.x + s];
        if (x < red[q][threadIdx.x]) red[q][threadIdx.x] = x;
        const double y = red[3 + q][threadIdx.x + s];
        if (y > red[3 + q][threadIdx.x]) red[3 + q][threadIdx.x] = y;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[(int64_t)blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kBlock) void k_bounds_final(const double *part, int32_t n_part,
                                                         double *out6) {
  __shared__ double red[6][kBlock];
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int32_t b = threadIdx.x; b < n_part; b += kBlock) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double x = part[(int64_t)b * 6 + q];
      const double y = part[(int64_t)b * 6 + 3 + q];
      v[q] = x < v[q] ? x : v[q];
      v[3 + q] = y > v[3 + q] ? y : v[3 + q];
    }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) red[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double x = red[q][threadIdx.x + s];
        if (x < red[q][threadIdx.x]) red[q][threadIdx.x] = x;
        const double y = red[3 + q][threadIdx.x + s];
        if (y > red[3 + q][threadIdx.x]) red[3 + q][threadIdx.x] = y;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) out6[threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Per-cell counts, and the reference total summed in 64 bits (total64, zero
// on entry): the 32-bit counts are exact (a cell holds fewer than 2^28
// primitives), but their sum may pass 2^32, which the scan would wrap; the
// host reads total64 and refuses the grid before the scatter.
__global__ __launch_bounds__(kBlock) void k_count(trh::BuildArgs a, uint32_t *count,
                                                  unsigned long long *total64) {
  __shared__ unsigned long long blk;
  if (threadIdx.x == 0) blk = 0ull;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = t / kLanes;
  unsigned long long mine = 0ull;
  if (k < (int64_t)a.n_s + a.n_c + a.n_t)
    for_prim_cells(a, k, (int)(t % kLanes), [&](uint32_t c) {
      atomicAdd(&count[c], 1u);
      ++mine;
    });
  if (mine) atomicAdd(&blk, mine);
  __syncthreads();
  if (threadIdx.x == 0 && blk) atomicAdd(total64, blk);
}

__global__ void k_scatter(trh::BuildArgs a, const uint32_t *cell_begin, uint32_t *cursor,
                          uint32_t *refs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = t / kLanes;
  if (k >= (int64_t)a.n_s + a.n_c + a.n_t) return;
  for_prim_cells(a, k, (int)(t % kLanes), [&](uint32_t c) {
    const uint32_t pos = atomicAdd(&cursor[c], 1u);
    refs[cell_begin[c] + pos] = (uint32_t)k;
  });
}

// Ascending ids inside each cell (the scatter's atomics leave them in any
// order).  A block orders the lists of kBlock consecutive cells, whose
// references are one contiguous range of refs.  The range and the block's cell
// offsets are staged in LDS with coalesced loads; then every reference, one
// per thread, finds its cell by binary search over the offsets and goes to
// the slot given by its rank, the number of smaller ids in the same list (a
// primitive enters a cell once, so ranks are distinct).  Work per thread is
// the length of its own list, so the long lists of dense regions do not hold
// a wave back the way a per-cell sort does.  A block whose range exceeds the
// stage sorts in place in global memory instead (same result).
constexpr int kSortStage = 8192;  // refs per block staged in LDS (32 KiB)

__global__ __launch_bounds__(kBlock) void k_sort_cells(const uint32_t *cell_begin, int64_t n_cells,
                                                       uint32_t *refs) {
  __shared__ uint32_t stage[kSortStage];
  __shared__ uint32_t offs[kBlock + 1];
  const int64_t c0 = (int64_t)blockIdx.x * kBlock;
  const int64_t c = c0 + threadIdx.x;
  const int nb = (int)min((int64_t)kBlock, n_cells - c0);  // cells in this block
  const uint32_t r0 = cell_begin[c0], r1 = cell_begin[c0 + nb];
  const uint32_t n = r1 - r0;
  if (n <= (uint32_t)kSortStage) {
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) stage[i] = refs[r0 + i];
    for (int i = threadIdx.x; i <= nb; i += kBlock) offs[i] = cell_begin[c0 + i] - r0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
      // last k with offs[k] <= i; offs[0] = 0 <= i < n = offs[nb]
      int lo = 0, hi = nb;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (offs[mid] <= i) lo = mid; else hi = mid;
      }
      const uint32_t b = offs[lo], e = offs[lo + 1];
      const uint32_t v = stage[i];
      uint32_t rank = 0;
      for (uint32_t j = b; j < e; ++j) rank += stage[j] < v ? 1u : 0u;
      refs[r0 + b + rank] = v;
    }
  } else if (c < n_cells) {
    const uint32_t b = cell_begin[c], e = cell_begin[c + 1];
    for (uint32_t i = b + 1; i < e; ++i) {
      const uint32_t v = refs[i];
      uint32_t j = i;
      while (j > b && refs[j - 1] > v) {
        refs[j] = refs[j - 1];
        --j;
      }
      refs[j] = v;
    }
  }
}

// ---- empty-space distance field for the FP32 traversal
// dist(c) = Chebyshev distance, in cells, from c to the nearest occupied
// cell, capped at cap <= kDistCap (0 for occupied cells; cap 1 turns the
// jumps off: the walk is then a plain 3D-DDA).  Computed as three
// separable passes g(x) = min_r max(|r|, g(x + r e_axis)): the L-infinity
// distance is the min over occupied y of max over axes of |x_a - y_a|, and
// max distributes over min, so the axes can be taken one at a time.
constexpr int kDistCap = 32;

__global__ void k_dist_init(const uint32_t *cell_begin, int64_t n_cells, uint8_t *d, int32_t cap) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  d[c] = cell_begin[c + 1] > cell_begin[c] ? 0 : (uint8_t)cap;
}

__global__ void k_dist_pass(const uint8_t *in, uint8_t *out, int32_t rx, int32_t ry, int32_t rz,
                            int axis, int32_t cap) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)rx * ry * rz;
  if (c >= n) return;
  const int32_t ix = (int32_t)(c % rx);
  const int32_t iy = (int32_t)((c / rx) % ry);
  const int32_t iz = (int32_t)(c / ((int64_t)rx * ry));
  const int32_t p = axis == 0 ? ix : (axis == 1 ? iy : iz);
  const int32_t len = axis == 0 ? rx : (axis == 1 ? ry : rz);
  const int64_t stride = axis == 0 ? 1 : (axis == 1 ? (int64_t)rx : (int64_t)rx * ry);
  int32_t best = in[c];
  for (int32_t r = 1; r < best; ++r) {  // a neighbour r away can only give >= r
    const int32_t a = p - r >= 0 ? (int32_t)in[c - r * stride] : cap;
    const int32_t b = p + r < len ? (int32_t)in[c + r * stride] : cap;
    const int32_t v = max(r, min(a, b));
    best = min(best, v);
  }
  out[c] = (uint8_t)best;
}

// Walk-list sizes: an occupied cell's references plus one end marker (the
// extra last entry is 0, so the exclusive scan leaves the total there).
__global__ void k_walk_sizes(const uint32_t *cell_begin, int64_t n_cells, uint32_t *w) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > n_cells) return;
  const uint32_t n = c < n_cells ? cell_begin[c + 1] - cell_begin[c] : 0u;
  w[c] = n ? n + 1u : 0u;
}

// Traversal view of a cell, after the scan of the walk-list sizes: an
// occupied cell copies its sorted references to its walk list, appends -1,
// and records (byte offset of the list, first entry); an empty cell records
// (-distance, -1).  One 8-byte load gives the walk the cell's first unit of
// work, and the end marker ends the list without an end index.  The lists
// hold each primitive as its record offset, 16 x its id (the byte offset of
// its 16-byte FP32 records), with bit 0 set on a list's last entry, and the
// walk moves through them by byte offset: neither needs a multiply on the
// walk, and the walk knows a cell's last test when it makes it.  (The host keeps ids below 2^27 and
// the lists below 2^29 words, so both fit a signed 32-bit word.)
__global__ void k_cellinfo(const uint32_t *cell_begin, const uint32_t *refs, const uint32_t *wbegin,
                           const uint8_t *d, int64_t n_cells, int32_t rx, int32_t ry, int32_t cap,
                           uint32_t *wrefs, trd::CellInfo *info) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  const uint32_t b = cell_begin[c], e = cell_begin[c + 1];
  trd::CellInfo r;
  if (b < e) {
    const uint32_t w = wbegin[c];
    // bit 0 (free: record offsets are multiples of 16) flags a list's last entry
    for (uint32_t i = 0; i < e - b; ++i) wrefs[w + i] = (refs[b + i] << 4) | (i + 1 == e - b ? 1u : 0u);
    wrefs[w + (e - b)] = 0xFFFFFFFFu;
    r.a = (int32_t)(w << 2);
    r.c = (int32_t)((refs[b] << 4) | (e - b == 1 ? 1u : 0u));
  } else {
    // An empty cell: its Chebyshev distance dc (the cube of half-size dc - 1
    // about it is empty), and per octant of a ray's direction the block
    // ahead of it that is empty.  From the cell, the block of side 2m + 1
    // that extends ahead in octant o (axis a towards -a where bit a of o is
    // set) is the cube of half-size m about the cell m steps along that
    // octant's diagonal, so it is empty when that cell's distance is at
    // least m + 1.  Such blocks grow with m while the condition holds; the
    // record keeps the largest m, M <= 7 (and 2M + 1 within the cap), in
    // three bits per octant, and a ray in that octant jumps max(dc, 2M + 1)
    // cells ahead.  (The walk is clamped to the part of the cube ahead of
    // it, so a block that is empty ahead of the cell is enough.)  The scan
    // stays inside the grid.
    const int32_t dc = max((int32_t)d[c], 1);
    const int32_t ix = (int32_t)(c % rx), iy = (int32_t)((c / rx) % ry),
                  iz = (int32_t)(c / ((int64_t)rx * ry));
    const int32_t rz = (int32_t)(n_cells / ((int64_t)rx * ry));
    const int32_t mcap = min(7, (cap - 1) / 2);
    uint32_t ext = 0;
    for (int32_t o = 0; o < 8; ++o) {
      const int32_t sx = (o & 1) ? -1 : 1, sy = (o & 2) ? -1 : 1, sz = (o & 4) ? -1 : 1;
      int32_t m = 0;
      while (m < mcap) {
        const int32_t jx = ix + (m + 1) * sx, jy = iy + (m + 1) * sy, jz = iz + (m + 1) * sz;
        if (jx < 0 || jx >= rx || jy < 0 || jy >= ry || jz < 0 || jz >= rz) break;
        if ((int32_t)d[((int64_t)jz * ry + jy) * rx + jx] < m + 2) break;
        ++m;
      }
      ext |= (uint32_t)m << (3 * o);
    }
    r.a = -dc;
    r.c = (int32_t)(0x80000000u | ext);
  }
  info[c] = r;
}

// ---- exclusive scan: blocks of kScanItems, block sums scanned recursively
constexpr int kScanPer = 4;
constexpr int kScanItems = kBlock * kScanPer;

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
  // Hillis-Steele over kBlock values in shared memory
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const uint32_t add = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  total = sh[kBlock - 1];
  const uint32_t incl = sh[threadIdx.x];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_block(uint32_t *data, int64_t n, uint32_t *sums) {
  __shared__ uint32_t sh[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  uint32_t run = 0;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    v[q] = base + q < n ? data[base + q] : 0u;
    run += v[q];
  }
  uint32_t total;
  uint32_t off = block_excl_scan(run, sh, total);
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    if (base + q < n) data[base + q] = off;
    off += v[q];
  }
  if (threadIdx.x == 0 && sums) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t *data, int64_t n,
                                                     const uint32_t *offs) {
  const uint32_t add = offs[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * kScanPer;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q)
    if (base + q < n) data[base + q] += add;
}

inline unsigned blocks_for(int64_t n, int b = kBlock) {
  return (unsigned)((n + b - 1) / b);
}

// ---- linear BVH (Karras, "Maximizing parallelism in the construction of
// BVHs, octrees, and k-d trees", HPG 2012).  Primitives are ordered by the
// 30-bit Morton code of their box centres (10 bits per axis over the grid
// box); the N - 1 internal nodes then follow from the sorted codes alone:
// node i covers the run of leaves that share the longest common prefix with
// leaf i, split where that prefix grows.  Equal codes are told apart by
// their position in the sorted order.

__device__ __forceinline__ uint32_t morton30(uint32_t x, uint32_t y, uint32_t z) {
  uint32_t m = 0;
#pragma unroll
  for (int b = 0; b < 10; ++b)
    m |= (((x >> b) & 1u) << (3 * b + 2)) | (((y >> b) & 1u) << (3 * b + 1)) | (((z >> b) & 1u) << (3 * b));
  return m;
}

__global__ void k_bvh_morton(const trh::BuildArgs a, int64_t n, double lx, double ly, double lz,
                             double sx, double sy, double sz, uint32_t *keys, uint32_t *vals) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double lo[3], hi[3];
  prim_box(a, k, lo, hi);
  const double c[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
  const double l[3] = {lx, ly, lz}, sc[3] = {sx, sy, sz};
  uint32_t q[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double f = floor((c[i] - l[i]) * sc[i]);
    f = f < 0.0 ? 0.0 : (f > 1023.0 ? 1023.0 : f);
    q[i] = (uint32_t)f;
  }
  keys[k] = morton30(q[0], q[1], q[2]);
  vals[k] = (uint32_t)k;
}

// Stable LSD radix sort of the codes (with their primitive ids), 8 bits a
// pass.  A block takes a tile of 1024 keys in four chunks of 256.  Pass
// structure: count each digit per tile, scan the digit-major count table (so
// a tile's slot for digit d follows every smaller digit and every earlier
// tile's d), then scatter: a key's place is its tile's slot for its digit,
// plus the keys of that digit in earlier chunks, in lower waves of its chunk
// (per-wave counts in LDS) and in lower lanes of its wave (the lanes whose
// digit matches, from 8 ballots).
constexpr int kRadixTile = 1024;

__global__ __launch_bounds__(256) void k_radix_count(const uint32_t *keys, int64_t n, int shift,
                                                     int64_t nb, uint32_t *cnt) {
  __shared__ uint32_t hist[256];
  const int t = threadIdx.x;
  const int64_t b = blockIdx.x;
  hist[t] = 0u;
  __syncthreads();
  for (int c = 0; c < 4; ++c) {
    const int64_t i = b * kRadixTile + c * 256 + t;
    if (i < n) atomicAdd(&hist[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  cnt[(int64_t)t * nb + b] = hist[t];
  if (b == 0 && t == 0) cnt[256 * nb] = 0u;
}

__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t *keys, const uint32_t *vals,
                                                       int64_t n, int shift, int64_t nb,
                                                       const uint32_t *off, uint32_t *keys2,
                                                       uint32_t *vals2) {
  __shared__ uint32_t run[256];      // next place of each digit in this tile
  __shared__ uint32_t wcnt[4][256];  // keys of each digit in each wave of the chunk
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t b = blockIdx.x;
  run[t] = off[(int64_t)t * nb + b];
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int q = 0; q < 4; ++q) wcnt[q][t] = 0u;
    __syncthreads();
    const int64_t i = b * kRadixTile + c * 256 + t;
    const bool valid = i < n;
    const uint32_t key = valid ? keys[i] : 0u;
    const uint32_t d = (key >> shift) & 255u;
    uint64_t m = __ballot(valid);  // valid lanes with the same digit
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t bb = __ballot((d >> bit) & 1u);
      m &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    const uint64_t below = m & ((1ull << lane) - 1ull);
    if (valid && below == 0) wcnt[w][d] = (uint32_t)__popcll(m);  // the digit's lowest lane
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + (uint32_t)__popcll(below);
      for (int q = 0; q < w; ++q) pos += wcnt[q][d];
      if ((int64_t)pos < n) {
        keys2[pos] = key;
        vals2[pos] = vals[i];
      }
    }
    __syncthreads();
    run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    __syncthreads();
  }
}

// Child encoding: c >= 0 internal node c; c < 0 leaf at sorted position -c - 1.
__device__ __forceinline__ int prefix_len(const uint32_t *keys, int64_t n, int64_t i, int64_t j) {
  if (j < 0 || j >= n) return -1;
  const uint32_t a = keys[i], b = keys[j];
  if (a == b) return 32 + __clz((uint32_t)(i ^ j));
  return __clz(a ^ b);
}

__global__ void k_bvh_internal(const uint32_t *keys, int64_t n, int32_t *left, int32_t *right,
                               int32_t *parent_i, int32_t *parent_l) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  const int64_t d = prefix_len(keys, n, i, i + 1) - prefix_len(keys, n, i, i - 1) >= 0 ? 1 : -1;
  const int dmin = prefix_len(keys, n, i, i - d);
  int64_t lmax = 2;
  while (lmax < 2 * n && prefix_len(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
  int64_t l = 0;
  for (int64_t t = lmax / 2; t >= 1; t /= 2)
    if (prefix_len(keys, n, i, i + (l + t) * d) > dmin) l += t;
  const int64_t j = i + l * d;
  const int dnode = prefix_len(keys, n, i, j);
  int64_t s = 0, t = 0, div = 2;
  do {
    t = (l + div - 1) / div;
    if (prefix_len(keys, n, i, i + (s + t) * d) > dnode) s += t;
    div *= 2;
  } while (t > 1);
  const int64_t g = i + s * d + (d < 0 ? -1 : 0);
  const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
  const int32_t lc = lo == g ? (int32_t)(-g - 1) : (int32_t)g;
  const int32_t rc = hi == g + 1 ? (int32_t)(-(g + 1) - 1) : (int32_t)(g + 1);
  left[i] = lc;
  right[i] = rc;
  if (lc >= 0) parent_i[lc] = (int32_t)i; else parent_l[-lc - 1] = (int32_t)i;
  if (rc >= 0) parent_i[rc] = (int32_t)i; else parent_l[-rc - 1] = (int32_t)i;
  if (i == 0) parent_i[0] = -1;
}

// Box of a child: a leaf's primitive box widened by margin, or the stored
// box of an internal node (written by an earlier launch).
__device__ __forceinline__ void child_box(const trh::BuildArgs &a, const uint32_t *vals,
                                          const double *ibox, int32_t c, double margin,
                                          double lo[3], double hi[3]) {
  if (c < 0) {
    prim_box(a, (int64_t)vals[-c - 1], lo, hi);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      lo[q] -= margin;
      hi[q] += margin;
    }
  } else {
    const double *b = ibox + 6 * (int64_t)c;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      lo[q] = b[q];
      hi[q] = b[3 + q];
    }
  }
}

// Depth of every internal node (links from the root), by pointer jumping
// over the parent links: after r rounds each node has summed 2^r links of its
// path (the root links to itself with 0).  A path's split lengths rise
// strictly through at most 62 values (30 code bits, then position bits), so
// depths stay below 64 and 6 rounds give them exactly.  Links are clamped to
// the node range.
__global__ void k_bvh_depth_init(const int32_t *parent_i, int64_t m, int32_t *dep, int32_t *nxt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t p = i ? parent_i[i] : 0;
  dep[i] = i ? 1 : 0;
  nxt[i] = (uint32_t)p < (uint32_t)m ? p : 0;
}

__global__ void k_bvh_depth_jump(const int32_t *dep, const int32_t *nxt, int64_t m, int32_t *dep2,
                                 int32_t *nxt2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t j = nxt[i];
  dep2[i] = dep[i] + dep[j];
  nxt2[i] = nxt[j];
}

// Largest depth: a wave maximum, then the workgroup's in LDS, then one
// atomic per workgroup (one per wave contends on the single word).
__global__ __launch_bounds__(kBlock) void k_bvh_depth_max(const int32_t *dep, int64_t m,
                                                          uint32_t *out) {
  __shared__ int32_t wmax[kBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t v = i < m ? dep[i] : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t b = wmax[0];
    for (int k = 1; k < kBlock / 64; ++k) b = max(b, wmax[k]);
    atomicMax(out, (uint32_t)b);
  }
}

// Boxes of the internal nodes at depth d: the union of their children's
// boxes (a deeper level's, stored by the previous launch, or a leaf's).
__global__ void k_bvh_level(const trh::BuildArgs a, const uint32_t *vals, int64_t m,
                            const int32_t *dep, int32_t d, const int32_t *left,
                            const int32_t *right, double *ibox, double margin) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m || dep[i] != d) return;
  double l0[3], h0[3], l1[3], h1[3];
  child_box(a, vals, ibox, left[i], margin, l0, h0);
  child_box(a, vals, ibox, right[i], margin, l1, h1);
  double *b = ibox + 6 * i;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    b[k] = l0[k] < l1[k] ? l0[k] : l1[k];
    b[3 + k] = h0[k] > h1[k] ? h0[k] : h1[k];
  }
}

// Traversal records, one per internal node (64 bytes): both children's
// boxes in the FP32 frame, rounded outwards, then the children (an internal
// node index, or -(primitive id) - 1 for a leaf).
__global__ void k_bvh_pack(const trh::BuildArgs a, const uint32_t *vals, int64_t n,
                           const int32_t *left, const int32_t *right, const double *ibox,
                           double margin, double ox, double oy, double oz, float4 *nodes) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  const double o[3] = {ox, oy, oz};
  float f[12];
  int32_t ch[2] = {left[i], right[i]};
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    double lo[3], hi[3];
    child_box(a, vals, ibox, ch[c], margin, lo, hi);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      f[6 * c + q] = __double2float_rd(lo[q] - o[q]);
      f[6 * c + 3 + q] = __double2float_ru(hi[q] - o[q]);
    }
    if (ch[c] < 0) ch[c] = -(int32_t)vals[-ch[c] - 1] - 1;
  }
  float4 *r = nodes + 4 * i;
  r[0] = make_float4(f[0], f[1], f[2], f[3]);
  r[1] = make_float4(f[4], f[5], f[6], f[7]);
  r[2] = make_float4(f[8], f[9], f[10], f[11]);
  r[3] = make_float4(__int_as_float(ch[0]), __int_as_float(ch[1]), 0.0f, 0.0f);
}

}  // namespace

namespace trh {

hipError_t launch_pack(const PackArgs &p, hipStream_t st) {
  const int64_t N = p.n_s + p.n_c + p.n_t;
  if (N == 0) return hipSuccess;
  k_pack<<<blocks_for(N), kBlock, 0, st>>>(p);
  return hipGetLastError();
}

hipError_t launch_pack32(const BuildArgs &a, const double4 *cylW64, const double origin[3],
                         float4 *sph32, float4 *cylA32, float4 *cylW32, float4 *triV32,
                         float4 *triE1_32, float4 *triE2_32, unsigned long long *rmax64,
                         hipStream_t st) {
  const int64_t N = (int64_t)a.n_s + a.n_c + a.n_t;
  if (N == 0) return hipSuccess;
  k_pack32<<<blocks_for(N), kBlock, 0, st>>>(a, cylW64, origin[0], origin[1], origin[2], sph32,
                                             cylA32, cylW32, triV32, triE1_32, triE2_32, rmax64);
  return hipGetLastError();
}

static int32_t bounds_blocks(int64_t N) {
  int64_t b = (N + kBlock * 8 - 1) / (kBlock * 8);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int32_t)b;
}

int64_t bounds_scratch_doubles(int64_t n_prims) { return 6 * (int64_t)bounds_blocks(n_prims); }

hipError_t launch_bounds(const BuildArgs &a, double *scratch, double *out6, hipStream_t st) {
  const int32_t nb = bounds_blocks((int64_t)a.n_s + a.n_c + a.n_t);
  k_bounds_partial<<<nb, kBlock, 0, st>>>(a, scratch);
  k_bounds_final<<<1, kBlock, 0, st>>>(scratch, nb, out6);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t b = blocks_for(n);
  if (b > 65536) b = 65536;
  k_fill_u32<<<(unsigned)b, kBlock, 0, st>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_count(const BuildArgs &a, uint32_t *count, unsigned long long *total64,
                        hipStream_t st) {
  const int64_t N = (int64_t)a.n_s + a.n_c + a.n_t;
  if (N == 0) return hipSuccess;
  k_count<<<blocks_for(N * kLanes), kBlock, 0, st>>>(a, count, total64);
  return hipGetLastError();
}

int64_t scan_scratch_u32(int64_t n) {
  int64_t total = 0;
  while (n > kScanItems) {
    n = (n + kScanItems - 1) / kScanItems;
    total += n;
  }
  return total + 1;
}

hipError_t launch_scan(uint32_t *data, int64_t n, uint32_t *scratch, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n <= kScanItems) {
    k_scan_block<<<1, kBlock, 0, st>>>(data, n, nullptr);
    return hipGetLastError();
  }
  const int64_t nb = (n + kScanItems - 1) / kScanItems;
  uint32_t *sums = scratch;
  k_scan_block<<<(unsigned)nb, kBlock, 0, st>>>(data, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan(sums, nb, scratch + nb, st);
  if (e != hipSuccess) return e;
  k_scan_add<<<(unsigned)nb, kBlock, 0, st>>>(data, n, sums);
  return hipGetLastError();
}

hipError_t launch_scatter(const BuildArgs &a, const uint32_t *cell_begin, uint32_t *cursor,
                          uint32_t *refs, hipStream_t st) {
  const int64_t N = (int64_t)a.n_s + a.n_c + a.n_t;
  if (N == 0) return hipSuccess;
  k_scatter<<<blocks_for(N * kLanes), kBlock, 0, st>>>(a, cell_begin, cursor, refs);
  return hipGetLastError();
}

int64_t bvh_sort_counts(int64_t n) { return 256 * ((n + kRadixTile - 1) / kRadixTile) + 1; }

hipError_t launch_bvh_tree(const BuildArgs &a, const double lo[3], const double hi[3],
                           BvhScratch &w, hipStream_t st) {
  const int64_t n = (int64_t)a.n_s + a.n_c + a.n_t;
  if (n < 2) return hipSuccess;
  const unsigned nb = blocks_for(n);
  double sc[3];
  for (int q = 0; q < 3; ++q) sc[q] = hi[q] > lo[q] ? 1024.0 / (hi[q] - lo[q]) : 0.0;
  k_bvh_morton<<<nb, kBlock, 0, st>>>(a, n, lo[0], lo[1], lo[2], sc[0], sc[1], sc[2], w.keys, w.vals);
  uint32_t *k0 = w.keys, *v0 = w.vals, *k1 = w.keys2, *v1 = w.vals2;
  const int64_t tiles = (n + kRadixTile - 1) / kRadixTile;
  for (int shift = 0; shift < 30; shift += 8) {
    k_radix_count<<<(unsigned)tiles, 256, 0, st>>>(k0, n, shift, tiles, w.flags);
    hipError_t e = launch_scan(w.flags, 256 * tiles + 1, w.scan_scratch, st);
    if (e != hipSuccess) return e;
    k_radix_scatter<<<(unsigned)tiles, 256, 0, st>>>(k0, v0, n, shift, tiles, w.flags, k1, v1);
    uint32_t *tk = k0, *tv = v0;
    k0 = k1;
    v0 = v1;
    k1 = tk;
    v1 = tv;
  }
  // 4 passes: the sorted arrays are back in keys / vals; keys2 / vals2 are free
  const int64_t m = n - 1;
  const unsigned nbm = blocks_for(m);
  k_bvh_internal<<<nbm, kBlock, 0, st>>>(w.keys, n, w.left, w.right, w.parent_i, w.parent_l);
  int32_t *dep = w.height, *nxt = (int32_t *)w.arrivals;
  int32_t *dep2 = (int32_t *)w.keys2, *nxt2 = (int32_t *)w.vals2;
  k_bvh_depth_init<<<nbm, kBlock, 0, st>>>(w.parent_i, m, dep, nxt);
  for (int r = 0; r < 6; ++r) {  // even: the depths end in dep
    k_bvh_depth_jump<<<nbm, kBlock, 0, st>>>(dep, nxt, m, dep2, nxt2);
    int32_t *td = dep, *tn = nxt;
    dep = dep2;
    nxt = nxt2;
    dep2 = td;
    nxt2 = tn;
  }
  hipError_t e = launch_fill_u32(w.flags, 1, 0u, st);
  if (e != hipSuccess) return e;
  k_bvh_depth_max<<<nbm, kBlock, 0, st>>>(w.height, m, w.flags);
  return hipGetLastError();
}

hipError_t launch_bvh_boxes(const BuildArgs &a, const BvhScratch &w, int32_t max_depth,
                            double margin, const double origin[3], float4 *nodes, hipStream_t st) {
  const int64_t n = (int64_t)a.n_s + a.n_c + a.n_t;
  if (n < 2) return hipSuccess;
  const int64_t m = n - 1;
  const unsigned nbm = blocks_for(m);
  for (int32_t d = max_depth; d >= 0; --d)
    k_bvh_level<<<nbm, kBlock, 0, st>>>(a, w.vals, m, w.height, d, w.left, w.right, w.ibox, margin);
  k_bvh_pack<<<nbm, kBlock, 0, st>>>(a, w.vals, n, w.left, w.right, w.ibox, margin, origin[0],
                                     origin[1], origin[2], nodes);
  return hipGetLastError();
}

hipError_t launch_sort_cells(const uint32_t *cell_begin, int64_t n_cells, uint32_t *refs,
                             hipStream_t st) {
  if (n_cells <= 0) return hipSuccess;
  k_sort_cells<<<(unsigned)((n_cells + kBlock - 1) / kBlock), kBlock, 0, st>>>(cell_begin, n_cells, refs);
  return hipGetLastError();
}

hipError_t launch_cellinfo(const uint32_t *cell_begin, const uint32_t *refs, const int32_t res[3],
                           int32_t cap, uint8_t *d0, uint8_t *d1, uint32_t *wsz,
                           uint32_t *scan_scratch, uint32_t *wrefs, trd::CellInfo *info,
                           hipStream_t st) {
  const int64_t n = (int64_t)res[0] * res[1] * res[2];
  if (n <= 0) return hipSuccess;
  const unsigned nb = blocks_for(n);
  if (cap < 1 || cap > kDistCap) cap = kDistCap;
  k_dist_init<<<nb, kBlock, 0, st>>>(cell_begin, n, d0, cap);
  k_dist_pass<<<nb, kBlock, 0, st>>>(d0, d1, res[0], res[1], res[2], 0, cap);
  k_dist_pass<<<nb, kBlock, 0, st>>>(d1, d0, res[0], res[1], res[2], 1, cap);
  k_dist_pass<<<nb, kBlock, 0, st>>>(d0, d1, res[0], res[1], res[2], 2, cap);
  k_walk_sizes<<<blocks_for(n + 1), kBlock, 0, st>>>(cell_begin, n, wsz);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan(wsz, n + 1, scan_scratch, st);
  if (e != hipSuccess) return e;
  k_cellinfo<<<nb, kBlock, 0, st>>>(cell_begin, refs, wsz, d1, n, res[0], res[1], cap, wrefs, info);
  return hipGetLastError();
}

}  // namespace trh
