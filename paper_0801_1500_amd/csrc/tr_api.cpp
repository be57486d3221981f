// tr_api.cpp -- the C ABI (include/tr.h): validation, scene build
// orchestration, job tables, launches, graphs and the autotuner.
//
// Host arithmetic that feeds bit-exact device work (camera basis, light
// normalisation, grid parameters) is compiled with -ffp-contract=off and
// written in the order of the method's definition.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "tr_internal.h"

using trd::JobDev;
using trd::SceneDev;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static tr_status fail(tr_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? TR_ENOMEM : TR_EDEVICE, "%s: %s (%s)",    \
                  #expr, hipGetErrorName(e_), hipGetErrorString(e_));                  \
  } while (0)

static bool finite3(const double *v) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

// ------------------------------------------------------------------ scene
struct tr_scene {
  int device = 0;
  int32_t key = 0;
  int64_t n_s = 0, n_c = 0, n_t = 0;
  int32_t n_lights = 0;
  double ldir[8][3] = {};
  double ldir_in[8][3] = {};  // light directions as given (saved by tr_scene_save)
  double lrgb[8][3] = {};
  double lambda = 24.0;
  int32_t max_skip = 32;  // cap of the empty-space distance field (1 = plain 3D-DDA)
  // device arrays
  double4 *sph64 = nullptr, *cylA64 = nullptr, *cylW64 = nullptr, *cylB64 = nullptr;
  float4 *sph32 = nullptr, *cylA32 = nullptr, *cylW32 = nullptr, *albedo = nullptr;
  double4 *triA64 = nullptr, *triB64 = nullptr, *triC64 = nullptr;
  float4 *bvh_nodes = nullptr;  // linear BVH (tr_scene_build_bvh), 4 per internal node
  int64_t bvh_n = 0;            // primitives it covers (0 = not built)
  int64_t bvh_cap = 0;          // internal-node records the buffer holds
  int32_t bvh_depth = 0;        // internal nodes on its longest root-to-leaf path
  float4 *triV32 = nullptr, *triE1_32 = nullptr, *triE2_32 = nullptr;
  uint32_t *cell_begin = nullptr, *refs = nullptr, *count = nullptr, *scan_scratch = nullptr;
  uint32_t *wrefs = nullptr;  // FP32 walk lists: per occupied cell its references, then -1
  trd::CellInfo *cellinfo = nullptr;
  uint8_t *dist0 = nullptr, *dist1 = nullptr;
  double *bounds_scratch = nullptr, *bounds = nullptr;
  // device: [0] reference total of the count pass, [1] bounding radius (FP64 bits)
  unsigned long long *total64 = nullptr;
  int64_t cap_cells = 0, cap_refs = 0, cap_scan = 0, cap_wrefs = 0;
  size_t bytes_arrays = 0;
  // pinned readback
  double *h_bounds = nullptr;
  unsigned long long *h_total = nullptr;
  trh::GridParams gp{};
  int64_t n_refs = 0;
  bool grid_ok = false;  // false after a failed (re)build: the scene cannot render
  bool has_trans = false;  // some primitive has opacity < 1 (kept in albedo.w)
  double org[3] = {0, 0, 0};  // origin of the FP32 frame: centre of the grid box
  double rbound = 0.0;  // largest distance from org of any point of any primitive
  SceneDev dev{};
};

static int32_t g_scene_key = 0;
static std::mutex g_mu;

static void free_scene_arrays(tr_scene *s) {
  void *ptrs[] = {s->sph64, s->cylA64, s->cylW64, s->cylB64, s->sph32,       s->cylA32,
                  s->cylW32, s->albedo, s->cell_begin, s->refs, s->count, s->scan_scratch,
                  s->bounds_scratch, s->bounds, s->cellinfo, s->dist0, s->dist1, s->wrefs,
                  s->triA64, s->triB64, s->triC64, s->triV32, s->triE1_32, s->triE2_32,
                  s->bvh_nodes, s->total64};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (s->h_bounds) (void)hipHostFree(s->h_bounds);
  if (s->h_total) (void)hipHostFree(s->h_total);
}

template <class T>
static hipError_t dmalloc(T **p, int64_t n) {
  if (n <= 0) n = 1;
  return hipMalloc((void **)p, (size_t)n * sizeof(T));
}

// Grid parameters from the scene bounds (same definition as documented in
// the grid build: widened box, cube-root resolution rule, margins).
static void grid_params(const double lo_in[3], const double hi_in[3], int64_t N, double lambda,
                        trh::GridParams &g) {
  double m = 0.0;
  for (int a = 0; a < 3; ++a)
    if (hi_in[a] - lo_in[a] > m) m = hi_in[a] - lo_in[a];
  const double pad = 1e-4 * m + 1e-6;
  double ext[3];
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = lo_in[a] - pad;
    g.hi[a] = hi_in[a] + pad;
    ext[a] = g.hi[a] - g.lo[a];
  }
  double mext = ext[0];
  if (ext[1] > mext) mext = ext[1];
  if (ext[2] > mext) mext = ext[2];
  const double V = ext[0] * ext[1] * ext[2];
  const double kk = std::cbrt((lambda * (double)N) / V);
  double hmin = INFINITY;
  for (int a = 0; a < 3; ++a) {
    double r = std::ceil(ext[a] * kk);
    if (!(r >= 1.0)) r = 1.0;
    if (r > 512.0) r = 512.0;
    g.res[a] = (int32_t)r;
    g.h[a] = ext[a] / (double)g.res[a];
    g.inv[a] = (double)g.res[a] / ext[a];
    if (g.h[a] < hmin) hmin = g.h[a];
  }
  g.delta = hmin / 1024.0 + mext / 65536.0;
  g.n_cells = (int64_t)g.res[0] * g.res[1] * g.res[2];
}

static void fill_scene_dev(tr_scene *s) {
  SceneDev &d = s->dev;
  d.n_s = (int32_t)s->n_s;
  d.n_c = (int32_t)s->n_c;
  d.n_t = (int32_t)s->n_t;
  d.triA64 = s->triA64;
  d.triB64 = s->triB64;
  d.triC64 = s->triC64;
  d.triV32 = s->triV32;
  d.triE1_32 = s->triE1_32;
  d.triE2_32 = s->triE2_32;
  d.bvh = s->bvh_nodes;
  d.bvh_n = (int32_t)s->bvh_n;
  d.bvh_depth = s->bvh_depth;
  d.sph64 = s->sph64;
  d.cylA64 = s->cylA64;
  d.cylW64 = s->cylW64;
  d.sph32 = s->sph32;
  d.cylA32 = s->cylA32;
  d.cylW32 = s->cylW32;
  d.albedo = s->albedo;
  d.cell_begin = s->cell_begin;
  d.refs = s->refs;
  d.wrefs = s->wrefs;
  d.cellinfo = s->cellinfo;
  for (int a = 0; a < 3; ++a) {
    d.lo[a] = s->gp.lo[a];
    d.hi[a] = s->gp.hi[a];
    d.h[a] = s->gp.h[a];
    d.inv[a] = s->gp.inv[a];
    // FP32 frame: positions relative to the box centre org (the FP32
    // primitive copies, the FP32 eye and every FP32 point of the walk)
    d.org[a] = s->org[a];
    d.lo32[a] = (float)(s->gp.lo[a] - s->org[a]);
    d.hi32[a] = (float)(s->gp.hi[a] - s->org[a]);
    d.org32[a] = (float)((s->org[a] - s->gp.lo[a]) * s->gp.inv[a]);  // cell coordinate of 0
    d.h32[a] = (float)s->gp.h[a];
    d.inv32[a] = (float)s->gp.inv[a];
    d.res[a] = s->gp.res[a];
  }
  // the bounding sphere, padded by 2^-10 and rounded up (squares in FP64)
  const double rp = s->rbound * (1.0 + 0x1p-10);
  d.rb2_32 = std::nextafter((float)(rp * rp), INFINITY);
  d.rguard2_32 = (float)(rp * rp * 0x1p20);
}

// Bounds -> parameters -> count -> scan -> scatter -> sort, from the resident
// FP64 arrays.  Two blocking readbacks (bounds, reference total).
static tr_status build_grid_impl(tr_scene *s, hipStream_t st) {
  const int64_t N = s->n_s + s->n_c + s->n_t;
  trh::BuildArgs a{};
  a.n_s = (int32_t)s->n_s;
  a.n_c = (int32_t)s->n_c;
  a.n_t = (int32_t)s->n_t;
  a.sph64 = s->sph64;
  a.cylA64 = s->cylA64;
  a.cylB64 = s->cylB64;
  a.triA64 = s->triA64;
  a.triB64 = s->triB64;
  a.triC64 = s->triC64;
  if (N == 0) {
    double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
    for (int a = 0; a < 3; ++a) {
      s->gp.lo[a] = lo[a];
      s->gp.hi[a] = hi[a];
      s->gp.h[a] = 1.0;
      s->gp.inv[a] = 1.0;
      s->gp.res[a] = 1;
    }
    s->gp.delta = 0.0;
    s->gp.n_cells = 1;
  } else {
    HIP_TRY(trh::launch_bounds(a, s->bounds_scratch, s->bounds, st));
    HIP_TRY(hipMemcpyAsync(s->h_bounds, s->bounds, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    grid_params(s->h_bounds, s->h_bounds + 3, N, s->lambda, s->gp);
  }
  for (int a = 0; a < 3; ++a) s->org[a] = 0.5 * (s->gp.lo[a] + s->gp.hi[a]);
  // reference total and bounding radius, both read back after the count pass
  HIP_TRY(trh::launch_fill_u32((uint32_t *)s->total64, 4, 0u, st));
  HIP_TRY(trh::launch_pack32(a, s->cylW64, s->org, s->sph32, s->cylA32, s->cylW32, s->triV32,
                             s->triE1_32, s->triE2_32, s->total64 + 1, st));
  const int64_t nc = s->gp.n_cells;
  if (nc + 1 > s->cap_cells) {
    if (s->cell_begin) (void)hipFree(s->cell_begin);
    if (s->count) (void)hipFree(s->count);
    if (s->cellinfo) (void)hipFree(s->cellinfo);
    if (s->dist0) (void)hipFree(s->dist0);
    if (s->dist1) (void)hipFree(s->dist1);
    s->cell_begin = s->count = nullptr;
    s->cellinfo = nullptr;
    s->dist0 = s->dist1 = nullptr;
    HIP_TRY(dmalloc(&s->cell_begin, nc + 1));
    HIP_TRY(dmalloc(&s->count, nc + 1));
    HIP_TRY(dmalloc(&s->cellinfo, nc + 1));
    HIP_TRY(dmalloc(&s->dist0, nc + 1));
    HIP_TRY(dmalloc(&s->dist1, nc + 1));
    s->cap_cells = nc + 1;
  }
  const int64_t need_scan = trh::scan_scratch_u32(nc + 1);
  if (need_scan > s->cap_scan) {
    if (s->scan_scratch) (void)hipFree(s->scan_scratch);
    s->scan_scratch = nullptr;
    HIP_TRY(dmalloc(&s->scan_scratch, need_scan));
    s->cap_scan = need_scan;
  }
  for (int q = 0; q < 3; ++q) {
    a.lo[q] = s->gp.lo[q];
    a.h[q] = s->gp.h[q];
    a.inv[q] = s->gp.inv[q];
    a.res[q] = s->gp.res[q];
  }
  a.delta = s->gp.delta;
  HIP_TRY(trh::launch_fill_u32(s->cell_begin, nc + 1, 0u, st));
  HIP_TRY(trh::launch_count(a, s->cell_begin, s->total64, st));
  HIP_TRY(hipMemcpyAsync(s->h_total, s->total64, 2 * sizeof(*s->h_total), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  // The total is summed in 64 bits: overlapping large primitives can list
  // more than 2^32 references, which the 32-bit scan would wrap.  Walk lists
  // (references plus one end marker per occupied cell) are addressed with
  // signed 32-bit byte offsets by the traversal, so the limit is checked
  // before the scan and the scatter run.
  const unsigned long long R64 = s->h_total[0];
  std::memcpy(&s->rbound, s->h_total + 1, sizeof(double));  // (0 for an empty scene)
  if (R64 + (unsigned long long)nc + 1ull > (1ull << 29))
    return fail(TR_EUNSUPPORTED,
                "grid has %llu references and %lld cells (limit 2^29 together); lower cells_per_prim",
                R64, (long long)nc);
  const int64_t R = (int64_t)R64;
  const int64_t W = R + nc + 1;  // bound on the walk-list total
  HIP_TRY(trh::launch_scan(s->cell_begin, nc + 1, s->scan_scratch, st));
  if (R > s->cap_refs) {
    if (s->refs) (void)hipFree(s->refs);
    s->refs = nullptr;
    HIP_TRY(dmalloc(&s->refs, R));
    s->cap_refs = R;
  }
  if (W > s->cap_wrefs) {
    if (s->wrefs) (void)hipFree(s->wrefs);
    s->wrefs = nullptr;
    HIP_TRY(dmalloc(&s->wrefs, W));
    s->cap_wrefs = W;
  }
  s->n_refs = R;
  HIP_TRY(trh::launch_fill_u32(s->count, nc, 0u, st));
  HIP_TRY(trh::launch_scatter(a, s->cell_begin, s->count, s->refs, st));
  HIP_TRY(trh::launch_sort_cells(s->cell_begin, nc, s->refs, st));
  HIP_TRY(trh::launch_cellinfo(s->cell_begin, s->refs, s->gp.res, s->max_skip, s->dist0, s->dist1,
                               s->count, s->scan_scratch, s->wrefs, s->cellinfo, st));
  fill_scene_dev(s);
  return TR_OK;
}

static tr_status build_grid(tr_scene *s, hipStream_t st) {
  s->grid_ok = false;
  const tr_status rc = build_grid_impl(s, st);
  s->grid_ok = rc == TR_OK;
  return rc;
}

extern "C" tr_status tr_scene_build(const tr_scene_desc *d, void *hip_stream, tr_scene **out) {
  if (!d || !out) return fail(TR_EINVAL, "tr_scene_build: NULL desc or out");
  *out = nullptr;
  if (d->n_spheres < 0 || d->n_cylinders < 0 || d->n_triangles < 0)
    return fail(TR_EINVAL, "negative primitive count");
  const int64_t n_all = d->n_spheres + d->n_cylinders + d->n_triangles;
  // the traversal names a primitive by its record offset, 16 x its id (the
  // byte offset of its 16-byte FP32 records), in a signed 32-bit word
  if (n_all >= (int64_t)1 << 27) return fail(TR_EINVAL, "too many primitives (limit 2^27 - 1)");
  if (d->n_lights < 0 || d->n_lights > 8) return fail(TR_EINVAL, "n_lights must be 0..8");
  if (!(d->cells_per_prim >= 0.0) || !std::isfinite(d->cells_per_prim))
    return fail(TR_EINVAL, "cells_per_prim must be finite and >= 0");
  if (d->max_skip < 0 || d->max_skip > 32) return fail(TR_EINVAL, "max_skip must be 0..32");
  if (d->n_spheres > 0 && (!d->sph_center || !d->sph_radius || !d->sph_rgb))
    return fail(TR_EINVAL, "NULL sphere array");
  if (d->n_cylinders > 0 && (!d->cyl_a || !d->cyl_b || !d->cyl_radius || !d->cyl_rgb))
    return fail(TR_EINVAL, "NULL cylinder array");
  if (d->n_lights > 0 && (!d->light_dir || !d->light_rgb)) return fail(TR_EINVAL, "NULL light array");
  if (d->n_triangles > 0 && (!d->tri_v0 || !d->tri_v1 || !d->tri_v2 || !d->tri_rgb))
    return fail(TR_EINVAL, "NULL triangle array");
  for (int64_t k = 0; k < d->n_triangles; ++k)
    if (!finite3(d->tri_v0 + 3 * k) || !finite3(d->tri_v1 + 3 * k) || !finite3(d->tri_v2 + 3 * k))
      return fail(TR_EINVAL, "triangle %lld: non-finite vertex", (long long)k);
  for (int64_t k = 0; k < d->n_spheres; ++k) {
    if (!finite3(d->sph_center + 3 * k) || !std::isfinite(d->sph_radius[k]))
      return fail(TR_EINVAL, "sphere %lld: non-finite value", (long long)k);
    if (!(d->sph_radius[k] > 0.0)) return fail(TR_EINVAL, "sphere %lld: radius <= 0", (long long)k);
  }
  for (int64_t k = 0; k < d->n_cylinders; ++k) {
    const double *a = d->cyl_a + 3 * k, *b = d->cyl_b + 3 * k;
    if (!finite3(a) || !finite3(b) || !std::isfinite(d->cyl_radius[k]))
      return fail(TR_EINVAL, "cylinder %lld: non-finite value", (long long)k);
    if (!(d->cyl_radius[k] > 0.0)) return fail(TR_EINVAL, "cylinder %lld: radius <= 0", (long long)k);
    if (a[0] == b[0] && a[1] == b[1] && a[2] == b[2])
      return fail(TR_EINVAL, "cylinder %lld: zero length", (long long)k);
  }
  bool has_trans = false;
  for (int64_t k = 0; k < n_all; ++k) {
    const int64_t nsc = d->n_spheres + d->n_cylinders;
    const float *op = k < d->n_spheres ? d->sph_opacity : (k < nsc ? d->cyl_opacity : d->tri_opacity);
    if (!op) continue;
    const float a = op[k < d->n_spheres ? k : (k < nsc ? k - d->n_spheres : k - nsc)];
    if (!(a > 0.0f && a <= 1.0f))
      return fail(TR_EINVAL, "primitive %lld: opacity must be in (0, 1]", (long long)k);
    has_trans |= a < 1.0f;
  }
  for (int l = 0; l < d->n_lights; ++l) {
    const double *v = d->light_dir + 3 * l;
    if (!finite3(v) || !finite3(d->light_rgb + 3 * l)) return fail(TR_EINVAL, "light %d: non-finite", l);
    if (v[0] == 0.0 && v[1] == 0.0 && v[2] == 0.0) return fail(TR_EINVAL, "light %d: zero direction", l);
  }
  hipStream_t st = (hipStream_t)hip_stream;
  tr_scene *s = new tr_scene();
  (void)hipGetDevice(&s->device);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    s->key = ++g_scene_key;
  }
  s->n_s = d->n_spheres;
  s->n_c = d->n_cylinders;
  s->n_t = d->n_triangles;
  s->n_lights = d->n_lights;
  s->has_trans = has_trans;
  s->lambda = d->cells_per_prim > 0.0 ? d->cells_per_prim : 24.0;
  s->max_skip = d->max_skip > 0 ? d->max_skip : 32;
  for (int l = 0; l < d->n_lights; ++l) {
    const double *v = d->light_dir + 3 * l;
    for (int a = 0; a < 3; ++a) s->ldir_in[l][a] = v[a];
    const double n = std::sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    for (int a = 0; a < 3; ++a) {
      s->ldir[l][a] = v[a] / n;
      s->lrgb[l][a] = d->light_rgb[3 * l + a];
    }
  }
  auto bail = [&](tr_status stt) {
    std::string msg = g_err;
    free_scene_arrays(s);
    delete s;
    g_err = msg;
    return stt;
  };
  const int64_t N = s->n_s + s->n_c + s->n_t;
  hipError_t e = hipSuccess;
#define ALLOC(p, n)                                                      \
  if (e == hipSuccess) e = dmalloc(&(p), (n));
  ALLOC(s->sph64, s->n_s);
  ALLOC(s->sph32, s->n_s + s->n_c);  // spheres, then the cylinders' bounding spheres
  ALLOC(s->cylA64, s->n_c);
  ALLOC(s->cylW64, s->n_c);
  ALLOC(s->cylB64, s->n_c);
  ALLOC(s->cylA32, s->n_c);
  ALLOC(s->cylW32, s->n_c);
  ALLOC(s->albedo, N);
  ALLOC(s->triA64, s->n_t);
  ALLOC(s->triB64, s->n_t);
  ALLOC(s->triC64, s->n_t);
  ALLOC(s->triV32, s->n_t);
  ALLOC(s->triE1_32, s->n_t);
  ALLOC(s->triE2_32, s->n_t);
  ALLOC(s->bounds_scratch, trh::bounds_scratch_doubles(N));
  ALLOC(s->bounds, 6);
  ALLOC(s->total64, 2);
#undef ALLOC
  if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_bounds, 6 * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_total, 2 * sizeof(*s->h_total), hipHostMallocDefault);
  if (e != hipSuccess)
    return bail(fail(e == hipErrorOutOfMemory ? TR_ENOMEM : TR_EDEVICE, "scene allocation: %s",
                     hipGetErrorString(e)));
  s->bytes_arrays = (size_t)s->n_s * (32 + 16) + (size_t)s->n_c * (3 * 32 + 3 * 16) +
                    (size_t)s->n_t * (3 * 32 + 3 * 16) + (size_t)N * 16;
  // upload the caller's arrays (temporary device copies), then pack
  double *t_sc = nullptr, *t_sr = nullptr, *t_ca = nullptr, *t_cb = nullptr, *t_cr = nullptr;
  float *t_srgb = nullptr, *t_crgb = nullptr, *t_sop = nullptr, *t_cop = nullptr;
  double *t_tv0 = nullptr, *t_tv1 = nullptr, *t_tv2 = nullptr;
  float *t_trgb = nullptr, *t_top = nullptr;
  auto free_tmp = [&]() {
    void *p[] = {t_sc, t_sr, t_ca, t_cb, t_cr, t_srgb, t_crgb, t_sop, t_cop,
                 t_tv0, t_tv1, t_tv2, t_trgb, t_top};
    for (void *q : p)
      if (q) (void)hipFree(q);
  };
  if (N > 0) {
    e = hipSuccess;
    if (s->n_s > 0) {
      if (e == hipSuccess) e = dmalloc(&t_sc, 3 * s->n_s);
      if (e == hipSuccess) e = dmalloc(&t_sr, s->n_s);
      if (e == hipSuccess) e = dmalloc(&t_srgb, 3 * s->n_s);
      if (e == hipSuccess) e = hipMemcpyAsync(t_sc, d->sph_center, 24 * s->n_s, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(t_sr, d->sph_radius, 8 * s->n_s, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(t_srgb, d->sph_rgb, 12 * s->n_s, hipMemcpyHostToDevice, st);
      if (d->sph_opacity) {
        if (e == hipSuccess) e = dmalloc(&t_sop, s->n_s);
        if (e == hipSuccess) e = hipMemcpyAsync(t_sop, d->sph_opacity, 4 * s->n_s, hipMemcpyHostToDevice, st);
      }
    }
    if (s->n_c > 0) {
      if (e == hipSuccess) e = dmalloc(&t_ca, 3 * s->n_c);
      if (e == hipSuccess) e = dmalloc(&t_cb, 3 * s->n_c);
      if (e == hipSuccess) e = dmalloc(&t_cr, s->n_c);
      if (e == hipSuccess) e = dmalloc(&t_crgb, 3 * s->n_c);
      if (e == hipSuccess) e = hipMemcpyAsync(t_ca, d->cyl_a, 24 * s->n_c, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(t_cb, d->cyl_b, 24 * s->n_c, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(t_cr, d->cyl_radius, 8 * s->n_c, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(t_crgb, d->cyl_rgb, 12 * s->n_c, hipMemcpyHostToDevice, st);
      if (d->cyl_opacity) {
        if (e == hipSuccess) e = dmalloc(&t_cop, s->n_c);
        if (e == hipSuccess) e = hipMemcpyAsync(t_cop, d->cyl_opacity, 4 * s->n_c, hipMemcpyHostToDevice, st);
      }
    }
    if (s->n_t > 0) {
      const int64_t nt = s->n_t;
      if (e == hipSuccess) e = dmalloc(&t_tv0, 3 * nt);
      if (e == hipSuccess) e = dmalloc(&t_tv1, 3 * nt);
      if (e == hipSuccess) e = dmalloc(&t_tv2, 3 * nt);
      if (e == hipSuccess) e = dmalloc(&t_trgb, 3 * nt);
      if (e == hipSuccess) e = hipMemcpyAsync(t_tv0, d->tri_v0, 24 * nt, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(t_tv1, d->tri_v1, 24 * nt, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(t_tv2, d->tri_v2, 24 * nt, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(t_trgb, d->tri_rgb, 12 * nt, hipMemcpyHostToDevice, st);
      if (d->tri_opacity) {
        if (e == hipSuccess) e = dmalloc(&t_top, nt);
        if (e == hipSuccess) e = hipMemcpyAsync(t_top, d->tri_opacity, 4 * nt, hipMemcpyHostToDevice, st);
      }
    }
    trh::PackArgs pk{};
    pk.n_s = s->n_s;
    pk.n_c = s->n_c;
    pk.n_t = s->n_t;
    pk.sc = t_sc;
    pk.sr = t_sr;
    pk.ca = t_ca;
    pk.cb = t_cb;
    pk.cr = t_cr;
    pk.tv0 = t_tv0;
    pk.tv1 = t_tv1;
    pk.tv2 = t_tv2;
    pk.srgb = t_srgb;
    pk.sop = t_sop;
    pk.crgb = t_crgb;
    pk.cop = t_cop;
    pk.trgb = t_trgb;
    pk.top = t_top;
    pk.sph64 = s->sph64;
    pk.cylA64 = s->cylA64;
    pk.cylW64 = s->cylW64;
    pk.cylB64 = s->cylB64;
    pk.triA64 = s->triA64;
    pk.triB64 = s->triB64;
    pk.triC64 = s->triC64;
    pk.albedo = s->albedo;
    if (e == hipSuccess) e = trh::launch_pack(pk, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    free_tmp();
    if (e != hipSuccess)
      return bail(fail(e == hipErrorOutOfMemory ? TR_ENOMEM : TR_EDEVICE, "scene upload: %s",
                       hipGetErrorString(e)));
  }
  tr_status rc = build_grid(s, st);
  if (rc != TR_OK) return bail(rc);
  *out = s;
  return TR_OK;
}

extern "C" tr_status tr_scene_rebuild(tr_scene *s, double cells_per_prim, void *hip_stream) {
  if (!s) return fail(TR_EINVAL, "tr_scene_rebuild: NULL scene");
  if (!(cells_per_prim >= 0.0) || !std::isfinite(cells_per_prim))
    return fail(TR_EINVAL, "cells_per_prim must be finite and >= 0");
  if (cells_per_prim > 0.0) s->lambda = cells_per_prim;
  return build_grid(s, (hipStream_t)hip_stream);
}

// Linear BVH over the resident primitives, for the BVH walk (tr_tune.accel).
// Needs the grid's box and margins, so a scene whose grid failed cannot build one.
extern "C" tr_status tr_scene_build_bvh(tr_scene *s, void *hip_stream) {
  if (!s) return fail(TR_EINVAL, "tr_scene_build_bvh: NULL scene");
  if (!s->grid_ok) return fail(TR_EINVAL, "scene grid is invalid (its last rebuild failed)");
  const int64_t n = s->n_s + s->n_c + s->n_t;
  // node records are addressed with 32-bit byte offsets (64 bytes per node)
  if (n >= ((int64_t)1 << 26)) return fail(TR_EUNSUPPORTED, "BVH needs fewer than 2^26 primitives");
  hipStream_t st = (hipStream_t)hip_stream;
  // renders on any stream may still read the old records
  if (s->bvh_nodes) HIP_TRY(hipDeviceSynchronize());
  s->bvh_n = 0;
  s->bvh_depth = 0;
  const int64_t n_nodes = n >= 2 ? n - 1 : 0;
  if (s->bvh_nodes && s->bvh_cap != n_nodes) {
    HIP_TRY(hipFree(s->bvh_nodes));
    s->bvh_nodes = nullptr;
    s->bvh_cap = 0;
  }
  int32_t depth = 0;
  if (n >= 2) {
    if (!s->bvh_nodes) {
      HIP_TRY(dmalloc(&s->bvh_nodes, 4 * n_nodes));
      s->bvh_cap = n_nodes;
    }
    // all scratch in one allocation, each array 256-byte aligned
    trh::BvhScratch w{};
    size_t total = 0;
    auto carve = [&](size_t bytes) {
      const size_t at = total;
      total += (bytes + 255) & ~(size_t)255;
      return at;
    };
    const size_t o_keys = carve(4 * n), o_vals = carve(4 * n), o_keys2 = carve(4 * n),
                 o_vals2 = carve(4 * n), o_pl = carve(4 * n),
                 o_flags = carve(4 * (size_t)trh::bvh_sort_counts(n)),
                 o_left = carve(4 * n_nodes), o_right = carve(4 * n_nodes),
                 o_pi = carve(4 * n_nodes), o_arr = carve(4 * n_nodes), o_h = carve(4 * n_nodes),
                 o_ibox = carve(48 * n_nodes),
                 o_scan = carve(4 * (size_t)trh::scan_scratch_u32(trh::bvh_sort_counts(n)));
    char *base = nullptr;
    hipError_t e = hipMalloc((void **)&base, total);
    if (e == hipSuccess) {
      w.keys = (uint32_t *)(base + o_keys);
      w.vals = (uint32_t *)(base + o_vals);
      w.keys2 = (uint32_t *)(base + o_keys2);
      w.vals2 = (uint32_t *)(base + o_vals2);
      w.parent_l = (int32_t *)(base + o_pl);
      w.flags = (uint32_t *)(base + o_flags);
      w.left = (int32_t *)(base + o_left);
      w.right = (int32_t *)(base + o_right);
      w.parent_i = (int32_t *)(base + o_pi);
      w.arrivals = (uint32_t *)(base + o_arr);
      w.height = (int32_t *)(base + o_h);
      w.ibox = (double *)(base + o_ibox);
      w.scan_scratch = (uint32_t *)(base + o_scan);
    }
    trh::BuildArgs a{};
    a.n_s = (int32_t)s->n_s;
    a.n_c = (int32_t)s->n_c;
    a.n_t = (int32_t)s->n_t;
    a.sph64 = s->sph64;
    a.cylA64 = s->cylA64;
    a.cylB64 = s->cylB64;
    a.triA64 = s->triA64;
    a.triB64 = s->triB64;
    a.triC64 = s->triC64;
    // hierarchy and node depths, then the boxes level by level (the host
    // reads the largest depth in between), then the records
    int32_t max_dep = -1;
    if (e == hipSuccess) e = trh::launch_bvh_tree(a, s->gp.lo, s->gp.hi, w, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s->h_total, w.flags, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) std::memcpy(&max_dep, s->h_total, sizeof(int32_t));
    if (e == hipSuccess && (max_dep < 0 || max_dep > 63)) e = hipErrorUnknown;  // cannot happen
    if (e == hipSuccess)
      e = trh::launch_bvh_boxes(a, w, max_dep, s->gp.delta, s->org, s->bvh_nodes, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    depth = max_dep + 1;  // internal nodes on the longest root-to-leaf path
    if (base) (void)hipFree(base);
    if (e != hipSuccess) {
      (void)hipFree(s->bvh_nodes);
      s->bvh_nodes = nullptr;
      s->bvh_cap = 0;
      return fail(e == hipErrorOutOfMemory ? TR_ENOMEM : TR_EDEVICE, "BVH build: %s", hipGetErrorString(e));
    }
  }
  s->bvh_n = n;
  s->bvh_depth = depth;
  fill_scene_dev(s);
  return TR_OK;
}

extern "C" tr_status tr_scene_bvh_nodes(const tr_scene *s, float *nodes, int64_t *n_nodes,
                                        int32_t *depth, void *hip_stream) {
  if (!s || !n_nodes) return fail(TR_EINVAL, "tr_scene_bvh_nodes: NULL scene or n_nodes");
  *n_nodes = s->bvh_n >= 2 ? s->bvh_n - 1 : 0;
  if (depth) *depth = s->bvh_n >= 2 ? s->bvh_depth : 0;
  if (nodes && *n_nodes > 0) {
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipMemcpyAsync(nodes, s->bvh_nodes, (size_t)*n_nodes * 64, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  return TR_OK;
}

extern "C" tr_status tr_scene_set_max_skip(tr_scene *s, int32_t max_skip, void *hip_stream) {
  if (!s) return fail(TR_EINVAL, "tr_scene_set_max_skip: NULL scene");
  if (max_skip < 0 || max_skip > 32) return fail(TR_EINVAL, "max_skip must be 0..32");
  s->max_skip = max_skip > 0 ? max_skip : 32;
  return build_grid(s, (hipStream_t)hip_stream);
}

extern "C" tr_status tr_scene_footprint(const tr_scene *s, size_t *bytes) {
  if (!s || !bytes) return fail(TR_EINVAL, "tr_scene_footprint: NULL argument");
  *bytes = s->bytes_arrays + (size_t)s->cap_cells * (8 + sizeof(trd::CellInfo) + 2) +
           (size_t)s->cap_refs * 4 + (size_t)s->cap_wrefs * 4 +
           (size_t)s->cap_scan * 4;
  return TR_OK;
}

extern "C" tr_status tr_scene_grid_info(const tr_scene *s, double lo[3], double hi[3],
                                        int32_t res[3], int64_t *n_refs) {
  if (!s) return fail(TR_EINVAL, "tr_scene_grid_info: NULL scene");
  for (int a = 0; a < 3; ++a) {
    if (lo) lo[a] = s->gp.lo[a];
    if (hi) hi[a] = s->gp.hi[a];
    if (res) res[a] = s->gp.res[a];
  }
  if (n_refs) *n_refs = s->n_refs;
  return TR_OK;
}

extern "C" tr_status tr_scene_grid_arrays(const tr_scene *s, uint32_t *cell_begin, uint32_t *refs,
                                          void *hip_stream) {
  if (!s) return fail(TR_EINVAL, "tr_scene_grid_arrays: NULL scene");
  hipStream_t st = (hipStream_t)hip_stream;
  if (cell_begin)
    HIP_TRY(hipMemcpyAsync(cell_begin, s->cell_begin, (size_t)(s->gp.n_cells + 1) * 4,
                           hipMemcpyDeviceToHost, st));
  if (refs && s->n_refs > 0)
    HIP_TRY(hipMemcpyAsync(refs, s->refs, (size_t)s->n_refs * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return TR_OK;
}

// ---------------------------------------------------------- scene files
// Binary scene file, little-endian (the "Parse" phase of Table 5 without a
// text format): char magic[8] = "TRSCENE1"; int64 n_spheres, n_cylinders;
// int32 n_lights, int32 flags; double cells_per_prim; then the arrays of
// tr_scene_desc in its order, each padded to 8 bytes: spheres, cylinders,
// lights; with flags bit 1 an int64 triangle count and the triangle arrays;
// with flags bit 0 the opacities (of the triangles too with bit 1).
static const char kSceneMagic[8] = {'T', 'R', 'S', 'C', 'E', 'N', 'E', '1'};

static int64_t pad8(int64_t b) { return (b + 7) & ~(int64_t)7; }

static constexpr int32_t kFileOpacity = 1;    // flags bit: opacity arrays follow
static constexpr int32_t kFileTriangles = 2;  // flags bit: triangle section follows

// bytes up to the end of the lights (where the triangle count sits)
static int64_t scene_file_head(int64_t ns, int64_t nc, int64_t nl) {
  return 40 + pad8(24 * ns) + pad8(8 * ns) + pad8(12 * ns) + pad8(24 * nc) + pad8(24 * nc) +
         pad8(8 * nc) + pad8(12 * nc) + 2 * pad8(24 * nl);
}

static int64_t scene_file_bytes(int64_t ns, int64_t nc, int64_t nl, int32_t flags, int64_t nt) {
  int64_t b = scene_file_head(ns, nc, nl);
  if (flags & kFileTriangles) b += 8 + 3 * pad8(24 * nt) + pad8(12 * nt);
  if (flags & kFileOpacity)
    b += pad8(4 * ns) + pad8(4 * nc) + ((flags & kFileTriangles) ? pad8(4 * nt) : 0);
  return b;
}

extern "C" tr_status tr_scene_save(const tr_scene *s, const char *path, void *hip_stream) {
  if (!s || !path) return fail(TR_EINVAL, "tr_scene_save: NULL scene or path");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t ns = s->n_s, nc = s->n_c, nt = s->n_t, nl = s->n_lights, N = ns + nc + nt;
  std::vector<double4> sph(ns), ca(nc), cb(nc), ta(nt), tb(nt), tc(nt);
  std::vector<float4> alb(N);
  if (nt) HIP_TRY(hipMemcpyAsync(ta.data(), s->triA64, nt * sizeof(double4), hipMemcpyDeviceToHost, st));
  if (nt) HIP_TRY(hipMemcpyAsync(tb.data(), s->triB64, nt * sizeof(double4), hipMemcpyDeviceToHost, st));
  if (nt) HIP_TRY(hipMemcpyAsync(tc.data(), s->triC64, nt * sizeof(double4), hipMemcpyDeviceToHost, st));
  if (ns) HIP_TRY(hipMemcpyAsync(sph.data(), s->sph64, ns * sizeof(double4), hipMemcpyDeviceToHost, st));
  if (nc) HIP_TRY(hipMemcpyAsync(ca.data(), s->cylA64, nc * sizeof(double4), hipMemcpyDeviceToHost, st));
  if (nc) HIP_TRY(hipMemcpyAsync(cb.data(), s->cylB64, nc * sizeof(double4), hipMemcpyDeviceToHost, st));
  if (N) HIP_TRY(hipMemcpyAsync(alb.data(), s->albedo, N * sizeof(float4), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int32_t flags = (s->has_trans ? kFileOpacity : 0) | (nt > 0 ? kFileTriangles : 0);
  std::vector<char> buf((size_t)scene_file_bytes(ns, nc, nl, flags, nt), 0);
  char *p = buf.data();
  std::memcpy(p, kSceneMagic, 8);
  std::memcpy(p + 8, &ns, 8);
  std::memcpy(p + 16, &nc, 8);
  const int32_t nl32 = (int32_t)nl;
  std::memcpy(p + 24, &nl32, 4);
  std::memcpy(p + 28, &flags, 4);
  std::memcpy(p + 32, &s->lambda, 8);
  int64_t o = 40;
  auto put_d = [&](int64_t n, auto get) {
    for (int64_t i = 0; i < n; ++i) {
      const double v = get(i);
      std::memcpy(p + o + 8 * i, &v, 8);
    }
    o += pad8(8 * n);
  };
  auto put_f = [&](int64_t n, auto get) {
    for (int64_t i = 0; i < n; ++i) {
      const float v = get(i);
      std::memcpy(p + o + 4 * i, &v, 4);
    }
    o += pad8(4 * n);
  };
  auto comp = [](const double4 &v, int64_t a) { return a == 0 ? v.x : (a == 1 ? v.y : v.z); };
  auto compf = [](const float4 &v, int64_t a) { return a == 0 ? v.x : (a == 1 ? v.y : v.z); };
  put_d(3 * ns, [&](int64_t i) { return comp(sph[i / 3], i % 3); });
  put_d(ns, [&](int64_t i) { return sph[i].w; });
  put_f(3 * ns, [&](int64_t i) { return compf(alb[i / 3], i % 3); });
  put_d(3 * nc, [&](int64_t i) { return comp(ca[i / 3], i % 3); });
  put_d(3 * nc, [&](int64_t i) { return comp(cb[i / 3], i % 3); });
  put_d(nc, [&](int64_t i) { return ca[i].w; });
  put_f(3 * nc, [&](int64_t i) { return compf(alb[ns + i / 3], i % 3); });
  put_d(3 * nl, [&](int64_t i) { return s->ldir_in[i / 3][i % 3]; });
  put_d(3 * nl, [&](int64_t i) { return s->lrgb[i / 3][i % 3]; });
  if (flags & kFileTriangles) {
    std::memcpy(p + o, &nt, 8);
    o += 8;
    put_d(3 * nt, [&](int64_t i) { return comp(ta[i / 3], i % 3); });
    put_d(3 * nt, [&](int64_t i) { return comp(tb[i / 3], i % 3); });
    put_d(3 * nt, [&](int64_t i) { return comp(tc[i / 3], i % 3); });
    put_f(3 * nt, [&](int64_t i) { return compf(alb[ns + nc + i / 3], i % 3); });
  }
  if (flags & kFileOpacity) {
    put_f(ns, [&](int64_t i) { return alb[i].w; });
    put_f(nc, [&](int64_t i) { return alb[ns + i].w; });
    if (flags & kFileTriangles) put_f(nt, [&](int64_t i) { return alb[ns + nc + i].w; });
  }
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(TR_EINVAL, "tr_scene_save: cannot open %s for writing", path);
  const size_t w = std::fwrite(buf.data(), 1, buf.size(), f);
  const int c = std::fclose(f);
  if (w != buf.size() || c != 0) return fail(TR_EINVAL, "tr_scene_save: write to %s failed", path);
  return TR_OK;
}

extern "C" tr_status tr_scene_load(const char *path, void *hip_stream, tr_scene **out) {
  if (!path || !out) return fail(TR_EINVAL, "tr_scene_load: NULL path or out");
  *out = nullptr;
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(TR_EINVAL, "tr_scene_load: cannot open %s", path);
  std::fseek(f, 0, SEEK_END);
  const long size = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  if (size < 40) {
    std::fclose(f);
    return fail(TR_EINVAL, "tr_scene_load: %s is not a scene file (too short)", path);
  }
  std::vector<double> store(((size_t)size + 7) / 8);  // 8-byte aligned
  char *p = (char *)store.data();
  const size_t r = std::fread(p, 1, (size_t)size, f);
  std::fclose(f);
  if (r != (size_t)size) return fail(TR_EINVAL, "tr_scene_load: read of %s failed", path);
  if (std::memcmp(p, kSceneMagic, 8) != 0)
    return fail(TR_EINVAL, "tr_scene_load: %s is not a scene file (bad magic)", path);
  int64_t ns, nc;
  int32_t nl, flags;
  double lambda;
  std::memcpy(&ns, p + 8, 8);
  std::memcpy(&nc, p + 16, 8);
  std::memcpy(&nl, p + 24, 4);
  std::memcpy(&flags, p + 28, 4);
  std::memcpy(&lambda, p + 32, 8);
  if (flags & ~(kFileOpacity | kFileTriangles))
    return fail(TR_EINVAL, "tr_scene_load: %s has unknown flags", path);
  if (ns < 0 || nc < 0 || ns >= ((int64_t)1 << 28) || nc >= ((int64_t)1 << 28) || nl < 0 || nl > 8)
    return fail(TR_EINVAL, "tr_scene_load: %s has bad counts", path);
  int64_t nt = 0;
  if (flags & kFileTriangles) {
    const int64_t at = scene_file_head(ns, nc, nl);
    if (at + 8 > (int64_t)size)
      return fail(TR_EINVAL, "tr_scene_load: %s has %ld bytes, its counts need more", path, size);
    std::memcpy(&nt, p + at, 8);
    if (nt < 0 || nt >= ((int64_t)1 << 28))
      return fail(TR_EINVAL, "tr_scene_load: %s has bad counts", path);
  }
  if (scene_file_bytes(ns, nc, nl, flags, nt) != (int64_t)size)
    return fail(TR_EINVAL, "tr_scene_load: %s has %ld bytes, its counts need %lld", path, size,
                (long long)scene_file_bytes(ns, nc, nl, flags, nt));
  int64_t o = 40;
  auto take = [&](int64_t bytes) {
    const char *q = p + o;
    o += pad8(bytes);
    return q;
  };
  tr_scene_desc d{};
  d.n_spheres = ns;
  d.sph_center = (const double *)take(24 * ns);
  d.sph_radius = (const double *)take(8 * ns);
  d.sph_rgb = (const float *)take(12 * ns);
  d.n_cylinders = nc;
  d.cyl_a = (const double *)take(24 * nc);
  d.cyl_b = (const double *)take(24 * nc);
  d.cyl_radius = (const double *)take(8 * nc);
  d.cyl_rgb = (const float *)take(12 * nc);
  d.n_lights = nl;
  d.light_dir = (const double *)take(24 * nl);
  d.light_rgb = (const double *)take(24 * nl);
  d.cells_per_prim = lambda;
  if (flags & kFileTriangles) {
    take(8);
    d.n_triangles = nt;
    d.tri_v0 = (const double *)take(24 * nt);
    d.tri_v1 = (const double *)take(24 * nt);
    d.tri_v2 = (const double *)take(24 * nt);
    d.tri_rgb = (const float *)take(12 * nt);
  }
  if (flags & kFileOpacity) {
    d.sph_opacity = (const float *)take(4 * ns);
    d.cyl_opacity = (const float *)take(4 * nc);
    if (flags & kFileTriangles) d.tri_opacity = (const float *)take(4 * nt);
  }
  return tr_scene_build(&d, hip_stream, out);
}

extern "C" tr_status tr_scene_walk_arrays(const tr_scene *s, int32_t *cellinfo, uint32_t *wrefs,
                                          int64_t *n_walk, void *hip_stream) {
  if (!s || !n_walk) return fail(TR_EINVAL, "tr_scene_walk_arrays: NULL scene or n_walk");
  if (!s->grid_ok) return fail(TR_EINVAL, "scene grid is invalid (its last rebuild failed)");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t nc = s->gp.n_cells;
  // the walk-list total is the last entry of the scanned sizes (kept in count)
  *s->h_total = 0ull;
  HIP_TRY(hipMemcpyAsync(s->h_total, s->count + nc, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  uint32_t n_w = 0;
  std::memcpy(&n_w, s->h_total, sizeof(n_w));
  *n_walk = (int64_t)n_w;
  if (cellinfo)
    HIP_TRY(hipMemcpyAsync(cellinfo, s->cellinfo, (size_t)nc * sizeof(trd::CellInfo),
                           hipMemcpyDeviceToHost, st));
  if (wrefs && *n_walk > 0)
    HIP_TRY(hipMemcpyAsync(wrefs, s->wrefs, (size_t)*n_walk * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return TR_OK;
}

extern "C" void tr_scene_destroy(tr_scene *s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  free_scene_arrays(s);
  delete s;
}

// ------------------------------------------------------------------- jobs
static bool valid_tile_w(int32_t w) { return w == 4 || w == 8 || w == 16 || w == 32 || w == 64; }

// Tiles of one 64-pixel row segment by default: a tile's frame write is one
// 768-byte run, so few cache lines are shared between tiles (finished at
// different times, a shared line tends to leave the L2 twice).
constexpr int32_t kDefaultTileW = 64;

static tr_status default_tune(tr_tune *t) {
  t->tile_w = kDefaultTileW;
  t->banks = 2;
  t->waves_per_cu = 20;
  t->refill_below = 32;
  t->count_ops = 0;
  t->accel = 0;
  t->stripe = 64;
  return TR_OK;
}

static tr_status check_tune(const tr_tune &t) {
  if (!valid_tile_w(t.tile_w)) return fail(TR_EINVAL, "tune.tile_w must be 4, 8, 16, 32 or 64");
  if (t.banks != 2 && t.banks != 3) return fail(TR_EINVAL, "tune.banks must be 2 or 3");
  if (t.waves_per_cu < 1 || t.waves_per_cu > 32) return fail(TR_EINVAL, "tune.waves_per_cu must be 1..32");
  if (t.refill_below < 1 || t.refill_below > 64) return fail(TR_EINVAL, "tune.refill_below must be 1..64");
  if (t.accel != 0 && t.accel != 1) return fail(TR_EINVAL, "tune.accel must be 0 or 1");
  if (t.stripe < 1 || t.stripe > 1024 || (t.stripe & (t.stripe - 1)))
    return fail(TR_EINVAL, "tune.stripe must be a power of two 1..1024");
  return TR_OK;
}

static tr_status check_camera(const tr_camera *c) {
  if (!c) return fail(TR_EINVAL, "NULL camera");
  if (c->width <= 0 || c->height <= 0) return fail(TR_EINVAL, "width and height must be > 0");
  if ((int64_t)c->width * c->height > (int64_t)INT32_MAX - 1)
    return fail(TR_EINVAL, "width*height must be < 2^31");
  if (!finite3(c->eye) || !finite3(c->lookat) || !finite3(c->up) || !std::isfinite(c->fovy_deg))
    return fail(TR_EINVAL, "non-finite camera");
  if (!(c->fovy_deg > 0.0 && c->fovy_deg < 180.0)) return fail(TR_EINVAL, "fovy must be in (0, 180)");
  return TR_OK;
}

static constexpr int32_t kMaxAASamples = 256;
static constexpr int32_t kMaxLayers = 64;
static int32_t aa_count(const tr_params &p) { return p.aa_samples > 1 ? p.aa_samples : 1; }

static tr_status check_params(const tr_params *p, const tr_frame *f) {
  if (!p) return fail(TR_EINVAL, "NULL params");
  if (!f || !f->rgb) return fail(TR_EINVAL, "NULL frame or frame->rgb");
  if (p->ao_samples < 0 || p->ao_samples > 65535) return fail(TR_EINVAL, "ao_samples must be 0..65535");
  if (!(p->ao_maxdist > 0.0)) return fail(TR_EINVAL, "ao_maxdist must be > 0");
  if (f->ao_mask && p->ao_samples > 32) return fail(TR_EINVAL, "ao_mask needs ao_samples <= 32");
  if (p->aa_samples < 0 || p->aa_samples > kMaxAASamples)
    return fail(TR_EINVAL, "aa_samples must be 0..%d", kMaxAASamples);
  if (p->max_layers < 0 || p->max_layers > kMaxLayers)
    return fail(TR_EINVAL, "max_layers must be 0..%d", kMaxLayers);
  if (!(p->specular >= 0.0) || !std::isfinite(p->specular))
    return fail(TR_EINVAL, "specular must be finite and >= 0");
  if (p->specular > 0.0 && !(p->shininess > 0.0 && std::isfinite(p->shininess)))
    return fail(TR_EINVAL, "shininess must be finite and > 0 when specular > 0");
  if (p->precision < TR_PREC_FP64 || p->precision > TR_PREC_FP32_RESOLVE)
    return fail(TR_EINVAL, "unknown precision %d", p->precision);
  if (!std::isfinite(p->light_rescale) || !std::isfinite(p->skylight))
    return fail(TR_EINVAL, "non-finite light_rescale or skylight");
  return TR_OK;
}

static void cross3(const double a[3], const double b[3], double r[3]) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double a[3], const double b[3]) {
  return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

static tr_status make_job(const tr_scene *s, const tr_camera *c, const tr_params *p,
                          const tr_frame *f, int32_t tile_w, JobDev &J) {
  tr_status rc = check_camera(c);
  if (rc != TR_OK) return rc;
  rc = check_params(p, f);
  if (rc != TR_OK) return rc;
  if (!s) return fail(TR_EINVAL, "NULL scene");
  if (!s->grid_ok) return fail(TR_EINVAL, "scene grid is invalid (its last rebuild failed)");
  std::memset(&J, 0, sizeof J);
  J.sc = s->dev;
  double fw[3] = {c->lookat[0] - c->eye[0], c->lookat[1] - c->eye[1], c->lookat[2] - c->eye[2]};
  const double nf = std::sqrt(dot3(fw, fw));
  if (!(nf > 0.0)) return fail(TR_EINVAL, "eye == lookat");
  for (int a = 0; a < 3; ++a) J.f[a] = fw[a] / nf;
  double rr[3];
  cross3(J.f, c->up, rr);
  const double nr = std::sqrt(dot3(rr, rr));
  const double nu = std::sqrt(dot3(c->up, c->up));
  if (!(nr > 1e-12 * nu)) return fail(TR_EINVAL, "up is zero or parallel to the view direction");
  for (int a = 0; a < 3; ++a) J.r[a] = rr[a] / nr;
  cross3(J.r, J.f, J.u);
  J.th = std::tan((c->fovy_deg * M_PI) / 360.0);
  J.aspect = (double)c->width / (double)c->height;
  for (int a = 0; a < 3; ++a) {
    J.eye[a] = c->eye[a];
    J.eye32[a] = (float)(c->eye[a] - s->org[a]);  // FP32 frame (relative to the box centre)
    J.f32[a] = (float)J.f[a];
    J.r32[a] = (float)J.r[a];
    J.u32[a] = (float)J.u[a];
  }
  J.th32 = (float)J.th;
  J.aspect32 = (float)J.aspect;
  J.W = c->width;
  J.H = c->height;
  J.S = (p->ao_samples > 0 && p->skylight > 0.0) ? p->ao_samples : 0;
  J.n_lights = s->n_lights;
  for (int l = 0; l < s->n_lights; ++l)
    for (int a = 0; a < 3; ++a) {
      J.ldir[l][a] = s->ldir[l][a];
      J.lcol[l][a] = p->light_rescale * s->lrgb[l][a];
      J.ldir32[l][a] = (float)J.ldir[l][a];
      J.lcol32[l][a] = (float)J.lcol[l][a];
    }
  J.sky = p->skylight;
  J.sky32 = (float)p->skylight;
  J.ao_maxdist = p->ao_maxdist;
  J.ao_maxdist32 = (float)p->ao_maxdist;
  J.ks = p->specular;
  J.shin = p->specular > 0.0 ? p->shininess : 1.0;
  J.ks32 = (float)J.ks;
  J.shin32 = (float)J.shin;
  J.layers = (p->max_layers > 1 && s->has_trans) ? p->max_layers : 1;
  J.key0 = (uint32_t)(p->seed & 0xFFFFFFFFull);
  J.key1 = (uint32_t)(p->seed >> 32);
  J.view_id = p->view_id;
  J.resolve = p->precision == TR_PREC_FP32_RESOLVE;
  for (int a = 0; a < 3; ++a) J.bg[a] = p->background[a];
  J.rgb = f->rgb;
  J.hit_id = f->hit_id;
  J.ao_mask = f->ao_mask;
  J.light_mask = f->light_mask;
  J.tile_w = tile_w;
  J.tile_h = 64 / tile_w;
  J.tiles_x = (c->width + tile_w - 1) / tile_w;
  J.tiles_y = (c->height + J.tile_h - 1) / J.tile_h;
  J.tile_begin = 0;
  J.tile_end = (int64_t)J.tiles_x * J.tiles_y;
  J.scene_key = s->key;
  return TR_OK;
}

// ------------------------------------------------------ launch resources
// Per-stream ring of job tables: pinned staging + device table + tile
// counter, each slot reusable once the launch that used it has completed.
struct LaunchSlot {
  JobDev *h_jobs = nullptr;
  JobDev *d_jobs = nullptr;
  uint32_t *d_counter = nullptr;  // tile queue counters + stall flag (kQueueWords)
  int32_t cap = 0;
  hipEvent_t done = nullptr;
  bool used = false;
};
struct StreamRing {
  LaunchSlot slot[4];
  int next = 0;
};
static std::map<std::pair<int, hipStream_t>, StreamRing> g_rings;

static int g_num_cus = 0;

static int num_cus() {
  if (g_num_cus == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) g_num_cus = prop.multiProcessorCount;
    if (g_num_cus <= 0) g_num_cus = 256;
  }
  return g_num_cus;
}

static tr_status acquire_slot(hipStream_t st, int32_t n, LaunchSlot **out) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_mu);
  StreamRing &ring = g_rings[{dev, st}];
  LaunchSlot &ls = ring.slot[ring.next];
  ring.next = (ring.next + 1) % 4;
  if (ls.used) HIP_TRY(hipEventSynchronize(ls.done));
  if (!ls.done) HIP_TRY(hipEventCreateWithFlags(&ls.done, hipEventDisableTiming));
  if (ls.cap < n) {
    if (ls.h_jobs) (void)hipHostFree(ls.h_jobs);
    if (ls.d_jobs) (void)hipFree(ls.d_jobs);
    ls.h_jobs = nullptr;
    ls.d_jobs = nullptr;
    int32_t cap = std::max(n, 8);
    HIP_TRY(hipHostMalloc((void **)&ls.h_jobs, sizeof(JobDev) * cap, hipHostMallocDefault));
    HIP_TRY(hipMalloc((void **)&ls.d_jobs, sizeof(JobDev) * cap));
    ls.cap = cap;
  }
  if (!ls.d_counter) HIP_TRY(hipMalloc((void **)&ls.d_counter, trd::kQueueWords * sizeof(uint32_t)));
  ls.used = true;
  *out = &ls;
  return TR_OK;
}

// The tuned-shape cache.
struct TuneKey {
  int dev;
  int n_bucket;
  int32_t W, H, S, prec;
  bool operator<(const TuneKey &o) const {
    return std::tie(dev, n_bucket, W, H, S, prec) < std::tie(o.dev, o.n_bucket, o.W, o.H, o.S, o.prec);
  }
};
static std::map<TuneKey, tr_tune> g_tune_cache;

static TuneKey tune_key(const tr_scene *s, const tr_camera *c, const tr_params *p) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int64_t N = s->n_s + s->n_c + s->n_t;
  int b = 0;
  while ((int64_t(1) << b) < N + 1) ++b;
  return TuneKey{dev, b, c->width, c->height, p->ao_samples, p->precision};
}

static tr_tune pick_tune(const tr_scene *s, const tr_camera *c, const tr_params *p,
                         const tr_tune *explicit_tune) {
  tr_tune t;
  default_tune(&t);
  if (explicit_tune) {
    t = *explicit_tune;
    tr_tune d;
    default_tune(&d);
    if (!t.tile_w) t.tile_w = d.tile_w;
    if (!t.banks) t.banks = d.banks;
    if (!t.waves_per_cu) t.waves_per_cu = d.waves_per_cu;
    if (!t.refill_below) t.refill_below = d.refill_below;
    if (!t.stripe) t.stripe = d.stripe;
    return t;
  }
  if (s && c && p) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tune_cache.find(tune_key(s, c, p));
    if (it != g_tune_cache.end()) t = it->second;
  }
  return t;
}

// ---------------------------------------------------------- antialiasing
// A frame with A > 1 primary samples per pixel is A jobs: job 0 (the pixel
// centres) writes the caller's buffers, and sample a = 1..A-1 writes its
// colours into plane a - 1 of a per-stream workspace.  After the render,
// one pass per frame folds the planes into the caller's rgb, summing in
// sample order (deterministic), and divides by A.
struct AAWork {
  float *buf = nullptr;
  int64_t cap = 0;  // floats
};
static std::map<std::pair<int, hipStream_t>, AAWork> g_aa_work;

static tr_status aa_workspace(hipStream_t st, int64_t n_floats, float **out) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_mu);
  AAWork &w = g_aa_work[{dev, st}];
  if (w.cap < n_floats) {
    if (w.buf) {  // earlier work on this stream may still read the old planes
      HIP_TRY(hipStreamSynchronize(st));
      HIP_TRY(hipFree(w.buf));
      w.buf = nullptr;
      w.cap = 0;
    }
    HIP_TRY(hipMalloc((void **)&w.buf, (size_t)n_floats * sizeof(float)));
    w.cap = n_floats;
  }
  *out = w.buf;
  return TR_OK;
}

struct AAMean {
  float *rgb;
  const float *planes;
  int32_t n_planes;
  int64_t n;  // floats per plane (W * H * 3)
};

// Append the sample jobs 1..A-1 of jobs[i] (A = aa[i]) and list the folds.
static tr_status expand_aa(std::vector<JobDev> &jobs, const std::vector<int32_t> &aa,
                           hipStream_t st, std::vector<AAMean> &means) {
  int64_t total = 0;
  for (size_t i = 0; i < aa.size(); ++i)
    if (aa[i] > 1) total += (int64_t)(aa[i] - 1) * jobs[i].W * jobs[i].H * 3;
  if (total == 0) return TR_OK;
  float *ws = nullptr;
  tr_status rc = aa_workspace(st, total, &ws);
  if (rc != TR_OK) return rc;
  int64_t off = 0;
  const size_t n0 = aa.size();
  for (size_t i = 0; i < n0; ++i) {
    if (aa[i] <= 1) continue;
    const JobDev base = jobs[i];
    const int64_t plane = (int64_t)base.W * base.H * 3;
    means.push_back(AAMean{base.rgb, ws + off, aa[i] - 1, plane});
    for (int32_t a = 1; a < aa[i]; ++a) {
      JobDev J = base;
      J.aa = a;
      J.rgb = ws + off;
      J.hit_id = nullptr;
      J.ao_mask = nullptr;
      J.light_mask = nullptr;
      jobs.push_back(J);
      off += plane;
    }
  }
  return TR_OK;
}

static tr_status run_aa_means(const std::vector<AAMean> &means, hipStream_t st) {
  for (const AAMean &m : means)
    HIP_TRY(trh::launch_aa_mean(m.rgb, m.planes, m.n_planes, m.n, st));
  return TR_OK;
}

// What the wavefront kernel needs of a job under the tuning: with the BVH
// walk, a built BVH that its stack can hold, and opaque rendering.
static tr_status check_wave_job(const JobDev &J, const tr_tune &t) {
  if (!t.accel) return TR_OK;
  if (J.sc.bvh_n != (int64_t)J.sc.n_s + J.sc.n_c + J.sc.n_t)
    return fail(TR_EINVAL, "tune.accel = 1 needs tr_scene_build_bvh on every scene");
  if (J.layers > 1)
    return fail(TR_EUNSUPPORTED, "the BVH walk renders opaque frames (max_layers <= 1)");
  if (J.sc.bvh_depth > trh::kBvhStack)
    return fail(TR_EUNSUPPORTED, "BVH depth %d exceeds the walk's stack of %d entries",
                (int)J.sc.bvh_depth, trh::kBvhStack);
  return TR_OK;
}

// Queue positions of the jobs' tiles; the total tile count.
static int64_t set_queue(JobDev *jobs, int32_t n) {
  int64_t total = 0;
  for (int32_t i = 0; i < n; ++i) {
    jobs[i].queue_begin = total;
    total += jobs[i].tile_end - jobs[i].tile_begin;
  }
  return total;
}

// The launch of the wavefront kernel over n jobs (queue set) whose device
// table and tile counter are given.
static trh::WaveLaunch wave_launch(const JobDev *jobs, int32_t n, int64_t total, const tr_tune &t,
                                   uint64_t *stats, const JobDev *d_jobs, uint32_t *d_counter) {
  trh::WaveLaunch L{};
  L.jobs = d_jobs;
  L.n_jobs = n;
  L.n_tiles = total;
  L.tile_counter = d_counter;
  L.stats = stats;
  L.tile_w = t.tile_w;
  L.banks = t.banks;
  L.refill_below = t.refill_below;
  L.count_ops = t.count_ops;
  L.stripe = t.stripe;
  int64_t waves = (int64_t)num_cus() * t.waves_per_cu;
  if (waves > total) waves = total;
  L.n_waves = (int32_t)waves;
  L.resolve = jobs[0].resolve;
  L.trans = 0;
  L.tri = 0;
  for (int32_t i = 0; i < n; ++i) {
    L.trans |= jobs[i].layers > 1;
    L.tri |= jobs[i].sc.n_t > 0;
  }
  L.bvh = t.accel;
  return L;
}

// Launch the wavefront kernel over the jobs (already filled, tiles set).
static tr_status launch_wave_jobs(std::vector<JobDev> &jobs, const tr_tune &t, uint64_t *stats,
                                  hipStream_t st) {
  for (const JobDev &J : jobs) {
    const tr_status rc = check_wave_job(J, t);
    if (rc != TR_OK) return rc;
  }
  const int64_t total = set_queue(jobs.data(), (int32_t)jobs.size());
  if (total == 0) return TR_OK;
  if (total > (int64_t)UINT32_MAX - 1) return fail(TR_EINVAL, "too many tiles in one launch");
  LaunchSlot *ls = nullptr;
  tr_status rc = acquire_slot(st, (int32_t)jobs.size(), &ls);
  if (rc != TR_OK) return rc;
  std::memcpy(ls->h_jobs, jobs.data(), sizeof(JobDev) * jobs.size());
  HIP_TRY(hipMemcpyAsync(ls->d_jobs, ls->h_jobs, sizeof(JobDev) * jobs.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(trh::launch_fill_u32(ls->d_counter, trd::kQueueWords, 0u, st));
  const trh::WaveLaunch L = wave_launch(jobs.data(), (int32_t)jobs.size(), total, t, stats,
                                        ls->d_jobs, ls->d_counter);
  HIP_TRY(trh::launch_render_wave(L, st));
  HIP_TRY(hipEventRecord(ls->done, st));
  return TR_OK;
}

// --------------------------------------------------------------- renders
extern "C" tr_status tr_render_tuned(const tr_scene *s, const tr_camera *c, const tr_params *p,
                                     const tr_frame *f, const tr_tune *tune, void *hip_stream) {
  if (!s) return fail(TR_EINVAL, "tr_render: NULL scene");
  tr_tune t = pick_tune(s, c, p, tune);
  tr_status rc = check_tune(t);
  if (rc != TR_OK) return rc;
  JobDev J;
  rc = make_job(s, c, p, f, t.tile_w, J);
  if (rc == TR_OK && p->precision != TR_PREC_FP64) rc = check_wave_job(J, t);
  if (rc != TR_OK) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<JobDev> jobs(1, J);
  std::vector<AAMean> means;
  rc = expand_aa(jobs, std::vector<int32_t>(1, aa_count(*p)), st, means);
  if (rc != TR_OK) return rc;
  if (p->precision == TR_PREC_FP64) {
    for (const JobDev &Js : jobs) HIP_TRY(trh::launch_render_plain_f64(Js, f->stats, st));
  } else {
    rc = launch_wave_jobs(jobs, t, f->stats, st);
    if (rc != TR_OK) return rc;
  }
  return run_aa_means(means, st);
}

extern "C" tr_status tr_render(const tr_scene *s, const tr_camera *c, const tr_params *p,
                               const tr_frame *f, void *hip_stream) {
  return tr_render_tuned(s, c, p, f, nullptr, hip_stream);
}

extern "C" int64_t tr_tile_count(int32_t width, int32_t height, int32_t tile_w) {
  if (tile_w == 0) tile_w = kDefaultTileW;
  if (!valid_tile_w(tile_w) || width <= 0 || height <= 0) return -1;
  const int32_t th = 64 / tile_w;
  return (int64_t)((width + tile_w - 1) / tile_w) * ((height + th - 1) / th);
}

static tr_status batch_impl(int32_t n, const tr_scene *const *scenes, const tr_camera *cams,
                            const tr_params *params, const tr_frame *frames, const int64_t *tb,
                            const int64_t *te, const tr_tune *tune, hipStream_t st) {
  if (n < 1 || n > 4096) return fail(TR_EINVAL, "batch size must be 1..4096");
  if (!scenes || !cams || !params || !frames) return fail(TR_EINVAL, "NULL batch array");
  // the first FP32 job sets the batch's FP32 precision and its tuning
  int32_t f0 = 0;
  while (f0 < n - 1 && params[f0].precision == TR_PREC_FP64) ++f0;
  tr_tune t = pick_tune(scenes[f0], &cams[f0], &params[f0], tune);
  tr_status rc = check_tune(t);
  if (rc != TR_OK) return rc;
  const int res = params[f0].precision == TR_PREC_FP32_RESOLVE;
  std::vector<JobDev> jobs, f64;
  std::vector<int32_t> aa, aa64;
  std::vector<uint64_t *> stats64;
  jobs.reserve(n);
  uint64_t *stats = frames[f0].stats;  // shared by the FP32 jobs
  // every job is checked before anything is enqueued: a failing batch
  // renders nothing
  for (int32_t i = 0; i < n; ++i) {
    JobDev J;
    rc = make_job(scenes[i], &cams[i], &params[i], &frames[i], t.tile_w, J);
    if (rc != TR_OK) return fail(rc, "job %d: %s", i, g_err.c_str());
    if (tb && aa_count(params[i]) > 1) return fail(TR_EUNSUPPORTED, "tile ranges need aa_samples <= 1");
    if (params[i].precision == TR_PREC_FP64) {
      if (tb) return fail(TR_EUNSUPPORTED, "tile ranges need an FP32 precision");
      f64.push_back(J);
      aa64.push_back(aa_count(params[i]));
      stats64.push_back(frames[i].stats);
      continue;
    }
    if ((params[i].precision == TR_PREC_FP32_RESOLVE) != (res != 0))
      return fail(TR_EINVAL, "all FP32 jobs of one batch must use the same precision");
    if (frames[i].stats != stats) return fail(TR_EINVAL, "all jobs of one batch must share one stats buffer");
    if (tb) {
      if (!te) return fail(TR_EINVAL, "NULL tile_end");
      if (tb[i] < 0 || te[i] < tb[i] || te[i] > J.tile_end)
        return fail(TR_EINVAL, "job %d: tile range [%lld, %lld) outside [0, %lld)", i,
                    (long long)tb[i], (long long)te[i], (long long)J.tile_end);
      J.tile_begin = tb[i];
      J.tile_end = te[i];
    }
    rc = check_wave_job(J, t);
    if (rc != TR_OK) return fail(rc, "job %d: %s", i, g_err.c_str());
    jobs.push_back(J);
    aa.push_back(aa_count(params[i]));
  }
  {
    int64_t tiles = 0;
    for (size_t k = 0; k < jobs.size(); ++k) tiles += (jobs[k].tile_end - jobs[k].tile_begin) * aa[k];
    if (tiles > (int64_t)UINT32_MAX - 1) return fail(TR_EINVAL, "too many tiles in one launch");
  }
  for (size_t k = 0; k < f64.size(); ++k) {  // plain FP64 jobs: one launch each
    std::vector<JobDev> one(1, f64[k]);
    std::vector<AAMean> means;
    rc = expand_aa(one, std::vector<int32_t>(1, aa64[k]), st, means);
    if (rc != TR_OK) return rc;
    for (const JobDev &Js : one) HIP_TRY(trh::launch_render_plain_f64(Js, stats64[k], st));
    rc = run_aa_means(means, st);
    if (rc != TR_OK) return rc;
  }
  if (jobs.empty()) return TR_OK;
  std::vector<AAMean> means;
  rc = expand_aa(jobs, aa, st, means);
  if (rc != TR_OK) return rc;
  // keep jobs of one scene adjacent so waves rarely switch scenes
  std::stable_sort(jobs.begin(), jobs.end(),
                   [](const JobDev &a, const JobDev &b) { return a.scene_key < b.scene_key; });
  rc = launch_wave_jobs(jobs, t, stats, st);
  if (rc != TR_OK) return rc;
  return run_aa_means(means, st);
}

// ----------------------------------------------- allocation-free batches
// tr_render_batch_noalloc keeps its job table and tile counter in this
// array of the library's static device memory (each device holds its own
// copy until the process ends).  In host code `scratch` names a host-side
// stand-in: its device address is looked up once per device and used
// instead, everywhere.
struct NoAllocScratch {
  JobDev jobs[TR_NOALLOC_MAX_JOBS];
  uint32_t counter[trd::kQueueWords];  // tile queue counters, stall flag
};
static __device__ __align__(256) unsigned char scratch[sizeof(NoAllocScratch)];
constexpr int kMaxDevices = 64;
static NoAllocScratch *g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (looked up on the first
// call on each device, with that device current).
static tr_status scratch_on_device(NoAllocScratch **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(TR_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(TR_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch[dev] = (NoAllocScratch *)ptr;
  }
  *out = g_scratch[dev];
  return TR_OK;
}

extern "C" tr_status tr_render_batch_noalloc(int32_t n, const tr_scene *const *scenes,
                                             const tr_camera *cams, const tr_params *params,
                                             const tr_frame *frames, const tr_tune *tune,
                                             void *hip_stream) {
  if (n < 1 || n > TR_NOALLOC_MAX_JOBS)
    return fail(TR_EINVAL, "tr_render_batch_noalloc: %d jobs (1..%d)", (int)n, TR_NOALLOC_MAX_JOBS);
  if (!scenes || !cams || !params || !frames) return fail(TR_EINVAL, "NULL batch array");
  hipStream_t st = (hipStream_t)hip_stream;
  // the first FP32 job sets the batch's FP32 precision, stats and tuning
  int32_t f0 = 0;
  while (f0 < n - 1 && params[f0].precision == TR_PREC_FP64) ++f0;
  const tr_tune t = pick_tune(scenes[f0], &cams[f0], &params[f0], tune);
  tr_status rc = check_tune(t);
  if (rc != TR_OK) return rc;
  const int res = params[f0].precision == TR_PREC_FP32_RESOLVE;
  uint64_t *stats = frames[f0].stats;
  // fixed-size tables on the stack: nothing is allocated
  JobDev jobs[TR_NOALLOC_MAX_JOBS], f64[TR_NOALLOC_MAX_JOBS];
  uint64_t *stats64[TR_NOALLOC_MAX_JOBS];
  int32_t nw = 0, n64 = 0;
  for (int32_t i = 0; i < n; ++i) {  // every job is checked before anything is enqueued
    JobDev J;
    rc = make_job(scenes[i], &cams[i], &params[i], &frames[i], t.tile_w, J);
    if (rc != TR_OK) return fail(rc, "job %d: %s", i, g_err.c_str());
    if (aa_count(params[i]) > 1)
      return fail(TR_EUNSUPPORTED, "job %d: antialiasing needs a workspace (aa_samples <= 1 here)", i);
    if (params[i].precision == TR_PREC_FP64) {
      stats64[n64] = frames[i].stats;
      f64[n64++] = J;
      continue;
    }
    if ((params[i].precision == TR_PREC_FP32_RESOLVE) != (res != 0))
      return fail(TR_EINVAL, "all FP32 jobs of one batch must use the same precision");
    if (frames[i].stats != stats) return fail(TR_EINVAL, "all jobs of one batch must share one stats buffer");
    rc = check_wave_job(J, t);
    if (rc != TR_OK) return fail(rc, "job %d: %s", i, g_err.c_str());
    jobs[nw++] = J;
  }
  // jobs of one scene adjacent (a stable insertion sort), as in tr_render_batch
  for (int32_t i = 1; i < nw; ++i)
    for (int32_t j = i; j > 0 && jobs[j - 1].scene_key > jobs[j].scene_key; --j) std::swap(jobs[j - 1], jobs[j]);
  const int64_t total = set_queue(jobs, nw);
  if (total > (int64_t)UINT32_MAX - 1) return fail(TR_EINVAL, "too many tiles in one launch");
  NoAllocScratch *S = nullptr;
  if (nw > 0 && total > 0) {
    rc = scratch_on_device(&S);
    if (rc != TR_OK) return rc;
  }
  for (int32_t k = 0; k < n64; ++k) HIP_TRY(trh::launch_render_plain_f64(f64[k], stats64[k], st));
  if (!S) return TR_OK;
  // clear the counter with a kernel (no memset node under graph capture),
  // write the table from kernel arguments, then render
  HIP_TRY(trh::launch_fill_u32(S->counter, trd::kQueueWords, 0u, st));
  for (int32_t k = 0; k < nw; ++k) HIP_TRY(trh::launch_put_job(jobs[k], &S->jobs[k], st));
  const trh::WaveLaunch L = wave_launch(jobs, nw, total, t, stats, S->jobs, S->counter);
  HIP_TRY(trh::launch_render_wave(L, st));
  return TR_OK;
}

extern "C" tr_status tr_render_batch(int32_t n, const tr_scene *const *scenes, const tr_camera *cams,
                                     const tr_params *params, const tr_frame *frames, void *hip_stream) {
  return batch_impl(n, scenes, cams, params, frames, nullptr, nullptr, nullptr, (hipStream_t)hip_stream);
}

extern "C" tr_status tr_render_batch_tiles(int32_t n, const tr_scene *const *scenes,
                                           const tr_camera *cams, const tr_params *params,
                                           const tr_frame *frames, const int64_t *tile_begin,
                                           const int64_t *tile_end, const tr_tune *tune,
                                           void *hip_stream) {
  if (!tile_begin || !tile_end) return fail(TR_EINVAL, "NULL tile range");
  return batch_impl(n, scenes, cams, params, frames, tile_begin, tile_end, tune,
                    (hipStream_t)hip_stream);
}

extern "C" tr_status tr_frame_quantize(const float *values, int64_t n, uint8_t *out,
                                       void *hip_stream) {
  if (n < 0) return fail(TR_EINVAL, "tr_frame_quantize: n < 0");
  if (n == 0) return TR_OK;
  if (!values || !out) return fail(TR_EINVAL, "tr_frame_quantize: NULL buffer");
  HIP_TRY(trh::launch_quantize_rgb8(values, n, out, (hipStream_t)hip_stream));
  return TR_OK;
}

// ------------------------------------------------------------ Targa file
extern "C" int64_t tr_tga_max_bytes(int32_t width, int32_t height) {
  if (width < 1 || width > 65535 || height < 1 || height > 65535) return -1;
  // a pixel costs at most 4 bytes (a raw packet's header and first pixel)
  return 18 + 26 + (int64_t)height * 4 * (int64_t)width;
}

// Per-stream scratch of the encoder: row sizes, row offsets, the file size
// (device) and its pinned read-back.
struct TgaWork {
  int64_t *rows = nullptr;  // [2 * cap + 1]: sizes, offsets, total
  int64_t *h_total = nullptr;
  int32_t cap = 0;
};
static std::map<std::pair<int, hipStream_t>, TgaWork> g_tga_work;

extern "C" tr_status tr_frame_encode_tga(const uint8_t *rgb8, int32_t width, int32_t height,
                                         uint8_t *out, int64_t capacity, int64_t *size,
                                         void *hip_stream) {
  if (!size) return fail(TR_EINVAL, "tr_frame_encode_tga: NULL size");
  *size = 0;
  if (width < 1 || width > 65535 || height < 1 || height > 65535)
    return fail(TR_EINVAL, "Targa width and height must be 1..65535");
  if (!rgb8) return fail(TR_EINVAL, "tr_frame_encode_tga: NULL image");
  if (capacity < 0 || (!out && capacity > 0)) return fail(TR_EINVAL, "tr_frame_encode_tga: bad output buffer");
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_mu);
  TgaWork &w = g_tga_work[{dev, st}];
  if (w.cap < height) {
    if (w.rows) {  // earlier work on this stream may still use the old scratch
      HIP_TRY(hipStreamSynchronize(st));
      HIP_TRY(hipFree(w.rows));
      w.rows = nullptr;
      w.cap = 0;
    }
    HIP_TRY(hipMalloc((void **)&w.rows, (2 * (size_t)height + 1) * sizeof(int64_t)));
    w.cap = height;
  }
  if (!w.h_total) HIP_TRY(hipHostMalloc((void **)&w.h_total, sizeof(int64_t), hipHostMallocDefault));
  int64_t *row_bytes = w.rows, *row_off = w.rows + w.cap, *total = w.rows + 2 * (int64_t)w.cap;
  HIP_TRY(trh::launch_tga_sizes(rgb8, width, height, row_bytes, row_off, total, st));
  HIP_TRY(hipMemcpyAsync(w.h_total, total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *size = *w.h_total;
  if (*size > capacity)
    return fail(TR_EINVAL, "Targa file needs %lld bytes, the buffer holds %lld", (long long)*size,
                (long long)capacity);
  HIP_TRY(trh::launch_tga_write(rgb8, width, height, row_off, total, out, st));
  return TR_OK;
}

extern "C" size_t tr_frame_footprint(const tr_camera *c, const tr_params *p, uint32_t flags) {
  if (!c || c->width <= 0 || c->height <= 0) return 0;
  (void)p;
  const size_t px = (size_t)c->width * (size_t)c->height;
  size_t b = 0;
  if (flags & 1u) b += px * 12;
  if (flags & 2u) b += px * 4;
  if (flags & 4u) b += px * 4;
  if (flags & 8u) b += px;
  return b;
}

// ----------------------------------------------------------------- graphs
struct tr_graph {
  int32_t n = 0;
  std::vector<JobDev> jobs;  // host copy (queue offsets filled)
  std::vector<const tr_scene *> scenes;
  std::vector<tr_frame> frames;
  std::vector<tr_camera> cams;
  std::vector<tr_params> params;
  tr_tune tune{};
  JobDev *h_jobs = nullptr, *d_jobs = nullptr;
  uint32_t *d_counter = nullptr;
  hipEvent_t staged = nullptr;    // the last job-table upload has run
  hipEvent_t launched = nullptr;  // the last replay has run
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t total_tiles = 0;
};

static void free_graph(tr_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->h_jobs) (void)hipHostFree(g->h_jobs);
  if (g->d_jobs) (void)hipFree(g->d_jobs);
  if (g->d_counter) (void)hipFree(g->d_counter);
  if (g->staged) (void)hipEventDestroy(g->staged);
  if (g->launched) (void)hipEventDestroy(g->launched);
  delete g;
}

// Stage the host job table and copy it to the device on the stream, after
// any replay already enqueued (on whatever stream) has finished reading it.
static tr_status graph_upload(tr_graph *g, hipStream_t st) {
  HIP_TRY(hipEventSynchronize(g->staged));  // previous staging copy has run
  std::memcpy(g->h_jobs, g->jobs.data(), sizeof(JobDev) * g->jobs.size());
  HIP_TRY(hipStreamWaitEvent(st, g->launched, 0));
  HIP_TRY(hipMemcpyAsync(g->d_jobs, g->h_jobs, sizeof(JobDev) * g->jobs.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(g->staged, st));
  return TR_OK;
}

// Capture the graph's launch for its current jobs and tune: the counter
// reset (a kernel, not a memset node) and the persistent launch.  Any
// previous capture is dropped once its replays have run.
static tr_status graph_capture(tr_graph *g) {
  HIP_TRY(hipEventSynchronize(g->launched));
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
  const int32_t n = g->n;
  hipStream_t cap = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    e = trh::launch_fill_u32(g->d_counter, trd::kQueueWords, 0u, cap);
    trh::WaveLaunch L{};
    L.jobs = g->d_jobs;
    L.n_jobs = n;
    L.n_tiles = g->total_tiles;
    L.tile_counter = g->d_counter;
    L.stats = g->frames[0].stats;
    L.tile_w = g->tune.tile_w;
    L.banks = g->tune.banks;
    L.refill_below = g->tune.refill_below;
    L.count_ops = g->tune.count_ops;
    L.stripe = g->tune.stripe;
    int64_t waves = (int64_t)num_cus() * g->tune.waves_per_cu;
    if (waves > g->total_tiles) waves = g->total_tiles;
    L.n_waves = (int32_t)std::max<int64_t>(waves, 1);
    L.resolve = g->params[0].precision == TR_PREC_FP32_RESOLVE;
    L.trans = 0;
    L.tri = 0;
    for (int32_t i = 0; i < n; ++i) L.tri |= g->jobs[i].sc.n_t > 0;
    L.bvh = g->tune.accel;
    if (e == hipSuccess) e = trh::launch_render_wave(L, cap);
    hipError_t e2 = hipStreamEndCapture(cap, &g->graph);
    if (e == hipSuccess) e = e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (cap) (void)hipStreamDestroy(cap);
  if (e != hipSuccess) return fail(TR_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  return TR_OK;
}

// Re-make the graph's jobs for tune t (its tile width sets the tile grid and
// the queue offsets), upload the table and capture the launch anew.
static tr_status graph_retune(tr_graph *g, const tr_tune &t, hipStream_t st) {
  tr_status rc = check_tune(t);
  if (rc != TR_OK) return rc;
  std::vector<JobDev> nj(g->n);
  int64_t total = 0;
  for (int32_t i = 0; i < g->n; ++i) {
    rc = make_job(g->scenes[i], &g->cams[i], &g->params[i], &g->frames[i], t.tile_w, nj[i]);
    if (rc == TR_OK) rc = check_wave_job(nj[i], t);
    if (rc != TR_OK) return fail(rc, "job %d: %s", i, g_err.c_str());
    nj[i].queue_begin = total;
    total += nj[i].tile_end;
  }
  g->jobs = nj;
  g->total_tiles = total;
  g->tune = t;
  rc = graph_upload(g, st);
  if (rc != TR_OK) return rc;
  return graph_capture(g);
}

extern "C" tr_status tr_graph_create(int32_t n, const tr_scene *const *scenes, const tr_camera *cams,
                                     const tr_params *params, const tr_frame *frames,
                                     const tr_tune *tune, void *hip_stream, tr_graph **out) {
  if (!out) return fail(TR_EINVAL, "NULL out");
  *out = nullptr;
  if (n < 1 || n > 4096) return fail(TR_EINVAL, "graph batch size must be 1..4096");
  if (!scenes || !cams || !params || !frames) return fail(TR_EINVAL, "NULL batch array");
  tr_graph *g = new tr_graph();
  g->n = n;
  g->tune = pick_tune(scenes[0], &cams[0], &params[0], tune);
  tr_status rc = check_tune(g->tune);
  if (rc != TR_OK) {
    free_graph(g);
    return rc;
  }
  int64_t total = 0;
  const int res = params[0].precision == TR_PREC_FP32_RESOLVE;
  for (int32_t i = 0; i < n; ++i) {
    JobDev J;
    rc = make_job(scenes[i], &cams[i], &params[i], &frames[i], g->tune.tile_w, J);
    if (rc == TR_OK && params[i].precision == TR_PREC_FP64)
      rc = fail(TR_EUNSUPPORTED, "graphs need an FP32 precision");
    if (rc == TR_OK && aa_count(params[i]) > 1)
      rc = fail(TR_EUNSUPPORTED, "graphs need aa_samples <= 1");
    if (rc == TR_OK && J.layers > 1)
      rc = fail(TR_EUNSUPPORTED, "graphs render opaque frames (max_layers <= 1)");
    if (rc == TR_OK && (params[i].precision == TR_PREC_FP32_RESOLVE) != (res != 0))
      rc = fail(TR_EINVAL, "all jobs of one graph must use the same precision");
    if (rc == TR_OK && frames[i].stats != frames[0].stats)
      rc = fail(TR_EINVAL, "all jobs of one graph must share one stats buffer");
    if (rc == TR_OK) rc = check_wave_job(J, g->tune);
    if (rc != TR_OK) {
      free_graph(g);
      return rc;
    }
    J.queue_begin = total;
    total += J.tile_end;
    g->jobs.push_back(J);
    g->scenes.push_back(scenes[i]);
    g->frames.push_back(frames[i]);
    g->cams.push_back(cams[i]);
    g->params.push_back(params[i]);
  }
  g->total_tiles = total;
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = hipHostMalloc((void **)&g->h_jobs, sizeof(JobDev) * n, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void **)&g->d_jobs, sizeof(JobDev) * n);
  if (e == hipSuccess) e = hipMalloc((void **)&g->d_counter, trd::kQueueWords * sizeof(uint32_t));
  if (e == hipSuccess) e = hipEventCreateWithFlags(&g->staged, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&g->launched, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(g->staged, st);
  if (e == hipSuccess) e = hipEventRecord(g->launched, st);
  if (e != hipSuccess) {
    free_graph(g);
    return fail(TR_EDEVICE, "graph resources: %s", hipGetErrorString(e));
  }
  rc = graph_upload(g, st);
  if (rc != TR_OK) {
    free_graph(g);
    return rc;
  }
  rc = graph_capture(g);
  if (rc != TR_OK) {
    free_graph(g);
    return rc;
  }
  *out = g;
  return TR_OK;
}

extern "C" tr_status tr_graph_update(tr_graph *g, const tr_camera *cams, const tr_params *params,
                                     void *hip_stream) {
  if (!g) return fail(TR_EINVAL, "NULL graph");
  // (with both NULL the job table is rebuilt from the scenes as they are
  // now, which picks up rebuilt grids and BVHs)
  std::vector<JobDev> nj(g->n);
  for (int32_t i = 0; i < g->n; ++i) {
    const tr_camera &c = cams ? cams[i] : g->cams[i];
    const tr_params &p = params ? params[i] : g->params[i];
    if (c.width != g->cams[i].width || c.height != g->cams[i].height)
      return fail(TR_EINVAL, "job %d: resolution differs from the captured one", i);
    if (p.precision != g->params[i].precision)
      return fail(TR_EINVAL, "job %d: precision differs from the captured one", i);
    if (aa_count(p) > 1) return fail(TR_EUNSUPPORTED, "job %d: graphs need aa_samples <= 1", i);
    tr_status rc = make_job(g->scenes[i], &c, &p, &g->frames[i], g->tune.tile_w, nj[i]);
    if (rc != TR_OK) return fail(rc, "job %d: %s", i, g_err.c_str());
    if (nj[i].layers > 1)
      return fail(TR_EUNSUPPORTED, "job %d: graphs render opaque frames (max_layers <= 1)", i);
    rc = check_wave_job(nj[i], g->tune);
    if (rc != TR_OK) return fail(rc, "job %d: %s", i, g_err.c_str());
    nj[i].queue_begin = g->jobs[i].queue_begin;
  }
  for (int32_t i = 0; i < g->n; ++i) {
    if (cams) g->cams[i] = cams[i];
    if (params) g->params[i] = params[i];
  }
  g->jobs = nj;
  return graph_upload(g, (hipStream_t)hip_stream);
}

extern "C" tr_status tr_graph_launch(tr_graph *g, void *hip_stream) {
  if (!g) return fail(TR_EINVAL, "NULL graph");
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(hipStreamWaitEvent(st, g->staged, 0));  // the latest job table is on the device
  HIP_TRY(hipGraphLaunch(g->exec, st));
  HIP_TRY(hipEventRecord(g->launched, st));
  return TR_OK;
}

extern "C" void tr_graph_destroy(tr_graph *g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  free_graph(g);
}

// ---------------------------------------------------------------- autotune
extern "C" tr_status tr_default_tune(tr_tune *out) {
  if (!out) return fail(TR_EINVAL, "NULL out");
  return default_tune(out);
}

// Tuning a captured graph on itself: grid density first, then the launch
// shape by coordinate descent, then the winner against the default shape.
namespace {
struct GraphTuner {
  tr_graph *g;
  hipStream_t st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  size_t px0 = 0, pxn = 0;
  std::vector<float> ref0, refn, cur0, curn;
  ~GraphTuner() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  tr_status init() {
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    px0 = (size_t)g->cams[0].width * g->cams[0].height;
    pxn = (size_t)g->cams[g->n - 1].width * g->cams[g->n - 1].height;
    ref0.resize(3 * px0);
    refn.resize(3 * pxn);
    cur0.resize(3 * px0);
    curn.resize(3 * pxn);
    return TR_OK;
  }
  // one warm-up replay, then the median of 3 timed replays
  tr_status time(double &ms) {
    tr_status rc = tr_graph_launch(g, st);
    if (rc != TR_OK) return rc;
    double t[3];
    for (int k = 0; k < 3; ++k) {
      HIP_TRY(hipEventRecord(e0, st));
      rc = tr_graph_launch(g, st);
      if (rc != TR_OK) return rc;
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      float f = 0.0f;
      HIP_TRY(hipEventElapsedTime(&f, e0, e1));
      t[k] = f;
    }
    std::sort(t, t + 3);
    ms = t[1];
    return TR_OK;
  }
  tr_status read(std::vector<float> &a, std::vector<float> &b) {
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipMemcpy(a.data(), g->frames[0].rgb, 12 * px0, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(b.data(), g->frames[g->n - 1].rgb, 12 * pxn, hipMemcpyDeviceToHost));
    return TR_OK;
  }
  // time the graph as it stands and check its first and last frames
  tr_status trial(double &ms, const char *what) {
    tr_status rc = time(ms);
    if (rc == TR_OK) rc = read(cur0, curn);
    if (rc != TR_OK) return rc;
    if (std::memcmp(cur0.data(), ref0.data(), 12 * px0) != 0 ||
        std::memcmp(curn.data(), refn.data(), 12 * pxn) != 0)
      return fail(TR_EDEVICE, "graph autotune: %s changed the frames", what);
    return TR_OK;
  }
};
}  // namespace

extern "C" tr_status tr_graph_autotune(tr_graph *g, int32_t n_lambdas, const double *lambdas,
                                       void *hip_stream, tr_tune *best, double *best_lambda,
                                       double *best_ms) {
  if (!g) return fail(TR_EINVAL, "NULL graph");
  if (n_lambdas < 0 || n_lambdas > 64 || (n_lambdas > 0 && !lambdas))
    return fail(TR_EINVAL, "tr_graph_autotune: n_lambdas must be 0..64 with a lambda array");
  for (int32_t i = 0; i < n_lambdas; ++i)
    if (!(lambdas[i] > 0.0) || !std::isfinite(lambdas[i]))
      return fail(TR_EINVAL, "tr_graph_autotune: lambda %d must be finite and > 0", i);
  GraphTuner T{g, (hipStream_t)hip_stream};
  tr_status rc = T.init();
  if (rc != TR_OK) return rc;
  // the graph's scenes, each once, with their own densities
  std::vector<tr_scene *> uniq;
  std::vector<double> own;
  for (const tr_scene *s : g->scenes) {
    tr_scene *m = const_cast<tr_scene *>(s);
    if (std::find(uniq.begin(), uniq.end(), m) == uniq.end()) {
      uniq.push_back(m);
      own.push_back(m->lambda);
    }
  }
  const tr_tune orig = g->tune;
  auto tune_all = [&]() -> tr_status {
    double cur_ms = 0.0;
    rc = T.time(cur_ms);
    if (rc == TR_OK) rc = T.read(T.ref0, T.refn);
    if (rc != TR_OK) return rc;
    // grid density: every scene at one candidate density (0 = their own)
    double lam = 0.0;
    auto set_lambda = [&](double l) -> tr_status {
      HIP_TRY(hipStreamSynchronize(T.st));
      for (size_t k = 0; k < uniq.size(); ++k) {
        const tr_status r = tr_scene_rebuild(uniq[k], l > 0.0 ? l : own[k], T.st);
        if (r != TR_OK) return r;
      }
      return tr_graph_update(g, nullptr, nullptr, T.st);
    };
    for (int32_t i = 0; i < n_lambdas; ++i) {
      rc = set_lambda(lambdas[i]);
      double ms = 0.0;
      if (rc == TR_OK) rc = T.trial(ms, "a grid density");
      else if (rc == TR_EUNSUPPORTED || rc == TR_ENOMEM) {  // that grid cannot be built: skip it
        rc = set_lambda(lam);
        if (rc != TR_OK) return rc;
        continue;
      }
      if (rc != TR_OK) return rc;
      if (ms < cur_ms) {
        cur_ms = ms;
        lam = lambdas[i];
      }
    }
    rc = set_lambda(lam);
    if (rc != TR_OK) return rc;
    // launch shape: one pass of coordinate descent
    tr_tune cur = g->tune;
    const std::vector<std::vector<int32_t>> axes = {
        {8, 16, 64}, {2, 3}, {12, 16, 20, 24}, {24, 32, 40, 48}, {16, 32, 64, 128, 256}};
    rc = T.trial(cur_ms, "the starting shape");  // re-time after the density change
    if (rc != TR_OK) return rc;
    for (size_t ax = 0; ax < axes.size(); ++ax) {
      for (int32_t v : axes[ax]) {
        tr_tune t = cur;
        int32_t *field = ax == 0   ? &t.tile_w
                         : ax == 1 ? &t.banks
                         : ax == 2 ? &t.waves_per_cu
                         : ax == 3 ? &t.refill_below
                                   : &t.stripe;
        if (*field == v) continue;
        *field = v;
        rc = graph_retune(g, t, T.st);
        double ms = 0.0;
        if (rc == TR_OK) rc = T.trial(ms, "a launch shape");
        if (rc != TR_OK) return rc;
        if (ms < cur_ms) {
          cur_ms = ms;
          cur = t;
        }
      }
    }
    // the winner against the default shape, interleaved, median of 5 each
    tr_tune def;
    default_tune(&def);
    def.count_ops = cur.count_ops;
    def.accel = cur.accel;
    if (std::memcmp(&def, &cur, sizeof(tr_tune)) != 0) {
      double a[5], b[5];
      for (int rep = 0; rep < 5; ++rep) {
        rc = graph_retune(g, def, T.st);
        if (rc == TR_OK) rc = T.trial(a[rep], "the default shape");
        if (rc == TR_OK) rc = graph_retune(g, cur, T.st);
        if (rc == TR_OK) rc = T.trial(b[rep], "a launch shape");
        if (rc != TR_OK) return rc;
      }
      std::sort(a, a + 5);
      std::sort(b, b + 5);
      if (a[2] <= b[2]) {
        cur = def;
        cur_ms = a[2];
      } else {
        cur_ms = b[2];
      }
    }
    rc = graph_retune(g, cur, T.st);
    if (rc != TR_OK) return rc;
    HIP_TRY(hipStreamSynchronize(T.st));
    if (best) *best = cur;
    if (best_lambda) *best_lambda = lam;
    if (best_ms) *best_ms = cur_ms;
    return TR_OK;
  };
  rc = tune_all();
  if (rc != TR_OK) {
    // put the graph and its scenes back as they were, keeping the error
    const std::string err = g_err;
    (void)hipStreamSynchronize(T.st);
    for (size_t k = 0; k < uniq.size(); ++k) (void)tr_scene_rebuild(uniq[k], own[k], T.st);
    (void)graph_retune(g, orig, T.st);
    g_err = err;
  }
  return rc;
}

extern "C" tr_status tr_measure_fp32_peak(void *hip_stream, double *tflops, double *clock_mhz,
                                          int32_t *n_cus) {
  if (!tflops) return fail(TR_EINVAL, "tr_measure_fp32_peak: NULL tflops");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  HIP_TRY(trh::measure_fma_rate((hipStream_t)hip_stream, prop.multiProcessorCount, tflops));
  if (clock_mhz) *clock_mhz = prop.clockRate * 1e-3;
  if (n_cus) *n_cus = prop.multiProcessorCount;
  return TR_OK;
}

extern "C" tr_status tr_autotune(const tr_scene *s, const tr_camera *c, const tr_params *p,
                                 void *hip_stream, tr_tune *best, double *best_ms) {
  if (!s || !c || !p) return fail(TR_EINVAL, "tr_autotune: NULL argument");
  tr_status rc = check_camera(c);
  if (rc != TR_OK) return rc;
  if (p->precision == TR_PREC_FP64) {
    tr_tune d;
    default_tune(&d);
    if (best) *best = d;
    if (best_ms) *best_ms = 0.0;
    return TR_OK;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t px = (size_t)c->width * c->height;
  float *rgb_ref = nullptr, *rgb = nullptr;
  int32_t *hid_ref = nullptr, *hid = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (rgb_ref) (void)hipFree(rgb_ref);
    if (rgb) (void)hipFree(rgb);
    if (hid_ref) (void)hipFree(hid_ref);
    if (hid) (void)hipFree(hid);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  {
    hipError_t e = hipMalloc((void **)&rgb_ref, px * 12);
    if (e == hipSuccess) e = hipMalloc((void **)&rgb, px * 12);
    if (e == hipSuccess) e = hipMalloc((void **)&hid_ref, px * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&hid, px * 4);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
      cleanup();
      return fail(e == hipErrorOutOfMemory ? TR_ENOMEM : TR_EDEVICE, "autotune buffers: %s",
                  hipGetErrorString(e));
    }
  }
  std::vector<float> h_a(px * 3), h_b(px * 3);
  std::vector<int32_t> i_a(px), i_b(px);
  auto run = [&](const tr_tune &t, float *out_rgb, int32_t *out_hid, double &ms) -> tr_status {
    tr_frame fr{out_rgb, out_hid, nullptr, nullptr, nullptr};
    tr_status r = tr_render_tuned(s, c, p, &fr, &t, st);  // warm-up
    if (r != TR_OK) return r;
    std::vector<double> times;
    for (int rep = 0; rep < 3; ++rep) {
      HIP_TRY(hipEventRecord(e0, st));
      r = tr_render_tuned(s, c, p, &fr, &t, st);
      if (r != TR_OK) return r;
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      float f = 0;
      HIP_TRY(hipEventElapsedTime(&f, e0, e1));
      times.push_back(f);
    }
    std::sort(times.begin(), times.end());
    ms = times[1];
    return TR_OK;
  };
  tr_tune cur;
  default_tune(&cur);
  double cur_ms = 0;
  rc = run(cur, rgb_ref, hid_ref, cur_ms);
  if (rc != TR_OK) {
    cleanup();
    return rc;
  }
  if (hipMemcpy(h_a.data(), rgb_ref, px * 12, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(i_a.data(), hid_ref, px * 4, hipMemcpyDeviceToHost) != hipSuccess) {
    cleanup();
    return fail(TR_EDEVICE, "autotune readback failed");
  }
  // coordinate descent over the launch-shape axes
  const std::vector<std::vector<int32_t>> axes = {
      {4, 8, 16, 32, 64}, {2, 3}, {8, 12, 16, 20, 24, 32}, {16, 24, 32, 40, 48, 56},
      {16, 32, 64, 128, 256}};
  for (int pass = 0; pass < 2; ++pass) {
    for (size_t ax = 0; ax < axes.size(); ++ax) {
      for (int32_t v : axes[ax]) {
        tr_tune t = cur;
        int32_t *field = ax == 0   ? &t.tile_w
                         : ax == 1 ? &t.banks
                         : ax == 2 ? &t.waves_per_cu
                         : ax == 3 ? &t.refill_below
                                   : &t.stripe;
        if (*field == v) continue;
        *field = v;
        double ms = 0;
        rc = run(t, rgb, hid, ms);
        if (rc != TR_OK) {
          cleanup();
          return rc;
        }
        if (hipMemcpy(h_b.data(), rgb, px * 12, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(i_b.data(), hid, px * 4, hipMemcpyDeviceToHost) != hipSuccess) {
          cleanup();
          return fail(TR_EDEVICE, "autotune readback failed");
        }
        if (std::memcmp(h_a.data(), h_b.data(), px * 12) != 0 ||
            std::memcmp(i_a.data(), i_b.data(), px * 4) != 0) {
          cleanup();
          return fail(TR_EDEVICE, "autotune: launch shape (%d,%d,%d,%d,%d) changed the frame",
                      t.tile_w, t.banks, t.waves_per_cu, t.refill_below, t.stripe);
        }
        if (ms < cur_ms) {
          cur_ms = ms;
          cur = t;
        }
      }
    }
  }
  // Single renders are noisy at the percent level: confirm the winner
  // against the default shape, interleaved, on the median of 7 each.
  {
    tr_tune def;
    default_tune(&def);
    if (std::memcmp(&def, &cur, sizeof(tr_tune)) != 0) {
      std::vector<double> a, b;
      for (int rep = 0; rep < 7 && rc == TR_OK; ++rep) {
        double ms = 0;
        rc = run(def, rgb, hid, ms);
        a.push_back(ms);
        if (rc == TR_OK) rc = run(cur, rgb, hid, ms);
        b.push_back(ms);
      }
      if (rc != TR_OK) {
        cleanup();
        return rc;
      }
      std::sort(a.begin(), a.end());
      std::sort(b.begin(), b.end());
      if (a[3] <= b[3]) {
        cur = def;
        cur_ms = a[3];
      } else {
        cur_ms = b[3];
      }
    }
  }
  cleanup();
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tune_cache[tune_key(s, c, p)] = cur;
  }
  if (best) *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return TR_OK;
}

// ------------------------------------------------------------------ debug
extern "C" tr_status tr_debug_philox(int64_t n, const uint32_t *ctr, const uint32_t *key,
                                     uint32_t *out, void *hip_stream) {
  if (n < 0 || (n > 0 && (!ctr || !key || !out))) return fail(TR_EINVAL, "tr_debug_philox: bad arguments");
  HIP_TRY(trh::launch_debug_philox(n, ctr, key, out, (hipStream_t)hip_stream));
  return TR_OK;
}

extern "C" tr_status tr_debug_ao_dirs(int64_t n, const float *normals, const uint32_t *pix,
                                      const uint32_t *sample, uint32_t view_id, uint64_t seed,
                                      float *w, void *hip_stream) {
  if (n < 0 || (n > 0 && (!normals || !pix || !sample || !w)))
    return fail(TR_EINVAL, "tr_debug_ao_dirs: bad arguments");
  HIP_TRY(trh::launch_debug_ao_dirs(n, normals, pix, sample, view_id, (uint32_t)(seed & 0xFFFFFFFFull),
                                    (uint32_t)(seed >> 32), w, (hipStream_t)hip_stream));
  return TR_OK;
}

extern "C" const char *tr_last_error(void) { return g_err.c_str(); }
extern "C" int32_t tr_abi_version(void) { return TR_ABI_VERSION; }
