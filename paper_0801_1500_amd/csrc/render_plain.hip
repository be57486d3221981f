// render_plain.hip -- the plain double-precision GPU path: one thread per
// pixel, every step in FP64, no queues.  This is the GPU counterpart of the
// paper's renderer as it was built ("double precision option for all
// calculations", Sec. 2) and the baseline the FP32 wavefront kernel is
// measured against.
//
// Compiled with -ffp-contract=off and written in the same expression order
// as the definition of the method (camera, intersections, normals,
// sampling, shading), so that primary hits reproduce bit for bit.
#include "tr_internal.h"

namespace {

using namespace trd;

constexpr double kEps = 1e-4;  // secondary-ray t_min (world units)

struct Cnt {
  uint32_t rays, cells, st, sh, ct, ch, tt, th;
};

// Nearest hit (lexicographic min of (t, id)) or any hit with t in
// (tmin, tmax], visiting the grid cells the ray crosses in order.
//
// On axis a the ray meets the grid plane of index p (at lo + p h) at
// t = b_a + p g_a, with b_a = (lo_a - o_a) / d_a and g_a = h_a / d_a: the
// first crossing is one FMA from the entry cell's plane, and each later one
// |g_a| further.  The walk keeps, per axis, the next crossing, the cells
// left before the grid's side and the step of the cell's linear index.  Any
// walk that visits every cell the segment crosses gives the same nearest
// hit: the lists hold every primitive within the insertion margin of a cell,
// far above the FP64 rounding of the crossings.
template <bool ANY, bool TRI>
__device__ int trace_f64(const SceneDev &S, const double o[3], const double d[3], double tmin,
                         double tmax, int32_t skip, double &bt, int32_t &bk, Cnt &c) {
  c.rays++;
  bool found = false;
  bt = INFINITY;
  bk = -1;
  // the part of (tmin, tmax] inside the grid box, axis by axis
  double tin = tmin, tout = tmax;
  double b[3], g[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (o[a] < S.lo[a] || o[a] > S.hi[a]) return 0;
      b[a] = g[a] = 0.0;
      continue;
    }
    b[a] = (S.lo[a] - o[a]) / d[a];
    g[a] = S.h[a] / d[a];
    const double tl = b[a], th = (S.hi[a] - o[a]) / d[a];
    tin = fmax(tin, fmin(tl, th));
    tout = fmin(tout, fmax(tl, th));
  }
  if (tin > tout) return 0;
  // entry cell (clamped into the grid); per axis the next crossing, the
  // time between crossings, the cells left to the grid's side and the step
  // of the linear index (a grid has at most 512^3 cells: 32-bit indices)
  int32_t left[3], stride[3];
  double tn[3], dt[3];
  const int32_t plane_cells[3] = {1, S.res[0], S.res[0] * S.res[1]};
  int32_t cell = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double f = floor((o[a] + tin * d[a] - S.lo[a]) * S.inv[a]);
    const int32_t i = f >= 0.0 ? (f < (double)S.res[a] ? (int32_t)f : S.res[a] - 1) : 0;
    cell += i * plane_cells[a];
    if (d[a] > 0.0) {
      tn[a] = fma((double)(i + 1), g[a], b[a]);
      dt[a] = g[a];
      left[a] = S.res[a] - 1 - i;
      stride[a] = plane_cells[a];
    } else if (d[a] < 0.0) {
      tn[a] = fma((double)i, g[a], b[a]);
      dt[a] = -g[a];
      left[a] = i;
      stride[a] = -plane_cells[a];
    } else {
      tn[a] = INFINITY;
      dt[a] = 0.0;
      left[a] = 0;
      stride[a] = 0;
    }
  }
  const double t1 = tout;
  for (;;) {
    c.cells++;
    const uint32_t e = S.cell_begin[(uint32_t)cell + 1u];
    for (uint32_t r = S.cell_begin[(uint32_t)cell]; r < e; ++r) {
      const int32_t k = (int32_t)S.refs[r];
      if (k == skip) continue;
      double t;
      int h;
      if (k < S.n_s) {
        c.st++;
        h = hit_sphere_f64(S.sph64[k], o, d, tmin, tmax, t);
        c.sh += h;
      } else if (TRI && k >= S.n_s + S.n_c) {
        const int32_t m = k - S.n_s - S.n_c;
        c.tt++;
        h = hit_triangle_f64(S.triA64[m], S.triB64[m], S.triC64[m], o, d, tmin, tmax, t);
        c.th += h;
      } else {
        c.ct++;
        h = hit_cylinder_f64(S.cylA64[k - S.n_s], S.cylW64[k - S.n_s], o, d, tmin, tmax, t);
        c.ch += h;
      }
      if (h) {
        if (ANY) {
          bt = t;
          bk = k;
          return 1;
        }
        if (!found || t < bt || (t == bt && k < bk)) {
          found = true;
          bt = t;
          bk = k;
        }
      }
    }
    // leave through the nearest plane; stop once the best hit lies in the
    // cells already seen, or at the end of the segment or the grid
    const int a = tn[0] <= tn[1] ? (tn[0] <= tn[2] ? 0 : 2) : (tn[1] <= tn[2] ? 1 : 2);
    if (!ANY && found && bt <= fmin(tn[a], t1)) return 1;
    if (!(tn[a] < t1) || left[a] == 0) return found;
    --left[a];
    cell += stride[a];
    tn[a] += dt[a];
  }
}

template <bool TRI>
__device__ __forceinline__ void normal_f64(const SceneDev &S, int32_t k, const double o[3],
                                           const double d[3], double t, double n[3]) {
  if (k < S.n_s) {
    const double4 s = S.sph64[k];
    const double P[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
    n[0] = (P[0] - s.x) / s.w;
    n[1] = (P[1] - s.y) / s.w;
    n[2] = (P[2] - s.z) / s.w;
  } else if (TRI && k >= S.n_s + S.n_c) {
    const int32_t m = k - S.n_s - S.n_c;
    triangle_normal_f64(S.triA64[m], S.triB64[m], S.triC64[m], n);
  } else {
    const double4 a = S.cylA64[k - S.n_s], w4 = S.cylW64[k - S.n_s];
    const double w[3] = {w4.x, w4.y, w4.z};
    const double D[3] = {o[0] - a.x, o[1] - a.y, o[2] - a.z};
    const double sax = dot3d(D, w) + t * dot3d(d, w);
#pragma unroll
    for (int q = 0; q < 3; ++q) n[q] = ((D[q] + t * d[q]) - sax * w[q]) / a.w;
  }
}

// Variants: layered compositing and triangles are compiled in only for jobs
// that need them (either costs registers, and so occupancy, in the others).
template <bool STATS, bool LAYERED, bool TRI>
__global__ __launch_bounds__(256) void k_render_plain_f64(const JobDev J, uint64_t *stats) {
  __shared__ uint32_t red[TR_STAT_COUNT];
  if (STATS) {
    if (threadIdx.x < TR_STAT_COUNT) red[threadIdx.x] = 0;
    __syncthreads();
  }
  const int32_t i = blockIdx.x * 16 + (threadIdx.x & 15);
  const int32_t j = blockIdx.y * 16 + (threadIdx.x >> 4);
  Cnt c{0, 0, 0, 0, 0, 0, 0, 0};
  uint32_t n_hit = 0, n_ao = 0, n_sh = 0;
  if (i < J.W && j < J.H) {
    const SceneDev &S = J.sc;
    const int64_t pid = (int64_t)j * J.W + i;
    double o[3], d[3];
    primary_ray_f64(J, i, j, o, d);
    // Surfaces along the primary ray, front to back: one for opaque
    // rendering; with layers, the ray continues through a primitive of
    // opacity < 1 from the hit point (skipping it only when leaving it) and
    // the colours composite by the transmittance in front of each surface.
    double acc[3] = {0.0, 0.0, 0.0};
    double T = 1.0;
    double tmin = 0.0;
    int32_t pskip = -1;
    int hit = 0;
    int32_t k0 = -1;
    uint32_t amask = 0;
    uint32_t lmask = 0;
    const int32_t layers = LAYERED ? J.layers : 1;
    for (int32_t layer = 0; layer < layers; ++layer) {
      double t;
      int32_t k;
      if (!trace_f64<false, TRI>(S, o, d, tmin, INFINITY, pskip, t, k, c)) break;
      if (layer == 0) {
        hit = 1;
        k0 = k;
        n_hit = 1;
      }
      double N[3], P[3];
      normal_f64<TRI>(S, k, o, d, t, N);
#pragma unroll
      for (int q = 0; q < 3; ++q) P[q] = o[q] + t * d[q];
      const bool front = dot3d(N, d) < 0.0;
      if (!front) {
        N[0] = -N[0];
        N[1] = -N[1];
        N[2] = -N[2];
      }
      const int32_t skip = front ? k : -1;
      uint32_t am = 0, lm = 0;
      double D[3] = {0.0, 0.0, 0.0};
      double Hs[3] = {0.0, 0.0, 0.0};  // Phong highlight (white, after the albedo)
      for (int l = 0; l < J.n_lights; ++l) {
        const double cl = dot3d(N, J.ldir[l]);
        if (!(cl > kLightMin)) continue;
        n_sh++;
        double tt;
        int32_t kk;
        if (trace_f64<true, TRI>(S, P, J.ldir[l], kEps, INFINITY, skip, tt, kk, c)) {
          lm |= 1u << l;
        } else {
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) D[ch] += J.lcol[l][ch] * cl;
          if (J.ks > 0.0) {
            // light direction mirrored about N, against the way back to the eye
            double R[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) R[q] = 2.0 * cl * N[q] - J.ldir[l][q];
            const double rv = -dot3d(R, d);
            if (rv > 0.0) {
              const double f = J.ks * pow(rv, J.shin);
#pragma unroll
              for (int ch = 0; ch < 3; ++ch) Hs[ch] += J.lcol[l][ch] * f;
            }
          }
        }
      }
      double ao = 1.0;
      if (J.S > 0) {
        int32_t aocc = 0;
        for (int s = 0; s < J.S; ++s) {
          uint32_t b1, b2;
          ao_uniform_bits((uint32_t)pid, (uint32_t)s + ((uint32_t)layer << 16), J.view_id,
                          (uint32_t)J.aa, J.key0, J.key1, b1, b2);
          double w[3];
          ao_dir_f64(N, b1, b2, w);
          n_ao++;
          double tt;
          int32_t kk;
          if (trace_f64<true, TRI>(S, P, w, kEps, J.ao_maxdist, skip, tt, kk, c)) {
            aocc++;
            if (s < 32) am |= 1u << s;
          }
        }
        ao = (double)(J.S - aocc) / (double)J.S;
      }
      if (layer == 0) {
        amask = am;
        lmask = lm;
      }
      const float4 alb = S.albedo[k];
      const double albv[3] = {(double)alb.x, (double)alb.y, (double)alb.z};
      const double alpha = LAYERED ? (double)alb.w : 1.0;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const double v = albv[ch] * (D[ch] + J.sky * ao) + Hs[ch];
        acc[ch] += T * alpha * (v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v));
      }
      T *= 1.0 - alpha;
      if (!(alpha < 1.0)) break;
#pragma unroll
      for (int q = 0; q < 3; ++q) o[q] = P[q];
      tmin = kEps;
      pskip = front ? -1 : k;
    }
    double col[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) col[ch] = acc[ch] + T * (double)J.bg[ch];
    J.rgb[pid * 3 + 0] = (float)col[0];
    J.rgb[pid * 3 + 1] = (float)col[1];
    J.rgb[pid * 3 + 2] = (float)col[2];
    if (J.hit_id) J.hit_id[pid] = hit ? k0 : -1;
    if (J.ao_mask) J.ao_mask[pid] = amask;
    if (J.light_mask) J.light_mask[pid] = (uint8_t)lmask;
    if (STATS) {
      atomicAdd(&red[TR_STAT_PIXELS], 1u);
      atomicAdd(&red[TR_STAT_HIT_PIXELS], n_hit);
      atomicAdd(&red[TR_STAT_AO_RAYS], n_ao);
      atomicAdd(&red[TR_STAT_SHADOW_RAYS], n_sh);
      atomicAdd(&red[TR_STAT_RAYS_TRACED], c.rays);
      atomicAdd(&red[TR_STAT_CELLS], c.cells);
      atomicAdd(&red[TR_STAT_SPH_TESTS], c.st);
      atomicAdd(&red[TR_STAT_SPH_HITS], c.sh);
      atomicAdd(&red[TR_STAT_CYL_TESTS], c.ct);
      atomicAdd(&red[TR_STAT_CYL_HITS], c.ch);
      atomicAdd(&red[TR_STAT_TRI_TESTS], c.tt);
      atomicAdd(&red[TR_STAT_TRI_HITS], c.th);
    }
  }
  if (STATS) {
    __syncthreads();
    if (threadIdx.x < TR_STAT_COUNT && red[threadIdx.x])
      atomicAdd((unsigned long long *)&stats[threadIdx.x], (unsigned long long)red[threadIdx.x]);
  }
}

}  // namespace

namespace trh {

hipError_t launch_render_plain_f64(const trd::JobDev &job, uint64_t *stats, hipStream_t st) {
  dim3 grid((unsigned)((job.W + 15) / 16), (unsigned)((job.H + 15) / 16));
  const bool lay = job.layers > 1, tri = job.sc.n_t > 0;
#define TR_PLAIN(S, L, T) k_render_plain_f64<S, L, T><<<grid, 256, 0, st>>>(job, S ? stats : nullptr)
  if (stats) {
    if (lay) { if (tri) TR_PLAIN(true, true, true); else TR_PLAIN(true, true, false); }
    else { if (tri) TR_PLAIN(true, false, true); else TR_PLAIN(true, false, false); }
  } else {
    if (lay) { if (tri) TR_PLAIN(false, true, true); else TR_PLAIN(false, true, false); }
    else { if (tri) TR_PLAIN(false, false, true); else TR_PLAIN(false, false, false); }
  }
#undef TR_PLAIN
  return hipGetLastError();
}

}  // namespace trh
