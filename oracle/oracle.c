/*
 * oracle.c -- plain, slow FP64 CPU reference renderer.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU baseline, never by the product path.  It shares no code
 * with the HIP implementation.  Built with -O2 -ffp-contract=off so every
 * expression rounds exactly as written.
 *
 * The paper gives the renderer's inputs and switches (resolution, light
 * rescale, sky light, ambient occlusion by Monte Carlo sampling, double
 * precision; Sec. 2, Strong scaling) but no formulas.  Each function below
 * states the reading it implements.  Floating-point expression order is part
 * of the definition (left to right as written) so that an independent
 * double-precision GPU path can reproduce primary hits bit for bit.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- vectors */
static double dot3(const double a[3], const double b[3]) {
  return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}
static void sub3(const double a[3], const double b[3], double r[3]) {
  r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static void cross3(const double a[3], const double b[3], double r[3]) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}
static void normalize3(const double v[3], double r[3]) {
  double n = sqrt(dot3(v, v));
  r[0] = v[0] / n; r[1] = v[1] / n; r[2] = v[2] / n;
}

/* ---------------------------------------------------------------- Philox
 * Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and
 * Shaw (SC'11).  One round multiplies words 0 and 2 by two fixed odd
 * constants, keeps both halves of each 64-bit product, and mixes the high
 * halves with words 1 and 3 and the round key; the key is bumped by two Weyl
 * constants between rounds.  Ten rounds. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void or_philox_many(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
  for (int64_t i = 0; i < n; ++i) or_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* Two uniforms on [0, 1) from one Philox draw: the top 24 bits of words 0
 * and 1, exact in both float and double. */
static void philox_uniforms(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed,
                            double *u1, double *u2) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
  uint32_t x[4];
  or_philox4x32_10(ctr, key, x);
  *u1 = (double)(x[0] >> 8) * (1.0 / 16777216.0);
  *u2 = (double)(x[1] >> 8) * (1.0 / 16777216.0);
}

/* AO sample s of pixel pix: counter (pix, s, view, 0), key (seed low, seed
 * high). */
void or_ao_uniforms(uint32_t pix, uint32_t s, uint32_t view_id, uint64_t seed, double *u1,
                    double *u2) {
  philox_uniforms(pix, s, view_id, 0u, seed, u1, u2);
}

/* With several primary samples per pixel, AO sample s of primary sample a
 * uses counter (pix, s, view, a): a = 0 is the single-sample stream above,
 * and every primary sample has its own AO directions. */
void or_ao_uniforms_aa(uint32_t pix, uint32_t s, uint32_t view_id, uint32_t a, uint64_t seed,
                       double *u1, double *u2) {
  philox_uniforms(pix, s, view_id, a, seed, u1, u2);
}

/* Antialiasing (several primary rays per pixel; the renderer's option, not
 * used in the paper's runs).  Sample 0 goes through the pixel centre, so one
 * sample is the plain renderer; sample a >= 1 through a uniform random point
 * of the pixel square, from counter (pix, a, view, 0xFFFFFFFF), a stream no
 * AO draw uses (AO counters have word 3 = a primary sample index < 2^31). */
void or_aa_offset(uint32_t pix, uint32_t a, uint32_t view_id, uint64_t seed, double *ox,
                  double *oy) {
  if (a == 0) {
    *ox = 0.5;
    *oy = 0.5;
    return;
  }
  philox_uniforms(pix, a, view_id, 0xFFFFFFFFu, seed, ox, oy);
}

/* Cosine-weighted hemisphere direction around unit normal n (Malley's
 * method: a uniform point on the unit disc lifted to the hemisphere), in
 * the branchless orthonormal basis of Duff et al. (JCGT 2017).  The cosine
 * weighting makes the visible fraction estimate (1/pi) * integral of
 * V cos(theta) over the hemisphere -- the paper's "diffuse illumination"
 * from a uniform sky (Sec. 2, on ambient occlusion). */
void or_ao_direction(const double n[3], double u1, double u2, double w[3]) {
  double r = sqrt(u1);
  double phi = 6.283185307179586 * u2;
  double lx = r * cos(phi);
  double ly = r * sin(phi);
  double lz = sqrt(1.0 - u1);
  double sigma = copysign(1.0, n[2]);
  double a = -1.0 / (sigma + n[2]);
  double b = n[0] * n[1] * a;
  double tx[3] = {1.0 + sigma * n[0] * n[0] * a, sigma * b, -sigma * n[0]};
  double bx[3] = {b, sigma + n[1] * n[1] * a, -n[1]};
  w[0] = (lx * tx[0] + ly * bx[0]) + lz * n[0];
  w[1] = (lx * tx[1] + ly * bx[1]) + lz * n[1];
  w[2] = (lx * tx[2] + ly * bx[2]) + lz * n[2];
}

/* -------------------------------------------------------------- camera
 * Pinhole camera, one ray through each pixel centre (the paper's -res W H
 * gives W columns and H rows; Sec. 2).  Row 0 is the top of the image. */
typedef struct {
  double eye[3], f[3], r[3], u[3];
  double th, aspect;
  int32_t W, H;
} cam_basis;

static void camera_basis(const or_camera *c, cam_basis *b) {
  double fwd[3], rr[3];
  sub3(c->lookat, c->eye, fwd);
  normalize3(fwd, b->f);
  cross3(b->f, c->up, rr);
  normalize3(rr, b->r);
  cross3(b->r, b->f, b->u);
  b->th = tan((c->fovy_deg * M_PI) / 360.0);
  b->aspect = (double)c->width / (double)c->height;
  memcpy(b->eye, c->eye, sizeof b->eye);
  b->W = c->width;
  b->H = c->height;
}

/* Ray through image position (px, py), in pixel units from the top-left
 * corner of the image (px = i + 1/2 is the centre of column i). */
static void basis_ray_at(const cam_basis *b, double px, double py, double o[3], double d[3]) {
  double x = (((2.0 * px) / (double)b->W) - 1.0) * b->th * b->aspect;
  double y = (1.0 - (2.0 * py) / (double)b->H) * b->th;
  double v[3];
  for (int a = 0; a < 3; ++a) v[a] = (b->f[a] + x * b->r[a]) + y * b->u[a];
  normalize3(v, d);
  memcpy(o, b->eye, 3 * sizeof(double));
}

static void basis_ray(const cam_basis *b, int32_t i, int32_t j, double o[3], double d[3]) {
  basis_ray_at(b, (double)i + 0.5, (double)j + 0.5, o, d);
}

void or_camera_ray(const or_camera *cam, int32_t i, int32_t j, double o[3], double d[3]) {
  cam_basis b;
  camera_basis(cam, &b);
  basis_ray(&b, i, j, o, d);
}

void or_camera_ray_at(const or_camera *cam, double px, double py, double o[3], double d[3]) {
  cam_basis b;
  camera_basis(cam, &b);
  basis_ray_at(&b, px, py, o, d);
}

/* ---------------------------------------------------------- intersections
 * Sphere, in the cancellation-resistant form of Haines et al. (Ray Tracing
 * Gems, 2019): the squared distance from the centre to the ray is taken from
 * the perpendicular vector rather than from |q|^2 - b^2.  d must be unit.
 * Returns the smaller root in (tmin, tmax], else the larger one, else none. */
int or_hit_sphere(const double c[3], double r, const double o[3], const double d[3],
                  double tmin, double tmax, double *t) {
  double q[3], l[3];
  sub3(c, o, q);
  double b = dot3(q, d);
  l[0] = q[0] - b * d[0]; l[1] = q[1] - b * d[1]; l[2] = q[2] - b * d[2];
  double disc = r * r - dot3(l, l);
  if (disc < 0.0) return 0;
  double s = sqrt(disc);
  double t0 = b - s, t1 = b + s;
  if (t0 > tmin && t0 <= tmax) { *t = t0; return 1; }
  if (t1 > tmin && t1 <= tmax) { *t = t1; return 1; }
  return 0;
}

/* Open finite cylinder (no caps) between end points a and b, radius rho.
 * Solve |perp(o - a + t d)|^2 = rho^2, i.e. A t^2 + 2 B t + C = 0, with the
 * stable pair of roots q/A and C/q, and keep a root whose axial coordinate
 * s = (o - a + t d).w lies in [0, L].  A ray parallel to the axis misses. */
typedef struct { double a[3], w[3], L, rho; } cyl_frame;

static void cylinder_frame(const double a[3], const double b[3], double rho, cyl_frame *cf) {
  double ab[3];
  sub3(b, a, ab);
  cf->L = sqrt(dot3(ab, ab));
  cf->w[0] = ab[0] / cf->L; cf->w[1] = ab[1] / cf->L; cf->w[2] = ab[2] / cf->L;
  memcpy(cf->a, a, sizeof cf->a);
  cf->rho = rho;
}

static int hit_cyl_frame(const cyl_frame *cf, const double o[3], const double d[3],
                         double tmin, double tmax, double *t) {
  double D[3], dp[3], Dp[3];
  sub3(o, cf->a, D);
  double dw = dot3(d, cf->w);
  double Dw = dot3(D, cf->w);
  for (int k = 0; k < 3; ++k) {
    dp[k] = d[k] - dw * cf->w[k];
    Dp[k] = D[k] - Dw * cf->w[k];
  }
  double A = dot3(dp, dp);
  double B = dot3(dp, Dp);
  double C = dot3(Dp, Dp) - cf->rho * cf->rho;
  if (A <= 1e-12 * dot3(d, d)) return 0;
  double disc = B * B - A * C;
  if (disc < 0.0) return 0;
  double sq = sqrt(disc);
  double qq = -(B + (B >= 0.0 ? sq : -sq));
  if (qq == 0.0) return 0;
  double r0 = qq / A, r1 = C / qq;
  double tl = r0 < r1 ? r0 : r1;
  double th = r0 < r1 ? r1 : r0;
  double roots[2] = {tl, th};
  for (int k = 0; k < 2; ++k) {
    double tt = roots[k];
    if (tt > tmin && tt <= tmax) {
      double s = Dw + tt * dw;
      if (s >= 0.0 && s <= cf->L) { *t = tt; return 1; }
    }
  }
  return 0;
}

int or_hit_cylinder(const double a[3], const double b[3], double rho, const double o[3],
                    const double d[3], double tmin, double tmax, double *t) {
  cyl_frame cf;
  cylinder_frame(a, b, rho, &cf);
  return hit_cyl_frame(&cf, o, d, tmin, tmax, t);
}

/* Triangle (v0, v1, v2), two-sided, by the method of Moller and Trumbore
 * (JGT 1997): with e1 = v1 - v0, e2 = v2 - v0, P = d x e2, det = e1.P,
 * T = o - v0, Q = T x e1, the barycentric coordinates are u = T.P / det and
 * v = d.Q / det and the distance t = e2.Q / det.  A hit needs det != 0,
 * u >= 0, v >= 0, u + v <= 1 (edges belong to the triangle) and t in
 * (tmin, tmax]. */
int or_hit_triangle(const double v0[3], const double v1[3], const double v2[3],
                    const double o[3], const double d[3], double tmin, double tmax, double *t) {
  double e1[3], e2[3], P[3], T[3], Q[3];
  sub3(v1, v0, e1);
  sub3(v2, v0, e2);
  cross3(d, e2, P);
  double det = dot3(e1, P);
  if (det == 0.0) return 0;
  sub3(o, v0, T);
  double u = dot3(T, P) / det;
  if (!(u >= 0.0 && u <= 1.0)) return 0;
  cross3(T, e1, Q);
  double v = dot3(d, Q) / det;
  if (!(v >= 0.0 && u + v <= 1.0)) return 0;
  double tt = dot3(e2, Q) / det;
  if (!(tt > tmin && tt <= tmax)) return 0;
  *t = tt;
  return 1;
}

/* Geometric normal of primitive k at the hit point o + t d (not flipped). */
void or_normal(const or_scene *s, int64_t k, const double o[3], const double d[3], double t,
               double n[3]) {
  double P[3];
  for (int a = 0; a < 3; ++a) P[a] = o[a] + t * d[a];
  if (k < s->n_spheres) {
    const double *c = s->sph_center + 3 * k;
    double r = s->sph_radius[k];
    for (int a = 0; a < 3; ++a) n[a] = (P[a] - c[a]) / r;
  } else if (k >= s->n_spheres + s->n_cylinders) {
    /* triangle: the unit normal of its plane, e1 x e2 */
    int64_t m = k - s->n_spheres - s->n_cylinders;
    double e1[3], e2[3], c[3];
    sub3(s->tri_v1 + 3 * m, s->tri_v0 + 3 * m, e1);
    sub3(s->tri_v2 + 3 * m, s->tri_v0 + 3 * m, e2);
    cross3(e1, e2, c);
    normalize3(c, n);
  } else {
    int64_t m = k - s->n_spheres;
    cyl_frame cf;
    cylinder_frame(s->cyl_a + 3 * m, s->cyl_b + 3 * m, s->cyl_radius[m], &cf);
    double D[3];
    sub3(o, cf.a, D);
    double sax = dot3(D, cf.w) + t * dot3(d, cf.w);
    for (int a = 0; a < 3; ++a) n[a] = ((D[a] + t * d[a]) - sax * cf.w[a]) / cf.rho;
  }
}

/* One primitive test: 1 and its smallest root in (tmin, tmax] on a hit. */
static int hit_prim(const or_scene *s, int64_t k, const double o[3], const double d[3],
                    double tmin, double tmax, double *t, or_counters *cnt) {
  if (k < s->n_spheres) {
    if (cnt) cnt->sph_tests++;
    int h = or_hit_sphere(s->sph_center + 3 * k, s->sph_radius[k], o, d, tmin, tmax, t);
    if (h && cnt) cnt->sph_hits++;
    return h;
  }
  if (k >= s->n_spheres + s->n_cylinders) {
    int64_t m = k - s->n_spheres - s->n_cylinders;
    if (cnt) cnt->tri_tests++;
    int h = or_hit_triangle(s->tri_v0 + 3 * m, s->tri_v1 + 3 * m, s->tri_v2 + 3 * m, o, d, tmin,
                            tmax, t);
    if (h && cnt) cnt->tri_hits++;
    return h;
  }
  int64_t m = k - s->n_spheres;
  if (cnt) cnt->cyl_tests++;
  int h = or_hit_cylinder(s->cyl_a + 3 * m, s->cyl_b + 3 * m, s->cyl_radius[m], o, d, tmin,
                          tmax, t);
  if (h && cnt) cnt->cyl_hits++;
  return h;
}

/* ------------------------------------------------------------ uniform grid
 * Definition of the grid (shared by contract, not by code, with the GPU
 * build, which must produce the identical cell lists):
 *   primitive boxes: sphere [c - r, c + r]; cylinder [min(a,b) - rho,
 *     max(a,b) + rho]; triangle [min, max] of its vertices, per axis;
 *   scene box [Lo, Hi] = union of primitive boxes, widened on every side by
 *     pad = 1e-4 * m + 1e-6, m = largest extent of the union;
 *   resolution res_a = clamp(ceil(ext_a * cbrt(lambda * N / V)), 1, 512),
 *     ext = Hi - Lo, V = ext_x ext_y ext_z, N = primitive count;
 *   h_a = ext_a / res_a, inv_a = res_a / ext_a;
 *   cell of x on axis a: clamp(floor((x - Lo_a) * inv_a), 0, res_a - 1);
 *   insertion margin delta = h_min / 1024 + m / 65536;
 *   a primitive is listed in every cell (i, j, k) of the range spanned by
 *     its box widened by delta; a sphere additionally only where its centre
 *     lies within r of the cell box widened by delta (squared distance,
 *     per-axis gaps summed x, y, z);
 *   cell id = (k * res_y + j) * res_x + i; ids inside a cell ascending.
 * The margins make traversal conservative: a primitive hit within a cell's
 * reach is always listed there, so grid traversal returns exactly the brute
 * force answer (pinned by the tests). */
struct or_grid {
  double lo[3], hi[3], h[3], inv[3], delta;
  int32_t res[3];
  int64_t n_cells, n_refs;
  uint32_t *cell_begin;
  uint32_t *refs;
};

static void prim_box(const or_scene *s, int64_t k, double lo[3], double hi[3]) {
  if (k < s->n_spheres) {
    const double *c = s->sph_center + 3 * k;
    double r = s->sph_radius[k];
    for (int a = 0; a < 3; ++a) { lo[a] = c[a] - r; hi[a] = c[a] + r; }
  } else if (k >= s->n_spheres + s->n_cylinders) {
    int64_t m = k - s->n_spheres - s->n_cylinders;
    const double *v[3] = {s->tri_v0 + 3 * m, s->tri_v1 + 3 * m, s->tri_v2 + 3 * m};
    for (int a = 0; a < 3; ++a) {
      double mn = v[0][a], mx = v[0][a];
      for (int q = 1; q < 3; ++q) {
        mn = v[q][a] < mn ? v[q][a] : mn;
        mx = v[q][a] > mx ? v[q][a] : mx;
      }
      lo[a] = mn;
      hi[a] = mx;
    }
  } else {
    int64_t m = k - s->n_spheres;
    const double *A = s->cyl_a + 3 * m, *B = s->cyl_b + 3 * m;
    double rho = s->cyl_radius[m];
    for (int a = 0; a < 3; ++a) {
      double mn = A[a] < B[a] ? A[a] : B[a];
      double mx = A[a] < B[a] ? B[a] : A[a];
      lo[a] = mn - rho;
      hi[a] = mx + rho;
    }
  }
}

static int32_t cell_coord(const or_grid *g, int a, double x) {
  double f = floor((x - g->lo[a]) * g->inv[a]);
  if (!(f >= 0.0)) return 0;
  if (f > (double)(g->res[a] - 1)) return g->res[a] - 1;
  return (int32_t)f;
}

static int sphere_in_cell(const or_grid *g, const double c[3], double r, int32_t i, int32_t j,
                          int32_t k) {
  int32_t idx[3] = {i, j, k};
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    double cl = (g->lo[a] + (double)idx[a] * g->h[a]) - g->delta;
    double ch = (g->lo[a] + (double)(idx[a] + 1) * g->h[a]) + g->delta;
    double e = 0.0;
    if (c[a] < cl) e = cl - c[a];
    else if (c[a] > ch) e = c[a] - ch;
    d2 = d2 + e * e;
  }
  return d2 <= r * r;
}

/* calls visit(cell id) for every cell primitive k is listed in */
static int64_t prim_cells(const or_scene *s, const or_grid *g, int64_t k, uint32_t *out_cells) {
  double lo[3], hi[3];
  prim_box(s, k, lo, hi);
  int32_t c0[3], c1[3];
  for (int a = 0; a < 3; ++a) {
    c0[a] = cell_coord(g, a, lo[a] - g->delta);
    c1[a] = cell_coord(g, a, hi[a] + g->delta);
  }
  int64_t n = 0;
  for (int32_t kz = c0[2]; kz <= c1[2]; ++kz)
    for (int32_t jy = c0[1]; jy <= c1[1]; ++jy)
      for (int32_t ix = c0[0]; ix <= c1[0]; ++ix) {
        if (k < s->n_spheres &&
            !sphere_in_cell(g, s->sph_center + 3 * k, s->sph_radius[k], ix, jy, kz))
          continue;
        if (out_cells)
          out_cells[n] = (uint32_t)(((int64_t)kz * g->res[1] + jy) * g->res[0] + ix);
        ++n;
      }
  return n;
}

or_grid *or_grid_new(const or_scene *s, double lambda) {
  or_grid *g = (or_grid *)calloc(1, sizeof(or_grid));
  if (!g) return NULL;
  int64_t N = s->n_spheres + s->n_cylinders + s->n_triangles;
  if (lambda <= 0.0) lambda = 4.0;
  if (N == 0) {
    for (int a = 0; a < 3; ++a) { g->lo[a] = 0.0; g->hi[a] = 1.0; g->res[a] = 1; g->h[a] = 1.0; g->inv[a] = 1.0; }
    g->n_cells = 1;
    g->cell_begin = (uint32_t *)calloc(2, sizeof(uint32_t));
    g->refs = (uint32_t *)calloc(1, sizeof(uint32_t));
    return g;
  }
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t k = 0; k < N; ++k) {
    double bl[3], bh[3];
    prim_box(s, k, bl, bh);
    for (int a = 0; a < 3; ++a) {
      if (bl[a] < lo[a]) lo[a] = bl[a];
      if (bh[a] > hi[a]) hi[a] = bh[a];
    }
  }
  double m = 0.0;
  for (int a = 0; a < 3; ++a) if (hi[a] - lo[a] > m) m = hi[a] - lo[a];
  double pad = 1e-4 * m + 1e-6;
  double ext[3];
  for (int a = 0; a < 3; ++a) {
    g->lo[a] = lo[a] - pad;
    g->hi[a] = hi[a] + pad;
    ext[a] = g->hi[a] - g->lo[a];
  }
  double mext = ext[0];
  if (ext[1] > mext) mext = ext[1];
  if (ext[2] > mext) mext = ext[2];
  double V = ext[0] * ext[1] * ext[2];
  double kk = cbrt((lambda * (double)N) / V);
  double hmin = INFINITY;
  for (int a = 0; a < 3; ++a) {
    double r = ceil(ext[a] * kk);
    if (!(r >= 1.0)) r = 1.0;
    if (r > 512.0) r = 512.0;
    g->res[a] = (int32_t)r;
    g->h[a] = ext[a] / (double)g->res[a];
    g->inv[a] = (double)g->res[a] / ext[a];
    if (g->h[a] < hmin) hmin = g->h[a];
  }
  g->delta = hmin / 1024.0 + mext / 65536.0;
  g->n_cells = (int64_t)g->res[0] * g->res[1] * g->res[2];
  uint32_t *count = (uint32_t *)calloc((size_t)g->n_cells, sizeof(uint32_t));
  int64_t total = 0;
  int64_t maxc = 0;
  for (int64_t k = 0; k < N; ++k) {
    int64_t n = prim_cells(s, g, k, NULL);
    if (n > maxc) maxc = n;
  }
  uint32_t *tmp = (uint32_t *)malloc((size_t)(maxc > 0 ? maxc : 1) * sizeof(uint32_t));
  for (int64_t k = 0; k < N; ++k) {
    int64_t n = prim_cells(s, g, k, tmp);
    for (int64_t q = 0; q < n; ++q) count[tmp[q]]++;
    total += n;
  }
  g->n_refs = total;
  g->cell_begin = (uint32_t *)malloc((size_t)(g->n_cells + 1) * sizeof(uint32_t));
  g->refs = (uint32_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(uint32_t));
  uint32_t run = 0;
  for (int64_t c = 0; c < g->n_cells; ++c) { g->cell_begin[c] = run; run += count[c]; }
  g->cell_begin[g->n_cells] = run;
  memset(count, 0, (size_t)g->n_cells * sizeof(uint32_t));
  /* ascending k => ids ascend inside each cell */
  for (int64_t k = 0; k < N; ++k) {
    int64_t n = prim_cells(s, g, k, tmp);
    for (int64_t q = 0; q < n; ++q) {
      uint32_t c = tmp[q];
      g->refs[g->cell_begin[c] + count[c]++] = (uint32_t)k;
    }
  }
  free(tmp);
  free(count);
  return g;
}

void or_grid_free(or_grid *g) {
  if (!g) return;
  free(g->cell_begin);
  free(g->refs);
  free(g);
}

void or_grid_info(const or_grid *g, double lo[3], double hi[3], int32_t res[3], int64_t *n_refs) {
  for (int a = 0; a < 3; ++a) { lo[a] = g->lo[a]; hi[a] = g->hi[a]; res[a] = g->res[a]; }
  *n_refs = g->n_refs;
}

void or_grid_arrays(const or_grid *g, uint32_t *cell_begin, uint32_t *refs) {
  if (cell_begin) memcpy(cell_begin, g->cell_begin, (size_t)(g->n_cells + 1) * sizeof(uint32_t));
  if (refs && g->n_refs) memcpy(refs, g->refs, (size_t)g->n_refs * sizeof(uint32_t));
}

/* ------------------------------------------------------------- traversal
 * Nearest hit = lexicographic minimum of (t, id) over all primitives with a
 * root in (tmin, tmax]; any hit = whether such a primitive exists.  Brute
 * force is the definition; the grid walk (3D-DDA of Amanatides and Woo,
 * 1987) visits the cells along the ray in order and stops once the best hit
 * lies within the cell just visited. */
typedef struct {
  int any;
  int64_t skip;
  int found;
  double best_t;
  int64_t best_k;
} hit_state;

static void consider(const or_scene *s, int64_t k, const double o[3], const double d[3],
                     double tmin, double tmax, hit_state *hs, or_counters *cnt) {
  if (k == hs->skip) return;
  double t;
  if (!hit_prim(s, k, o, d, tmin, tmax, &t, cnt)) return;
  if (!hs->found || t < hs->best_t || (t == hs->best_t && k < hs->best_k)) {
    hs->found = 1;
    hs->best_t = t;
    hs->best_k = k;
  }
}

static double boundary_t(const or_grid *g, int a, int32_t idx, int step, const double o[3],
                         const double d[3]) {
  int32_t plane = step > 0 ? idx + 1 : idx;
  return ((g->lo[a] + (double)plane * g->h[a]) - o[a]) / d[a];
}

static void grid_walk(const or_scene *s, const or_grid *g, const double o[3], const double d[3],
                      double tmin, double tmax, hit_state *hs, or_counters *cnt) {
  double t0 = tmin, t1 = tmax;
  for (int a = 0; a < 3; ++a) {
    if (d[a] != 0.0) {
      double ta = (g->lo[a] - o[a]) / d[a];
      double tb = (g->hi[a] - o[a]) / d[a];
      if (ta > tb) { double x = ta; ta = tb; tb = x; }
      if (ta > t0) t0 = ta;
      if (tb < t1) t1 = tb;
    } else if (o[a] < g->lo[a] || o[a] > g->hi[a]) {
      return;
    }
  }
  if (t0 > t1) return;
  int32_t idx[3];
  int step[3];
  double tn[3];
  for (int a = 0; a < 3; ++a) {
    idx[a] = cell_coord(g, a, o[a] + t0 * d[a]);
    if (d[a] > 0.0) { step[a] = 1; tn[a] = boundary_t(g, a, idx[a], 1, o, d); }
    else if (d[a] < 0.0) { step[a] = -1; tn[a] = boundary_t(g, a, idx[a], -1, o, d); }
    else { step[a] = 0; tn[a] = INFINITY; }
  }
  for (;;) {
    if (cnt) cnt->cells++;
    int64_t c = ((int64_t)idx[2] * g->res[1] + idx[1]) * g->res[0] + idx[0];
    for (uint32_t q = g->cell_begin[c]; q < g->cell_begin[c + 1]; ++q) {
      consider(s, (int64_t)g->refs[q], o, d, tmin, tmax, hs, cnt);
      if (hs->any && hs->found) return;
    }
    int a = 0;
    if (tn[1] < tn[a]) a = 1;
    if (tn[2] < tn[a]) a = 2;
    double t_exit = tn[a] < t1 ? tn[a] : t1;
    if (!hs->any && hs->found && hs->best_t <= t_exit) return;
    if (tn[a] >= t1) return;
    idx[a] += step[a];
    if (idx[a] < 0 || idx[a] >= g->res[a]) return;
    tn[a] = boundary_t(g, a, idx[a], step[a], o, d);
  }
}

int or_trace(const or_scene *s, const or_grid *g, const double o[3], const double d[3],
             double tmin, double tmax, int64_t skip, int any_hit, double *t, int64_t *k,
             or_counters *cnt) {
  hit_state hs = {any_hit, skip, 0, INFINITY, -1};
  if (cnt) cnt->rays_traced++;
  if (g) {
    grid_walk(s, g, o, d, tmin, tmax, &hs, cnt);
  } else {
    int64_t N = s->n_spheres + s->n_cylinders + s->n_triangles;
    for (int64_t q = 0; q < N; ++q) {
      consider(s, q, o, d, tmin, tmax, &hs, cnt);
      if (any_hit && hs.found) break;
    }
  }
  if (t) *t = hs.best_t;
  if (k) *k = hs.best_k;
  return hs.found;
}

/* Brute force over the n primitive ids of order[], visited in that order.
 * The nearest hit is a lexicographic minimum, so the result must not depend
 * on the order (the tie-break pins visit duplicates in both directions). */
int or_trace_list(const or_scene *s, const int64_t *order, int64_t n, const double o[3],
                  const double d[3], double tmin, double tmax, int64_t skip, int any_hit,
                  double *t, int64_t *k) {
  hit_state hs = {any_hit, skip, 0, INFINITY, -1};
  for (int64_t q = 0; q < n; ++q) {
    consider(s, order[q], o, d, tmin, tmax, &hs, NULL);
    if (any_hit && hs.found) break;
  }
  if (t) *t = hs.best_t;
  if (k) *k = hs.best_k;
  return hs.found;
}

/* ------------------------------------------------------------- rendering
 * Per pixel: nearest hit of the camera ray; on a hit, the shading normal
 * faces the viewer; each light with N.L > 2^-40 casts one shadow ray; S AO rays
 * sample the cosine-weighted hemisphere with Philox uniforms keyed by
 * (pixel, sample); secondary rays start at the hit point with t in
 * (1e-4, ...] and skip the hit primitive when it was hit on its outside.
 * Colour = clamp(albedo * (rescale * sum_l I_l (N.L_l) V_l + skylight * AO)
 * + H, 0, 1) per channel, AO = unoccluded fraction (1 if no AO rays are
 * cast).  H is the optional Phong highlight (a shading option of the
 * renderer the paper drives, not used in its runs): rescale * sum_l I_l V_l
 * k_s max(0, R_l.V)^n over the lights with N.L_l > 2^-40, R_l the light
 * direction mirrored about N and V = -d the direction back to the eye; it is
 * white (not scaled by the albedo) and 0 when k_s = 0. */
#define OR_EPS 1e-4
/* A light counts, and casts its shadow ray, when N.L exceeds 2^-40 (reading
 * A8).  N.L at or below that is rounding noise of a light in the plane of the
 * surface (a flat face exactly perpendicular to a light): its term would add
 * at most 2^-40 of the light, invisible in the output, while its shadow ray
 * runs along the surface, where being blocked depends only on the rounding of
 * the hit point, in any precision. */
#define OR_LIGHT_MIN 0x1p-40

static void add_counters(or_counters *dst, const or_counters *src) {
  dst->pixels += src->pixels;
  dst->primary_rays += src->primary_rays;
  dst->hit_pixels += src->hit_pixels;
  dst->shadow_rays += src->shadow_rays;
  dst->ao_rays += src->ao_rays;
  dst->rays_traced += src->rays_traced;
  dst->cells += src->cells;
  dst->sph_tests += src->sph_tests;
  dst->sph_hits += src->sph_hits;
  dst->cyl_tests += src->cyl_tests;
  dst->cyl_hits += src->cyl_hits;
  dst->tri_tests += src->tri_tests;
  dst->tri_hits += src->tri_hits;
}

static float prim_albedo(const or_scene *s, int64_t k, int ch) {
  if (k < s->n_spheres) return s->sph_rgb[3 * k + ch];
  if (k >= s->n_spheres + s->n_cylinders)
    return s->tri_rgb[3 * (k - s->n_spheres - s->n_cylinders) + ch];
  return s->cyl_rgb[3 * (k - s->n_spheres) + ch];
}

/* Opacity of primitive k (1 = opaque; no array = all opaque). */
static double prim_opacity(const or_scene *s, int64_t k) {
  if (k < s->n_spheres) return s->sph_opacity ? (double)s->sph_opacity[k] : 1.0;
  if (k >= s->n_spheres + s->n_cylinders) {
    int64_t m = k - s->n_spheres - s->n_cylinders;
    return s->tri_opacity ? (double)s->tri_opacity[m] : 1.0;
  }
  return s->cyl_opacity ? (double)s->cyl_opacity[k - s->n_spheres] : 1.0;
}

/* One primary sample: the ray through image position (px, py) and the
 * clamped colour of what it sees.  Without transparency (max_layers <= 1)
 * that is one surface: its nearest hit, direct light with shadow rays and
 * AO.  With it, the ray composites up to max_layers surfaces front to back
 * (see or_render); hit id, t and masks are those of the first surface. */
typedef struct {
  double col[3];
  int hit;
  int64_t k;
  double t;
  uint32_t amask;
  int32_t aocc;
  uint8_t lmask;
} sample_out;

/* Colour of the surface hit at t by the ray (o, d): shading normal facing
 * the viewer, shadow rays, AO rays (counter word 1 = s + 2^16 * layer), the
 * optional highlight; clamped.  Returns the masks and the hit point,
 * normal and facing through the pointers. */
static void shade_surface(const or_scene *s, const or_grid *g, const or_params *p,
                          const double ldir[8][3], int64_t pid, uint32_t a, uint32_t layer,
                          const double o[3], const double d[3], double t, int64_t k,
                          double col[3], uint32_t *amask, int32_t *aocc, uint8_t *lmask,
                          double P[3], int *front_out, or_counters *loc) {
  const int S = p->ao_samples;
  const int do_ao = (S > 0 && p->skylight > 0.0);
  double N[3];
  or_normal(s, k, o, d, t, N);
  for (int c = 0; c < 3; ++c) P[c] = o[c] + t * d[c];
  int front = dot3(N, d) < 0.0;
  if (!front) { N[0] = -N[0]; N[1] = -N[1]; N[2] = -N[2]; }
  *front_out = front;
  int64_t skip = front ? k : -1;
  *amask = 0;
  *aocc = 0;
  *lmask = 0;
  double D[3] = {0.0, 0.0, 0.0};
  double Hs[3] = {0.0, 0.0, 0.0}; /* specular highlights (white, after albedo) */
  for (int l = 0; l < s->n_lights; ++l) {
    double c = dot3(N, ldir[l]);
    if (!(c > OR_LIGHT_MIN)) continue;
    loc->shadow_rays++;
    if (or_trace(s, g, P, ldir[l], OR_EPS, INFINITY, skip, 1, NULL, NULL, loc)) {
      *lmask |= (uint8_t)(1u << l);
    } else {
      for (int ch = 0; ch < 3; ++ch) D[ch] += (p->light_rescale * s->light_rgb[3 * l + ch]) * c;
      if (p->specular > 0.0) {
        /* Phong: mirror the light direction about N, compare with the
         * direction back to the eye, -d */
        double R[3], rv;
        for (int q = 0; q < 3; ++q) R[q] = 2.0 * c * N[q] - ldir[l][q];
        rv = -dot3(R, d);
        if (rv > 0.0) {
          double f = p->specular * pow(rv, p->shininess);
          for (int ch = 0; ch < 3; ++ch) Hs[ch] += (p->light_rescale * s->light_rgb[3 * l + ch]) * f;
        }
      }
    }
  }
  double ao = 1.0;
  if (do_ao) {
    for (int smp = 0; smp < S; ++smp) {
      double u1, u2, w[3];
      or_ao_uniforms_aa((uint32_t)pid, (uint32_t)smp + (layer << 16), p->view_id, a, p->seed,
                        &u1, &u2);
      or_ao_direction(N, u1, u2, w);
      loc->ao_rays++;
      if (or_trace(s, g, P, w, OR_EPS, p->ao_maxdist, skip, 1, NULL, NULL, loc)) {
        (*aocc)++;
        if (smp < 32) *amask |= 1u << smp;
      }
    }
    ao = (double)(S - *aocc) / (double)S;
  }
  for (int ch = 0; ch < 3; ++ch) {
    double v = (double)prim_albedo(s, k, ch) * (D[ch] + p->skylight * ao) + Hs[ch];
    col[ch] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
  }
}

static void shade_sample(const or_scene *s, const or_grid *g, const or_params *p,
                         const cam_basis *cb, const double ldir[8][3], int64_t pid, uint32_t a,
                         double px, double py, sample_out *r, or_counters *loc) {
  const int layers = p->max_layers > 1 ? p->max_layers : 1;
  double o[3], d[3];
  basis_ray_at(cb, px, py, o, d);
  loc->primary_rays++;
  r->hit = 0;
  r->k = -1;
  r->t = INFINITY;
  r->amask = 0;
  r->aocc = 0;
  r->lmask = 0;
  double acc[3] = {0.0, 0.0, 0.0};
  double T = 1.0; /* transmittance in front of the current surface */
  double tmin = 0.0;
  int64_t skip = -1;
  int layer = 0;
  for (; layer < layers; ++layer) {
    double t;
    int64_t k;
    if (!or_trace(s, g, o, d, tmin, INFINITY, skip, 0, &t, &k, loc)) break;
    double col[3], P[3];
    uint32_t am;
    int32_t ac;
    uint8_t lm;
    int front;
    shade_surface(s, g, p, ldir, pid, a, (uint32_t)layer, o, d, t, k, col, &am, &ac, &lm, P,
                  &front, loc);
    if (layer == 0) {
      loc->hit_pixels++;
      r->hit = 1;
      r->k = k;
      r->t = t;
      r->amask = am;
      r->aocc = ac;
      r->lmask = lm;
    }
    const double alpha = layers > 1 ? prim_opacity(s, k) : 1.0;
    for (int ch = 0; ch < 3; ++ch) acc[ch] += T * alpha * col[ch];
    T *= 1.0 - alpha;
    if (!(alpha < 1.0)) break;
    /* continue through the surface: from the hit point, on the same line;
     * an outward ray cannot re-enter the convex primitive it leaves, an
     * inward one meets its far side */
    for (int c = 0; c < 3; ++c) o[c] = P[c];
    tmin = OR_EPS;
    skip = front ? -1 : k;
  }
  /* what the last surface lets through (a miss, or the layer limit) is
   * background */
  for (int ch = 0; ch < 3; ++ch) r->col[ch] = acc[ch] + T * p->background[ch];
}

int or_render(const or_scene *s, const or_camera *cam, const or_params *p, const or_grid *g,
              int64_t n_pix, const int64_t *pix, double *rgb, int32_t *hit_id,
              uint32_t *ao_mask, int32_t *ao_occluded, uint8_t *light_mask, double *t_hit,
              or_counters *cnt, int32_t n_threads) {
  if (!s || !cam || !p || cam->width <= 0 || cam->height <= 0) return -1;
  if (s->n_lights < 0 || s->n_lights > 8 || p->ao_samples < 0 || p->aa_samples < 0) return -1;
  cam_basis cb;
  camera_basis(cam, &cb);
  double ldir[8][3];
  for (int l = 0; l < s->n_lights; ++l) normalize3(s->light_dir + 3 * l, ldir[l]);
  const uint32_t A = p->aa_samples > 1 ? (uint32_t)p->aa_samples : 1u;
  const int64_t total = (int64_t)cam->width * cam->height;
  if (!pix) n_pix = total;
  or_counters acc;
  memset(&acc, 0, sizeof acc);
#ifdef _OPENMP
  int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel num_threads(nt)
#endif
  {
    or_counters loc;
    memset(&loc, 0, sizeof loc);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
    for (int64_t q = 0; q < n_pix; ++q) {
      int64_t pid = pix ? pix[q] : q;
      int32_t i = (int32_t)(pid % cam->width), j = (int32_t)(pid / cam->width);
      loc.pixels++;
      sample_out first, cur;
      double sum[3] = {0.0, 0.0, 0.0};
      for (uint32_t a = 0; a < A; ++a) {
        double ox, oy;
        or_aa_offset((uint32_t)pid, a, p->view_id, p->seed, &ox, &oy);
        shade_sample(s, g, p, &cb, ldir, pid, a, (double)i + ox, (double)j + oy,
                     a == 0 ? &first : &cur, &loc);
        const sample_out *r = a == 0 ? &first : &cur;
        for (int ch = 0; ch < 3; ++ch) sum[ch] += r->col[ch];
      }
      if (rgb)
        for (int ch = 0; ch < 3; ++ch) rgb[3 * q + ch] = A == 1 ? sum[ch] : sum[ch] / (double)A;
      if (hit_id) hit_id[q] = (int32_t)first.k;
      if (ao_mask) ao_mask[q] = first.amask;
      if (ao_occluded) ao_occluded[q] = first.aocc;
      if (light_mask) light_mask[q] = first.lmask;
      if (t_hit) t_hit[q] = first.t;
    }
#ifdef _OPENMP
#pragma omp critical
#endif
    add_counters(&acc, &loc);
  }
  if (cnt) add_counters(cnt, &acc);
  return 0;
}

int32_t or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* 8-bit output of a frame.  The paper writes its frames as images (the
 * "Image I/O" phase, Table 5) without stating the conversion; the reading
 * here: clamp to [0, 1], scale by 255, round half up.  In double the product
 * of a float and 255 is exact, so the rounding is exact too. */
void or_quantize_rgb8(int64_t n, const float *in, uint8_t *out) {
  for (int64_t i = 0; i < n; ++i) {
    double v = (double)in[i];
    if (!(v > 0.0)) v = 0.0; /* also NaN */
    if (v > 1.0) v = 1.0;
    out[i] = (uint8_t)floor(v * 255.0 + 0.5);
  }
}

/* ---- Targa file (definition in oracle.h) -------------------------------- */

static int px_eq(const uint8_t *row, int32_t a, int32_t b) {
  return row[3 * a] == row[3 * b] && row[3 * a + 1] == row[3 * b + 1] &&
         row[3 * a + 2] == row[3 * b + 2];
}

/* length of the run of pixels equal to pixel i, starting at i */
static int32_t run_from(const uint8_t *row, int32_t w, int32_t i) {
  int32_t j = i + 1;
  while (j < w && px_eq(row, j, i)) ++j;
  return j - i;
}

static void put(uint8_t *out, int64_t *at, uint8_t v) {
  if (out) out[*at] = v;
  ++*at;
}

static void put_px(uint8_t *out, int64_t *at, const uint8_t *p) {
  put(out, at, p[2]); /* B */
  put(out, at, p[1]); /* G */
  put(out, at, p[0]); /* R */
}

/* one row's packets; counts bytes only when out is NULL */
static void tga_row(const uint8_t *row, int32_t w, uint8_t *out, int64_t *at) {
  int32_t i = 0;
  while (i < w) {
    const int32_t r = run_from(row, w, i);
    if (r >= 2) { /* run packets */
      for (int32_t left = r; left > 0;) {
        const int32_t c = left < 128 ? left : 128;
        put(out, at, (uint8_t)(0x80 | (c - 1)));
        put_px(out, at, row + 3 * (int64_t)i);
        left -= c;
      }
      i += r;
    } else { /* raw packets over the stretch of pixels that start no run */
      int32_t j = i;
      while (j < w && run_from(row, w, j) == 1) ++j;
      for (int32_t k = i; k < j;) {
        const int32_t c = j - k < 128 ? j - k : 128;
        put(out, at, (uint8_t)(c - 1));
        for (int32_t q = 0; q < c; ++q) put_px(out, at, row + 3 * (int64_t)(k + q));
        k += c;
      }
      i = j;
    }
  }
}

int64_t or_tga_encode(const uint8_t *rgb, int32_t w, int32_t h, uint8_t *out, int64_t cap) {
  if (w < 1 || w > 65535 || h < 1 || h > 65535) return -1;
  int64_t size = 18 + 26;
  for (int32_t y = 0; y < h; ++y) tga_row(rgb + (int64_t)y * w * 3, w, NULL, &size);
  if (!out || cap < size) return size;
  static const char sig[18] = "TRUEVISION-XFILE.";
  int64_t at = 0;
  const uint8_t head[18] = {0, 0, 10, 0, 0, 0, 0, 0, 0, 0, 0, 0,
                            (uint8_t)(w & 255), (uint8_t)(w >> 8), (uint8_t)(h & 255),
                            (uint8_t)(h >> 8), 24, 0x20};
  for (int k = 0; k < 18; ++k) put(out, &at, head[k]);
  for (int32_t y = 0; y < h; ++y) tga_row(rgb + (int64_t)y * w * 3, w, out, &at);
  for (int k = 0; k < 8; ++k) put(out, &at, 0);
  for (int k = 0; k < 18; ++k) put(out, &at, (uint8_t)sig[k]);
  return at;
}
