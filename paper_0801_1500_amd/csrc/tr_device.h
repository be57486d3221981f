// tr_device.h -- device data layout and small device helpers of the HIP path.
//
// Layout in HBM (one scene):
//   sph64  double4[n_s]  (cx, cy, cz, r)          FP64 copy (grid build, FP64 path, re-solve)
//   cylA64 double4[n_c]  (ax, ay, az, rho)
//   cylW64 double4[n_c]  (wx, wy, wz, L)           unit axis and length, w = (b - a) / L
//   cylB64 double4[n_c]  (bx, by, bz, 0)           second end point (grid rebuild)
//   sph32  float4[n_s + n_c]  (cx, cy, cz, r^2) rounded copies for the FP32 traversal: one
//                        16-byte load per sphere; then per cylinder its bounding
//                        sphere (axis midpoint, padded squared radius), which the
//                        walk tests first, like a sphere, at the same record offset
//   cylA32 float4[n_c], cylW32 float4[n_c]  (ax, ay, az, rho^2), (wx, wy, wz, L): two
//                        16-byte loads per cylinder
//   triA64/triB64/triC64 double4[n_t]  triangle vertices (FP64)
//   triV32, triE1_32, triE2_32 float4[n_t]  (v0, |e1 x e2|), e1, e2: three loads per triangle
//                        (FP32 positions are relative to org, the centre of the grid
//                        box: lo32 = lo - org, hi32 = hi - org, eye32 = eye - org)
//   albedo float4[N]     (r, g, b, opacity) by global id
//   cell_begin uint32[n_cells + 1], refs uint32[n_refs + 64]   the uniform grid
//   cellinfo CellInfo[n_cells] (list byte offset, first entry) of an occupied cell,
//                            or (-distance to the nearest occupied cell, bit 31 and
//                            eight 3-bit empty blocks ahead, by octant) of an empty one:
//                            the FP32 walk's view, one load
//   wrefs uint32[n_refs + occupied cells]  per occupied cell its references (16 x id,
//                        bit 0 set on the last) then -1
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trd {

// Traversal record of one grid cell (8 bytes, read with one load).  The FP32
// walk reads an occupied cell's references from its own list in wrefs: the
// cell's sorted references followed by -1, so the walk needs no end index.
struct CellInfo {
  int32_t a;  // occupied: byte offset of the cell's list in wrefs; empty: -(Chebyshev distance)
  int32_t c;  // occupied: the list's first entry (16 x id, bit 0: the only one); empty: bit 31
              // set, and in bits 3o..3o+2 the M of the empty block of 2M + 1 cells per
              // axis ahead of the cell for a ray in octant o (bit a of o: direction
              // negative on axis a)
};
static_assert(sizeof(CellInfo) == 8, "CellInfo is two words");

// A light counts, and casts its shadow ray, when N.L exceeds 2^-40: below
// that, N.L is rounding noise of a light in the plane of the surface, whose
// term is invisible and whose shadow ray runs along the surface.
constexpr double kLightMin = 0x1p-40;

// ------------------------------------------------------------ tile queue
// Workgroups are dispatched to the chip's 8 XCDs in turn (workgroup i on XCD
// i mod 8), and each XCD has an L2 of its own.  The wavefront kernel's tile
// queue deals the tiles out in stripes of consecutive tiles (a power of two,
// tuned; 64 by default), stripe s to XCD s mod 8, with one counter per XCD (each on a 128-byte line
// of its own), so tiles side by side -- which share cache lines of the frame
// and most of the cells their rays visit -- go through the same L2.  A wave
// drains its own XCD's counter first and then the others' in turn: the
// placement is a hint, and every tile is taken exactly once whatever the
// dispatch order.  The word after the counters' lines is the stall flag.
constexpr int kQueueXcds = 8;
constexpr int kQueueStride = 32;  // words from one counter to the next
constexpr int kQueueWords = (kQueueXcds + 1) * kQueueStride;

// ----------------------------------------------------------------- scene
struct SceneDev {
  int32_t n_s, n_c, n_t;  // ids: spheres, then cylinders, then triangles
  const double4 *sph64, *cylA64, *cylW64;
  const double4 *triA64, *triB64, *triC64;  // triangle vertices (FP64)
  const float4 *sph32, *cylA32, *cylW32;
  const float4 *triV32, *triE1_32, *triE2_32;  // (v0 - org, |e1 x e2|), (e1, 0), (e2, 0)
  const float4 *bvh;   // linear BVH records (4 float4 per internal node), or null
  int32_t bvh_n;       // primitives covered by the BVH (0 = none built)
  int32_t bvh_depth;   // internal nodes on the BVH's longest root-to-leaf path
  const float4 *albedo;
  const uint32_t *cell_begin, *refs;
  const uint32_t *wrefs;  // walk lists (see CellInfo)
  const CellInfo *cellinfo;  // per cell: (list byte offset, first entry) or (-distance, -1)
  double lo[3], hi[3], h[3], inv[3];
  double org[3];  // origin of the FP32 frame (centre of the grid box)
  float lo32[3], hi32[3], h32[3], inv32[3];
  float org32[3];  // (org - lo) * inv: FP32 cell coordinate of x is floor(x * inv32 + org32)
  int32_t res[3];
  // Bounding sphere about org holding every point of every primitive, its
  // radius padded by 2^-10 of itself: rb2_32 = the padded radius squared;
  // rguard2_32 = (2^10 x the padded radius) squared, the distance from org
  // up to which a ray origin's FP32 rounding stays below the padding.
  float rb2_32, rguard2_32;
};

// One render job: scene + camera + parameters + outputs + its tile range.
struct JobDev {
  SceneDev sc;
  double eye[3], f[3], r[3], u[3];
  double th, aspect;
  float eye32[3], f32[3], r32[3], u32[3];
  float th32, aspect32;
  int32_t W, H;
  int32_t S;            // AO rays per hit pixel (0 when AO is off)
  int32_t n_lights;
  double ldir[8][3];    // unit, toward the light
  double lcol[8][3];    // light_rescale * intensity
  float ldir32[8][3];
  float lcol32[8][3];
  double sky;           // skylight
  double ao_maxdist;
  double ks, shin;      // Phong highlight strength (0 = none) and exponent
  float sky32, ao_maxdist32;
  float ks32, shin32;
  uint32_t key0, key1, view_id;
  int32_t resolve;      // FP64 re-solve of near-grazing tests
  float bg[3];
  float *rgb;
  int32_t *hit_id;
  uint32_t *ao_mask;
  uint8_t *light_mask;
  // tiles: 64-pixel tiles of tile_w x (64 / tile_w) pixels, row-major
  int32_t tile_w, tile_h, tiles_x, tiles_y;
  int64_t tile_begin, tile_end;  // range rendered by this launch
  int64_t queue_begin;           // index of this job's first tile in the launch's tile queue
  int32_t scene_key;             // jobs with equal keys share one scene
  int32_t aa;                    // antialiasing sample index (0 = the pixel centre)
  int32_t layers;                // surfaces composited per primary ray (1 = opaque)
  int32_t pad3_;
};

// --------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 32x32->64-bit multiplies whose high halves are xored into the other two
// words with the round key; the key advances by two Weyl constants.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    // one 32x32->64 multiply gives both halves
    const uint64_t p0 = (uint64_t)M0 * c.x, p1 = (uint64_t)M1 * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint4 n;
    // three-input XORs in one instruction each (v_bitop3_b32, truth table 0x96)
    n.x = __builtin_amdgcn_bitop3_b32(hi1, c.y, k0, 0x96);
    n.y = lo1;
    n.z = __builtin_amdgcn_bitop3_b32(hi0, c.w, k1, 0x96);
    n.w = lo0;
    c = n;
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// AO sample s of primary sample aa: counter (pix, s, view, aa).  The two
// uniforms are the top 24 bits of words 0 and 1 (exact in float and double).
__device__ __forceinline__ void ao_uniform_bits(uint32_t pix, uint32_t s, uint32_t view,
                                                uint32_t aa, uint32_t k0, uint32_t k1,
                                                uint32_t &b1, uint32_t &b2) {
  uint4 x = philox4x32_10(make_uint4(pix, s, view, aa), k0, k1);
  b1 = x.x >> 8;
  b2 = x.y >> 8;
}

// Position of primary sample aa >= 1 inside its pixel square, as 24-bit
// fractions of a pixel (value = bits * 2^-24): counter (pix, aa, view,
// 0xFFFFFFFF), which no AO draw uses.  Sample 0 is the pixel centre.
__device__ __forceinline__ void aa_offset_bits(uint32_t pix, uint32_t aa, uint32_t view,
                                               uint32_t k0, uint32_t k1, uint32_t &bx,
                                               uint32_t &by) {
  uint4 x = philox4x32_10(make_uint4(pix, aa, view, 0xFFFFFFFFu), k0, k1);
  bx = x.x >> 8;
  by = x.y >> 8;
}

// Cosine-weighted hemisphere direction around unit n (Malley: uniform disc
// point lifted to the hemisphere), basis of Duff et al. (JCGT 2017).
// FP32 version: sin/cos of 2*pi*u2 by the hardware's revolution-scaled
// sine and cosine, which take u2 in [0, 1) directly.
__device__ __forceinline__ void ao_dir_f32(float nx, float ny, float nz, uint32_t b1, uint32_t b2,
                                           float &wx, float &wy, float &wz) {
  const float u1 = (float)b1 * (1.0f / 16777216.0f);
  const float u2 = (float)b2 * (1.0f / 16777216.0f);
  // hardware square roots (about 1 ulp; the arguments are >= 2^-24 or 0)
  const float rr = __builtin_amdgcn_sqrtf(u1);
  const float lx = rr * __builtin_amdgcn_cosf(u2);
  const float ly = rr * __builtin_amdgcn_sinf(u2);
  const float lz = __builtin_amdgcn_sqrtf(1.0f - u1);
  const float sg = __builtin_copysignf(1.0f, nz);
  const float a = -__builtin_amdgcn_rcpf(sg + nz);  // |sg + nz| is in [1, 2]
  const float b = nx * ny * a;
  const float tx = 1.0f + sg * nx * nx * a, ty = sg * b, tz = -sg * nx;
  const float bx = b, by = sg + ny * ny * a, bz = -ny;
  wx = lx * tx + ly * bx + lz * nx;
  wy = lx * ty + ly * by + lz * ny;
  wz = lx * tz + ly * bz + lz * nz;
}

// ------------------------------------------------------------- FP64 code
// Everything below rounds exactly as written (no fused multiply-adds), in
// every translation unit: the plain FP64 path reproduces the reference
// order of operations, and the FP32 kernel's FP64 re-solves and sign
// decisions must round like it.  A unit compiled with -ffp-contract=on
// restores it after this header (TR_CONTRACT_ON).  (-ffp-contract=fast
// would fuse at code generation regardless of this pragma.)
#pragma clang fp contract(off)

// FP64 version in the operation order of the plain double-precision path.
__device__ __forceinline__ void ao_dir_f64(const double n[3], uint32_t b1, uint32_t b2,
                                           double w[3]) {
  const double u1 = (double)b1 * (1.0 / 16777216.0);
  const double u2 = (double)b2 * (1.0 / 16777216.0);
  const double rr = sqrt(u1);
  const double phi = 6.283185307179586 * u2;
  double sn, cs;
  sincos(phi, &sn, &cs);
  const double lx = rr * cs, ly = rr * sn, lz = sqrt(1.0 - u1);
  const double sg = copysign(1.0, n[2]);
  const double a = -1.0 / (sg + n[2]);
  const double b = n[0] * n[1] * a;
  const double tx[3] = {1.0 + sg * n[0] * n[0] * a, sg * b, -sg * n[0]};
  const double bx[3] = {b, sg + n[1] * n[1] * a, -n[1]};
  w[0] = (lx * tx[0] + ly * bx[0]) + lz * n[0];
  w[1] = (lx * tx[1] + ly * bx[1]) + lz * n[1];
  w[2] = (lx * tx[2] + ly * bx[2]) + lz * n[2];
}

// --------------------------------------------------------------- camera
__device__ __forceinline__ double dot3d(const double a[3], const double b[3]) {
  return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

// FP64 primary ray through the centre of pixel (i, j); row 0 at the top.
// Primary ray of pixel (i, j) for the job's antialiasing sample: through the
// pixel centre for sample 0, else through the sample's point of the pixel
// square (i + x offset, j + y offset, exact in double).
__device__ __forceinline__ void primary_ray_f64(const JobDev &J, int32_t i, int32_t j,
                                                double o[3], double d[3]) {
  double px = (double)i + 0.5, py = (double)j + 0.5;
  if (J.aa != 0) {
    uint32_t bx, by;
    aa_offset_bits((uint32_t)(j * J.W + i), (uint32_t)J.aa, J.view_id, J.key0, J.key1, bx, by);
    px = (double)i + (double)bx * 0x1p-24;
    py = (double)j + (double)by * 0x1p-24;
  }
  const double x = (((2.0 * px) / (double)J.W) - 1.0) * J.th * J.aspect;
  const double y = (1.0 - (2.0 * py) / (double)J.H) * J.th;
  double v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) v[a] = (J.f[a] + x * J.r[a]) + y * J.u[a];
  const double n = sqrt(dot3d(v, v));
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    d[a] = v[a] / n;
    o[a] = J.eye[a];
  }
}

// ------------------------------------------------------- FP64 intersections
// Sphere (centre-to-ray perpendicular form, unit d): smallest root in
// (tmin, tmax], 1 on a hit.
__device__ __forceinline__ int hit_sphere_f64(const double4 s, const double o[3], const double d[3],
                                              double tmin, double tmax, double &t) {
  const double q[3] = {s.x - o[0], s.y - o[1], s.z - o[2]};
  const double b = dot3d(q, d);
  const double l[3] = {q[0] - b * d[0], q[1] - b * d[1], q[2] - b * d[2]};
  const double disc = s.w * s.w - dot3d(l, l);
  if (disc < 0.0) return 0;
  const double sq = sqrt(disc);
  const double t0 = b - sq, t1 = b + sq;
  if (t0 > tmin && t0 <= tmax) { t = t0; return 1; }
  if (t1 > tmin && t1 <= tmax) { t = t1; return 1; }
  return 0;
}

// Open cylinder: A t^2 + 2 B t + C = 0 on the perpendicular components, stable
// roots q/A and C/q, axial coordinate in [0, L].
__device__ __forceinline__ int hit_cylinder_f64(const double4 aa, const double4 ww, const double o[3],
                                                const double d[3], double tmin, double tmax,
                                                double &t) {
  const double w[3] = {ww.x, ww.y, ww.z};
  const double D[3] = {o[0] - aa.x, o[1] - aa.y, o[2] - aa.z};
  const double dw = dot3d(d, w);
  const double Dw = dot3d(D, w);
  double dp[3], Dp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dp[k] = d[k] - dw * w[k];
    Dp[k] = D[k] - Dw * w[k];
  }
  const double A = dot3d(dp, dp);
  const double B = dot3d(dp, Dp);
  const double C = dot3d(Dp, Dp) - aa.w * aa.w;
  if (A <= 1e-12 * dot3d(d, d)) return 0;
  const double disc = B * B - A * C;
  if (disc < 0.0) return 0;
  const double sq = sqrt(disc);
  const double qq = -(B + (B >= 0.0 ? sq : -sq));
  if (qq == 0.0) return 0;
  const double r0 = qq / A, r1 = C / qq;
  const double tl = r0 < r1 ? r0 : r1;
  const double th = r0 < r1 ? r1 : r0;
  if (tl > tmin && tl <= tmax) {
    const double s = Dw + tl * dw;
    if (s >= 0.0 && s <= ww.w) { t = tl; return 1; }
  }
  if (th > tmin && th <= tmax) {
    const double s = Dw + th * dw;
    if (s >= 0.0 && s <= ww.w) { t = th; return 1; }
  }
  return 0;
}

// Triangle (two-sided), Moller and Trumbore: e1 = B - A, e2 = C - A,
// P = d x e2, det = e1.P, T = o - A, Q = T x e1; u = T.P / det,
// v = d.Q / det, t = e2.Q / det; a hit needs det != 0, u >= 0, v >= 0,
// u + v <= 1 and t in (tmin, tmax].
__device__ __forceinline__ void cross3d(const double a[3], const double b[3], double r[3]) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ int hit_triangle_f64(const double4 A, const double4 B, const double4 C,
                                                const double o[3], const double d[3], double tmin,
                                                double tmax, double &t) {
  const double e1[3] = {B.x - A.x, B.y - A.y, B.z - A.z};
  const double e2[3] = {C.x - A.x, C.y - A.y, C.z - A.z};
  double P[3], Q[3];
  cross3d(d, e2, P);
  const double det = dot3d(e1, P);
  if (det == 0.0) return 0;
  const double T[3] = {o[0] - A.x, o[1] - A.y, o[2] - A.z};
  const double u = dot3d(T, P) / det;
  if (!(u >= 0.0 && u <= 1.0)) return 0;
  cross3d(T, e1, Q);
  const double v = dot3d(d, Q) / det;
  if (!(v >= 0.0 && u + v <= 1.0)) return 0;
  const double tt = dot3d(e2, Q) / det;
  if (!(tt > tmin && tt <= tmax)) return 0;
  t = tt;
  return 1;
}

// Unit normal e1 x e2 of triangle (A, B, C), not flipped.
__device__ __forceinline__ void triangle_normal_f64(const double4 A, const double4 B,
                                                    const double4 C, double n[3]) {
  const double e1[3] = {B.x - A.x, B.y - A.y, B.z - A.z};
  const double e2[3] = {C.x - A.x, C.y - A.y, C.z - A.z};
  double c[3];
  cross3d(e1, e2, c);
  const double m = sqrt(dot3d(c, c));
  n[0] = c[0] / m;
  n[1] = c[1] / m;
  n[2] = c[2] / m;
}

}  // namespace trd

#ifdef TR_CONTRACT_ON
#pragma clang fp contract(on)
#endif
