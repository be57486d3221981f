// render_wave.hip -- the FP32 persistent-wavefront ray kernel.
//
// Each workgroup is one 64-lane wave that lives for the whole launch and
// pulls 64-pixel tiles from a global tile counter (tiles of many frames may
// share one launch).  A wave keeps BANKS tiles in flight.  Their pixels own
// "slots" in LDS holding the shading state of a hit (point, normal, hit id,
// pending-ray count, occlusion bits).  Primary rays, light shadow rays and
// AO rays are all traced by the same grid-walking loop, one ray per lane:
//
//   finish   lanes whose ray ended hand in the result: a primary hit writes
//            its slot and queues the slot on the wave's LDS FIFO; a shadow or
//            AO ray sets its occlusion bit; the last ray of a pixel shades it
//            and writes the frame.  Lanes paused on a near-grazing test are
//            re-solved in FP64 just before this phase and resume;
//   refill   idle lanes are compacted (ballot + mbcnt) onto the next
//            secondary rays of the FIFO, then onto fresh primary rays, and a
//            new tile is fetched when a bank frees;
//   traverse every busy lane advances its ray by one unit of work per
//            iteration -- test one primitive reference, or step to the next
//            grid cell (3D-DDA) -- until too few lanes are busy.
//
// Secondary rays are not stored: a FIFO entry is a slot, and a lane rebuilds
// ray s of that slot from the slot's hit point and normal (the AO direction
// from Philox keyed by pixel and sample), so the queue costs one byte per
// pixel.  Intersection and shading run in FP32.  A sphere or cylinder test
// whose discriminant is within 2^-12 of its scale, or whose axial hit lies
// within 2^-12 L of a cylinder end, pauses the lane; the re-solve phase
// repeats it in FP64 with the FP64 primitive (primary rays regenerated in
// FP64 from their pixel) and the walk resumes.  Keeping all FP64 code out of
// the traversal loop keeps the loop's register footprint, and so the
// occupancy, that of the FP32 path.
// This unit fuses the multiply-adds of each expression (-ffp-contract=on);
// the FP64 helpers of tr_device.h keep their exact rounding (the header
// turns contraction off for them and back on after them).
#define TR_CONTRACT_ON 1
#include "tr_internal.h"

namespace {

using namespace trd;

constexpr float kEps = 1e-4f;
constexpr float kKappa = 1.0f / 4096.0f;
constexpr double kEpsD = 1e-4;

// Ray kinds.  kCont continues a primary ray through a transparent surface
// (nearest hit, from the hit point); kinds >= kShadow are any-hit rays.
enum : int32_t { kIdle = 0, kPrimary = 1, kCont = 2, kShadow = 3, kAO = 4 };
// lane state of the ray it holds (an idle lane counts as finished)
enum : int32_t { kRun = 0, kDone = 1, kPaused = 2 };

// Per-bank copy of the job fields secondary rays and shading need.
struct BankInfo {
  int32_t job, x0, y0, vw, n, done;
  int32_t vmagic;       // ceil(2^16 / vw): q / vw = (q * vmagic) >> 16 for q < 64
  int32_t W, H, S, n_lights;
  uint32_t key0, key1, view;
  int32_t aa;           // antialiasing sample index (0 = pixel centre)
  float maxd, sky;
  float ks, shin;       // Phong highlight strength (0 = none) and exponent
  int32_t layers;       // surfaces composited per primary ray (1 = opaque)
  float eye[3], f[3], r[3], u[3], th, aspect;  // FP32 camera
  float rw2, rh2;       // 2 / W, 2 / H
  float rS;             // 1 / S (0 when S = 0)
  float bg[3];
  float *rgb;
  int32_t *hit_id;
  uint32_t *ao_mask;
  uint8_t *light_mask;
  float ldir[8][3];
  float lcol[8][3];
};

// Bank record of a lane's slot (bank index < BANKS): the byte offset by the
// 24-bit multiplier (the compiler would use a slow 32-bit multiply).
template <int BANKS>
__device__ __forceinline__ BankInfo &bank_of(BankInfo (&bank)[BANKS], int32_t bk) {
  return *(BankInfo *)((char *)bank + __umul24((uint32_t)bk, (uint32_t)sizeof(BankInfo)));
}

// Pixel of slot offset q (0..63) in a bank's tile: row-major over vw columns.
__device__ __forceinline__ void bank_pixel(const BankInfo &B, int32_t q, int32_t &x, int32_t &y) {
  const int32_t qy = (int32_t)(__umul24((uint32_t)q, (uint32_t)B.vmagic) >> 16);
  x = B.x0 + q - (int32_t)__umul24((uint32_t)qy, (uint32_t)B.vw);
  y = B.y0 + qy;
}

// Write bank b's finished tile to the frame from the colours its slots hold
// in px, py, pz.  Lane l stores floats l, l + 64, l + 128 of the tile taken
// row by row, so each tile row is one contiguous run of 12 vw bytes written
// together (one 12-byte store per pixel as pixels finish, spread over many
// rounds, leaves the L2 to write partly filled lines back several times).
template <typename LdsT>
__device__ __forceinline__ void write_tile(const LdsT &L, int32_t b, int32_t lane) {
  const BankInfo &B = L.bank[b];
  const int32_t nf = 3 * B.n;
  float *const base = B.rgb + ((int64_t)B.y0 * B.W + B.x0) * 3;
  for (int32_t f = lane; f < nf; f += 64) {
    const int32_t q = f / 3, c = f - 3 * q;  // pixel of the bank, colour channel
    const int32_t qy = (int32_t)(__umul24((uint32_t)q, (uint32_t)B.vmagic) >> 16);
    const int32_t qx = q - (int32_t)__umul24((uint32_t)qy, (uint32_t)B.vw);
    const int32_t s = b * 64 + q;
    const float v = c == 0 ? L.px[s] : (c == 1 ? L.py[s] : L.pz[s]);
    base[((int64_t)qy * B.W + qx) * 3 + c] = v;
  }
}

constexpr int kStack = trh::kBvhStack;  // BVH traversal stack entries per lane

template <int BANKS, bool TRANS, bool BVH>
struct Lds {
  static constexpr int NS = BANKS * 64;
  static constexpr int NT = TRANS ? NS : 1;  // transparency state only when compositing
  float px[NS], py[NS], pz[NS];
  float nx[NS], ny[NS], nz[NS];
  int32_t prim[NS];     // hit primitive (record offset)
  // Secondary rays not yet finished (bits 0-30), and in bit 31 whether the
  // rays leave the surface outward (then they skip prim; from inside they
  // take only its far root): see slot_skip.  Decrements never reach bit 31.
  int32_t pend[NS];
  // Lights with N.L > 0 (bits 0-7), lights occluded (8-15) and AO rays
  // occluded (16-31: at most 65535), updated by atomics on disjoint bits.
  uint32_t acc[NS];
  uint32_t aomask[NS];  // AO sample s occluded (bit s < 32; the optional output)
  // FIFO of slots with secondary rays to issue, one word each: slot (bits
  // 0-7), lights with N.L > 0 (8-11), continuation (12), AO rays (16-31);
  // the refill reads an entry with one load
  uint32_t fifo[NS];
  BankInfo bank[BANKS];
  uint32_t cnt[24];
  // compositing across surfaces: colour so far, transmittance in front of the
  // current surface, its index, and whether the FIFO entry is a continuation
  float acc_r[NT], acc_g[NT], acc_b[NT], trn[NT];
  uint8_t layer[NT];
  // BVH walk: per lane a stack of node / leaf items, entry e at e * 64 + lane
  int32_t stk[BVH ? 64 * kStack : 1];
  // the skip rule of the slot's secondary rays (see Ray::skip)
  __device__ __forceinline__ int32_t slot_skip(int32_t slot) const {
    const int32_t k = prim[slot];
    return pend[slot] < 0 ? k : -2 - k;
  }
};

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Lane mask of p over the wave (scalar compare result, no VGPR round trip).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

// floor(x) as an integer in one instruction (the compiler emits floor + convert)
__device__ __forceinline__ int32_t cvt_floor(float x) {
  int32_t r;
  asm volatile("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// IEEE min of two floats without the operand canonicalisation the compiler
// adds to fminf when it cannot see where a value came from
__device__ __forceinline__ float vminf(float a, float b) {
  float r;
  asm volatile("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// a * b + c on the 24-bit multiplier (a, b < 2^24; b wave-uniform)
__device__ __forceinline__ uint32_t mad24(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm volatile("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
  return r;
}

// median of three: clamp of x to [lo, hi] when lo <= hi
__device__ __forceinline__ int32_t med3i(int32_t x, int32_t lo, int32_t hi) {
  int32_t r;
  asm volatile("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
  return r;
}
__device__ __forceinline__ float sqrtf_fast(float x) { return __builtin_amdgcn_sqrtf(x); }

// Per-lane ray and traversal state.
struct Ray {
  float ox, oy, oz, dx, dy, dz;
  float tmin, tmax;  // t interval of accepted hits (tmax is folded into t1 at setup)
  float t1;          // exit of the grid box clipped to tmax: every primitive lies
                     // inside the box, so hits are accepted in (tmin, t1]
  float bx, by, bz;  // the walk enters cell i of axis a at t = b_a + i * h_a
  float hx, hy, hz;
  int32_t cx, cy, cz;
  int32_t sx, sy, sz;  // minus the step signs (-1, 0, 1 for d > 0, = 0, < 0)
  int32_t o3;          // 3 x the octant of d (bit a set for d_a < 0): the position of
                       // its empty block ahead in an empty cell's record
  int32_t rc;          // byte offset of the cursor in the cell's walk list; -(distance) in an empty cell
  int32_t nk;          // the entry at rc: the next primitive (record offset, 16 x id;
                       // bit 0 set on the cell's last), or negative: an empty cell's
                       // second record word, or bit 31 alone once the cell is done
                       // (loaded ahead)
  float bt;            // best t; before a hit the float just above t1, so the
                       // walk ends at min(t1, best t) with one compare
  int32_t bk;          // best primitive, record offset (-1 = none)
  int32_t skip;         // k >= 0: never report k; -2 - k: k is the ray's own surface,
                        // left from inside; -1: none (k: record offsets)
};

// Scene fields used by the traversal, loaded (wave-uniform) from the job
// table at the start of each phase.
// Hot pointers are in the global address space so loads compile to global
// (not flat) instructions with a scalar base.
#define TR_GLOBAL __attribute__((address_space(1)))
#define TR_CONST __attribute__((address_space(4)))
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef uint32_t vu2 __attribute__((ext_vector_type(2)));
// A primitive's record offset: 16 x its global id, the byte offset of its
// 16-byte FP32 records (the form the walk lists store ids in).
constexpr int kRecShift = 4;
static_assert(sizeof(vf4) == (1 << kRecShift), "FP32 primitive records are 16 bytes");
struct SceneHot {
  const TR_GLOBAL uint32_t *refs;
  const TR_GLOBAL trd::CellInfo *cellinfo;
  const TR_GLOBAL vf4 *sph32, *cylA32, *cylW32, *albedo;
  const TR_GLOBAL vf4 *triV32, *triE1_32, *triE2_32;
  const TR_GLOBAL vf4 *bvh;  // 4 records per internal node
  int32_t bvh_n;             // primitives in the BVH
  // Inside this kernel a primitive is named by its record offset, 16 x its
  // global id (every FP32 record is 16 bytes; the walk lists store ids that
  // way), so an id addresses its record without a multiply: spheres are the
  // offsets below s_end, cylinders those below c_end, triangles the rest.
  int32_t s_end;  // 16 n_s
  int32_t c_end;  // 16 (n_s + n_c)
  int32_t res[3];
  float lo32[3], hi32[3], inv32[3], h32[3];
  float org32[3];  // cell coordinate of the FP32 frame's origin
  float rb2, rguard2;  // bounding sphere (see SceneDev)
};

// The job table is read-only for the whole launch, so it is read through the
// constant address space: with a wave-uniform job index the fields are scalar
// loads and stay in SGPRs.
__device__ __forceinline__ SceneHot load_hot(const JobDev *Jg) {
  const TR_CONST JobDev *J = (const TR_CONST JobDev *)Jg;
  SceneHot H;
  H.refs = (const TR_GLOBAL uint32_t *)J->sc.wrefs;
  H.cellinfo = (const TR_GLOBAL trd::CellInfo *)J->sc.cellinfo;
  H.sph32 = (const TR_GLOBAL vf4 *)J->sc.sph32;
  H.cylA32 = (const TR_GLOBAL vf4 *)J->sc.cylA32;
  H.cylW32 = (const TR_GLOBAL vf4 *)J->sc.cylW32;
  H.albedo = (const TR_GLOBAL vf4 *)J->sc.albedo;
  H.triV32 = (const TR_GLOBAL vf4 *)J->sc.triV32;
  H.triE1_32 = (const TR_GLOBAL vf4 *)J->sc.triE1_32;
  H.triE2_32 = (const TR_GLOBAL vf4 *)J->sc.triE2_32;
  H.bvh = (const TR_GLOBAL vf4 *)J->sc.bvh;
  H.bvh_n = J->sc.bvh_n;
  H.s_end = J->sc.n_s << kRecShift;
  H.c_end = (J->sc.n_s + J->sc.n_c) << kRecShift;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    H.res[q] = J->sc.res[q];
    H.lo32[q] = J->sc.lo32[q];
    H.hi32[q] = J->sc.hi32[q];
    H.inv32[q] = J->sc.inv32[q];
    H.h32[q] = J->sc.h32[q];
    H.org32[q] = J->sc.org32[q];
  }
  H.rb2 = J->sc.rb2_32;
  H.rguard2 = J->sc.rguard2_32;
  return H;
}

// base[i] addressed by a 32-bit byte offset from a wave-uniform base (one
// global load with a scalar base, no 64-bit address arithmetic).  The host
// bounds every array this is used on below 2^32 bytes.
template <class T>
__device__ __forceinline__ T ldg(const TR_GLOBAL T *base, uint32_t i) {
  return *(const TR_GLOBAL T *)((const TR_GLOBAL char *)base + i * (uint32_t)sizeof(T));
}
// base at a byte offset (no scaling)
template <class T>
__device__ __forceinline__ T ldgb(const TR_GLOBAL T *base, uint32_t off) {
  return *(const TR_GLOBAL T *)((const TR_GLOBAL char *)base + off);
}

// Colour of a finished hit pixel from its slot: the lights whose shadow rays
// got through, the unoccluded share of its AO rays, its albedo and the
// optional highlight, clamped (the first surface, or the current one when
// compositing).  alpha: the primitive's opacity.
template <typename LdsT>
__device__ __forceinline__ void shade_slot(const LdsT &L, const BankInfo &B, int32_t slot,
                                           int32_t k, const TR_GLOBAL vf4 *albedo, float &cr,
                                           float &cg, float &cb, float &alpha) {
  const float Nx = L.nx[slot], Ny = L.ny[slot], Nz = L.nz[slot];
  const uint32_t ac = L.acc[slot];
  const uint32_t lv = ac & 0xFFu, lm = (ac >> 8) & 0xFFu;
  float Dr = 0.0f, Dg = 0.0f, Db = 0.0f;
  float Hr = 0.0f, Hg = 0.0f, Hb = 0.0f;  // Phong highlight (white, after the albedo)
  for (int l = 0; l < B.n_lights; ++l) {
    if (!((lv >> l) & 1u) || ((lm >> l) & 1u)) continue;
    const float cl = Nx * B.ldir[l][0] + Ny * B.ldir[l][1] + Nz * B.ldir[l][2];
    Dr += B.lcol[l][0] * cl;
    Dg += B.lcol[l][1] * cl;
    Db += B.lcol[l][2] * cl;
    if (B.ks > 0.0f) {
      // light direction mirrored about N, against the way back to the eye
      const float vx = B.eye[0] - L.px[slot], vy = B.eye[1] - L.py[slot],
                  vz = B.eye[2] - L.pz[slot];
      const float rv = ((2.0f * cl * Nx - B.ldir[l][0]) * vx +
                        (2.0f * cl * Ny - B.ldir[l][1]) * vy +
                        (2.0f * cl * Nz - B.ldir[l][2]) * vz) *
                       __builtin_amdgcn_rsqf(vx * vx + vy * vy + vz * vz);
      if (rv > 0.0f) {
        // rv^n as 2^(n log2 rv) on the hardware log and exp (about
        // 1 ulp each; rv <= 1, so the error is ~ n |log2 rv| ulp)
        const float f = B.ks * __builtin_amdgcn_exp2f(B.shin * __builtin_amdgcn_logf(rv));
        Hr += B.lcol[l][0] * f;
        Hg += B.lcol[l][1] * f;
        Hb += B.lcol[l][2] * f;
      }
    }
  }
  float ao = 1.0f;
  if (B.S > 0) ao = (float)(B.S - (int32_t)(ac >> 16)) * B.rS;
  const vf4 alb = ldgb(albedo, (uint32_t)k);  // (k: record offset)
  const float sk = B.sky * ao;
  cr = fminf(fmaxf(alb.x * (Dr + sk) + Hr, 0.0f), 1.0f);
  cg = fminf(fmaxf(alb.y * (Dg + sk) + Hg, 0.0f), 1.0f);
  cb = fminf(fmaxf(alb.z * (Db + sk) + Hb, 0.0f), 1.0f);
  alpha = alb.w;
}

// Opaque rendering: a bank's pixels are shaded when its last one finishes,
// one lane per pixel (shading as pixels finish would run the shading code
// for the few lanes that finish in each round); the colours then wait in the
// slots' hit-point words for write_tile, and hit ids and masks go out here.
template <typename LdsT>
__device__ __forceinline__ void shade_tile(LdsT &L, int32_t b, int32_t lane,
                                           const TR_GLOBAL vf4 *albedo) {
  const BankInfo &B = L.bank[b];
  if (lane < B.n) {
    const int32_t slot = b * 64 + lane;
    const int32_t k = L.prim[slot];  // -1: the primary ray missed
    float cr = B.bg[0], cg = B.bg[1], cb = B.bg[2], alpha;
    if (k >= 0) shade_slot(L, B, slot, k, albedo, cr, cg, cb, alpha);
    if (B.hit_id || B.ao_mask || B.light_mask) {
      int32_t x, y;
      bank_pixel(B, lane, x, y);
      const int64_t pid = (int64_t)y * B.W + x;
      if (B.hit_id) B.hit_id[pid] = k >> kRecShift;  // the global id (-1 stays -1)
      if (B.ao_mask) B.ao_mask[pid] = k >= 0 ? L.aomask[slot] : 0u;
      if (B.light_mask) B.light_mask[pid] = k >= 0 ? (uint8_t)(L.acc[slot] >> 8) : (uint8_t)0;
    }
    L.px[slot] = cr;
    L.py[slot] = cg;
    L.pz[slot] = cb;
  }
  __syncthreads();
}


__device__ __forceinline__ void load_cell(Ray &R, const SceneHot &S) {
  // res <= 512 per axis: the products fit the 24-bit multiplier
  const uint32_t cell = mad24(mad24((uint32_t)R.cz, (uint32_t)S.res[1], (uint32_t)R.cy),
                              (uint32_t)S.res[0], (uint32_t)R.cx);
  // one 8-byte load: byte offset of the cell's list in wrefs (or -distance)
  // and its first entry (-1 if empty)
  const vu2 ci = ldg((const TR_GLOBAL vu2 *)S.cellinfo, cell);
  R.rc = (int32_t)ci.x;
  R.nk = (int32_t)ci.y;
}

// Clip to the grid box and to the scene's bounding sphere, and position the
// walk at the entry cell.  Returns false when the ray misses either.
__device__ __forceinline__ bool ray_setup(Ray &R, const SceneHot &S) {
  const float ix = rcpf(R.dx), iy = rcpf(R.dy), iz = rcpf(R.dz);
  // slab times of the box's lower and upper planes on each axis
  const float ax = (S.lo32[0] - R.ox) * ix, bx = (S.hi32[0] - R.ox) * ix;
  const float ay = (S.lo32[1] - R.oy) * iy, by = (S.hi32[1] - R.oy) * iy;
  const float az = (S.lo32[2] - R.oz) * iz, bz = (S.hi32[2] - R.oz) * iz;
  float t0 = fmaxf(R.tmin, fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fminf(az, bz)));
  float t1 = fminf(R.tmax, fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz)));
  {
    // Every hit lies inside the bounding sphere about the FP32 frame's
    // origin (the box centre), so the walk runs only over the ray's chord of
    // it: the box's corners beyond the sphere hold nothing, and escaping
    // shadow and AO rays would otherwise cross them by empty-space jumps.
    // Closest-approach form (as the sphere test): b = t of the closest point,
    // l = its offset, chord half-length sqrt(rb^2 - |l|^2), with no
    // cancellation of the origin's distance.  The padding (2^-10 of the
    // radius) covers the FP32 rounding while the origin lies within 2^10
    // radii of the centre (|o|^2 = b^2 + |l|^2); farther out the box alone
    // clips.  (d is a unit vector.)
    const float b = -(R.ox * R.dx + R.oy * R.dy + R.oz * R.dz);
    const float lx = fmaf(b, R.dx, R.ox), ly = fmaf(b, R.dy, R.oy), lz = fmaf(b, R.dz, R.oz);
    const float ll = lx * lx + ly * ly + lz * lz;
    const float disc = S.rb2 - ll;
    if (fmaf(b, b, ll) < S.rguard2) {
      const float sq = sqrtf_fast(fmaxf(disc, 0.0f));
      t0 = fmaxf(t0, b - sq);
      t1 = disc >= 0.0f ? fminf(t1, b + sq) : -INFINITY;
    }
  }
  R.t1 = t1;
  R.bk = -1;
  if (!(t0 <= t1)) return false;
  R.bt = __int_as_float(__float_as_int(t1) + 1);  // (0 <= t1 < inf here)
  const float ex = fmaf(t0, R.dx, R.ox), ey = fmaf(t0, R.dy, R.oy), ez = fmaf(t0, R.dz, R.oz);
  R.cx = min(max(cvt_floor((ex - S.lo32[0]) * S.inv32[0]), 0), S.res[0] - 1);
  R.cy = min(max(cvt_floor((ey - S.lo32[1]) * S.inv32[1]), 0), S.res[1] - 1);
  R.cz = min(max(cvt_floor((ez - S.lo32[2]) * S.inv32[2]), 0), S.res[2] - 1);
  const int32_t sx = R.dx > 0.0f ? 1 : (R.dx < 0.0f ? -1 : 0);
  const int32_t sy = R.dy > 0.0f ? 1 : (R.dy < 0.0f ? -1 : 0);
  const int32_t sz = R.dz > 0.0f ? 1 : (R.dz < 0.0f ? -1 : 0);
  R.sx = -sx;
  R.sy = -sy;
  R.sz = -sz;
  R.o3 = 3 * ((sx < 0 ? 1 : 0) | (sy < 0 ? 2 : 0) | (sz < 0 ? 4 : 0));
  // Plane of the grid crossed when the walk enters cell i of axis a: at
  // b_a + i * h_a, with b_a taken one cell up for negative steps (the plane
  // between cells i and i + 1).  An axis with d_a = 0 gets b_a = inf, h_a = 0:
  // its plane is never the next one.
  R.hx = sx ? S.h32[0] * ix : 0.0f;
  R.hy = sy ? S.h32[1] * iy : 0.0f;
  R.hz = sz ? S.h32[2] * iz : 0.0f;
  R.bx = sx > 0 ? ax : (sx < 0 ? ax + R.hx : INFINITY);
  R.by = sy > 0 ? ay : (sy < 0 ? ay + R.hy : INFINITY);
  R.bz = sz > 0 ? az : (sz < 0 ? az + R.hz : INFINITY);
  load_cell(R, S);
  return true;
}

// BVH walk state in the ray's grid fields: hx/hy/hz = 1/d, cx = stack depth,
// rc = node to visit (-1 none), nk = primitive to test (-1 none); t1 = tmax.
__device__ __forceinline__ bool bvh_setup(Ray &R, const SceneHot &S) {
  R.hx = rcpf(R.dx);
  R.hy = rcpf(R.dy);
  R.hz = rcpf(R.dz);
  R.t1 = R.tmax;
  R.bt = INFINITY;
  R.bk = -1;
  R.cx = 0;
  R.rc = S.bvh_n >= 2 ? 0 : -1;
  R.nk = S.bvh_n == 1 ? 0 : -1;
  return S.bvh_n > 0;
}

// Sign decisions of a triangle hit in FP64, in the reference's order of
// operations: the unit normal e1 x e2 from the FP64 vertices, its facing
// against the ray (a primary ray regenerated in FP64 from its pixel; a
// continuation ray's FP32 direction promoted), N.L > 0 per light, and the
// sign of N.z, which picks the AO basis.  The FP32 normal becomes the FP64
// one rounded, so every sign (of a zero too) is the FP64 one.
__device__ __forceinline__ void tri_signs_f64(const JobDev &J, int32_t m, bool primary, int32_t px,
                                              int32_t py, float dx, float dy, float dz, float &Nx,
                                              float &Ny, float &Nz, bool &front, uint32_t &lv) {
  const SceneDev &S = J.sc;
  double n[3], o[3], d[3];
  triangle_normal_f64(S.triA64[m], S.triB64[m], S.triC64[m], n);
  if (primary) {
    primary_ray_f64(J, px, py, o, d);
  } else {
    const double v[3] = {(double)dx, (double)dy, (double)dz};
    const double nv = sqrt(dot3d(v, v));
    d[0] = v[0] / nv;
    d[1] = v[1] / nv;
    d[2] = v[2] / nv;
  }
  front = dot3d(n, d) < 0.0;
  if (!front) {
    n[0] = -n[0];
    n[1] = -n[1];
    n[2] = -n[2];
  }
  uint32_t m_l = 0;
  for (int l = 0; l < J.n_lights; ++l)
    if (dot3d(n, J.ldir[l]) > kLightMin) m_l |= 1u << l;
  lv = m_l;
  Nx = (float)n[0];
  Ny = (float)n[1];
  Nz = (float)n[2];
}

// FP64 test of primitive k (global id) against the ray: 1 and its root.
template <bool TRI>
__device__ __forceinline__ int hit_prim_f64(const SceneDev &S, int32_t k, const double o[3],
                                            const double d[3], double tmin, double tmax, double &t) {
  if (k < S.n_s) return hit_sphere_f64(S.sph64[k], o, d, tmin, tmax, t);
  if (TRI && k >= S.n_s + S.n_c) {
    const int32_t m = k - S.n_s - S.n_c;
    return hit_triangle_f64(S.triA64[m], S.triB64[m], S.triC64[m], o, d, tmin, tmax, t);
  }
  return hit_cylinder_f64(S.cylA64[k - S.n_s], S.cylW64[k - S.n_s], o, d, tmin, tmax, t);
}

struct WaveArgs {
  const JobDev *jobs;
  int32_t n_jobs;
  int64_t n_tiles;
  uint32_t *tile_counter;
  uint64_t *stats;
  int32_t tile_w, refill_below;
  int32_t stripe_log2;  // tiles per stripe of the tile queue, log2
};

__device__ __forceinline__ int32_t find_job(const TR_CONST JobDev *jobs, int32_t n, int64_t tile) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (jobs[mid].queue_begin <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int BANKS, bool RESOLVE, bool COUNT, bool TRANS, bool TRI, bool BVH>
// Occupancy targets: 5 waves per SIMD for the plain two-bank kernel (96
// VGPRs); compositing adds LDS state that allows fewer waves anyway, and the
// triangle test needs more registers than 96 without spilling; the BVH
// walk's per-lane stacks (12 KB of LDS per wave) leave room for 2.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(BVH ? 2 : (TRANS ? 3 : (BANKS == 2 && !COUNT && !TRI ? 5 : 4))))) void k_render_wave(const WaveArgs A) {
  __shared__ Lds<BANKS, TRANS, BVH> L;
  constexpr int NS = BANKS * 64;
  constexpr int kMinIters = 2;
  const int32_t lane = threadIdx.x;
  const int32_t TW = A.tile_w;
  const int32_t TH = 64 / TW;
  if (lane < 24) L.cnt[lane] = 0;

  // ---- wave-uniform control state
  int32_t q_head = 0, q_tail = 0, head_issued = 0;
  int32_t issue_bank = -1, issue_next = 0;
  uint32_t bank_busy = 0;
  bool tiles_left = true;
  int32_t xq = (int32_t)(blockIdx.x % kQueueXcds);  // tile queue drawn from: this XCD's first
  int32_t xq_left = kQueueXcds;                       // queues not yet found drained
  int64_t held_tile = -1;
  int32_t held_job = 0, held_key = -1;
  int32_t cur_key = -1;   // scene loaded in this wave
  int32_t scene_job = 0;  // a job whose scene is the current one
  int32_t idle_rounds = 0;
  bool stalled = false;  // left with work outstanding (reported in the stats)

  // ---- counters (wave-uniform)
  uint64_t c_rays = 0;
  uint32_t l_cells = 0, l_st = 0, l_sh = 0, l_ct = 0, l_ch = 0, l_res = 0, l_jumps = 0;  // per lane
  uint32_t l_tt = 0, l_th = 0, l_ovf = 0;
  uint32_t l_rs = 0, l_rc = 0, l_rt = 0, l_rn = 0;  // re-solves: sphere, cylinder, triangle, nearest-hit rays
  uint32_t l_sg = 0;  // triangle hits whose sign decisions were taken in FP64
  // by ray kind: cells entered and tests by AO and shadow rays; tests of the
  // primitive a secondary ray leaves (skipped, but an iteration spent)
  uint32_t l_cells_ao = 0, l_tests_ao = 0, l_cells_sh = 0, l_tests_sh = 0, l_own = 0;
  uint64_t c_iters = 0, c_lanes = 0, c_refills = 0;
  uint64_t c_cyc_trav = 0, c_cyc_res = 0, c_cyc_fin = 0, c_cyc_ref = 0;  // shader clocks by phase
  const uint64_t c_cyc_start = COUNT ? clock64() : 0;

  // ---- per-lane state
  int32_t kind = kIdle;
  int32_t st = kDone;  // kRun, kDone, or kPaused (waiting for an FP64 re-solve of primitive gk)
  int32_t gk = 0;
  int32_t slot = 0, ridx = 0;
  Ray R;
  R.bk = -1;
  R.rc = 0;
  R.nk = -1;
  __syncthreads();

  for (;;) {
    // ============================================================ re-solve
    const uint64_t cyc_r0 = COUNT ? clock64() : 0;
    if (RESOLVE && ballot(st == kPaused)) {
      if (st == kPaused) {
        const int32_t bk = slot >> 6;
        const JobDev *J = &A.jobs[bank_of(L.bank, bk).job];
        const SceneDev &S = J->sc;
        double o[3], d[3];
        if (kind == kPrimary) {
          int32_t px, py;
          bank_pixel(bank_of(L.bank, bk), slot & 63, px, py);
          primary_ray_f64(*J, px, py, o, d);
        } else {  // the FP32 origin, back from the FP32 frame
          o[0] = (double)R.ox + S.org[0];
          o[1] = (double)R.oy + S.org[1];
          o[2] = (double)R.oz + S.org[2];
          const double v[3] = {(double)R.dx, (double)R.dy, (double)R.dz};
          const double n = sqrt(dot3d(v, v));
          d[0] = v[0] / n;
          d[1] = v[1] / n;
          d[2] = v[2] / n;
        }
        const double tmin = kind == kPrimary ? 0.0 : kEpsD;
        const double tmax = kind == kAO ? J->ao_maxdist : INFINITY;
        double t = 0.0;
        const int h = hit_prim_f64<TRI>(S, gk >> kRecShift, o, d, tmin, tmax, t);
        int32_t nst = kRun;
        if (h) {
          const float tf = (float)t;
          if (kind >= kShadow) {
            R.bk = gk;
            R.bt = tf;
            nst = kDone;
          } else if (tf < R.bt || (tf == R.bt && gk < R.bk)) {
            R.bt = tf;
            R.bk = gk;
          }
        }
        st = nst;
      }
    }

    const uint64_t cyc_f0 = COUNT ? clock64() : 0;
    if (COUNT) c_cyc_res += cyc_f0 - cyc_r0;
    // ================================================================ finish
    if (ballot(kind != kIdle && st == kDone)) {
      const bool fin = kind != kIdle && st == kDone;
      const bool nearest = kind == kPrimary || kind == kCont;
      const bool fin_prim_hit = fin && nearest && R.bk >= 0;
      const bool fin_prim_miss = fin && nearest && R.bk < 0;
      bool finalize = fin_prim_miss;
      uint32_t nr = 0;
      uint32_t fifo_e = 0;  // FIFO word of a hit slot with secondary rays
      // every bank in flight renders the wave's current scene
      const SceneHot S = load_hot(&A.jobs[uni(scene_job)]);
      if (fin_prim_hit) {
        const int32_t bk = slot >> 6;
        const int32_t k = R.bk;
        const float t = R.bt;
        const float Px = R.ox + t * R.dx, Py = R.oy + t * R.dy, Pz = R.oz + t * R.dz;
        float Nx, Ny, Nz;
        if (k < S.s_end) {
          const vf4 s = ldgb(S.sph32, (uint32_t)k);
          Nx = Px - s.x;
          Ny = Py - s.y;
          Nz = Pz - s.z;
        } else if (TRI && k >= S.c_end) {  // triangle: e1 x e2
          const vf4 e1 = ldgb(S.triE1_32, (uint32_t)(k - S.c_end));
          const vf4 e2 = ldgb(S.triE2_32, (uint32_t)(k - S.c_end));
          Nx = e1.y * e2.z - e1.z * e2.y;
          Ny = e1.z * e2.x - e1.x * e2.z;
          Nz = e1.x * e2.y - e1.y * e2.x;
        } else {
          const vf4 a = ldgb(S.cylA32, (uint32_t)(k - S.s_end)), w = ldgb(S.cylW32, (uint32_t)(k - S.s_end));
          const float Dx = R.ox - a.x, Dy = R.oy - a.y, Dz = R.oz - a.z;
          const float sax = (Dx * w.x + Dy * w.y + Dz * w.z) + t * (R.dx * w.x + R.dy * w.y + R.dz * w.z);
          Nx = (Dx + t * R.dx) - sax * w.x;
          Ny = (Dy + t * R.dy) - sax * w.y;
          Nz = (Dz + t * R.dz) - sax * w.z;
        }
        const float inv = __builtin_amdgcn_rsqf(Nx * Nx + Ny * Ny + Nz * Nz);
        Nx *= inv;
        Ny *= inv;
        Nz *= inv;
        const float nd = Nx * R.dx + Ny * R.dy + Nz * R.dz;
        bool front = nd < 0.0f;
        if (!front) {
          Nx = -Nx;
          Ny = -Ny;
          Nz = -Nz;
        }
        uint32_t lv = 0;
        bool near0 = false;  // a sign decision within 2^-12 of zero
        const BankInfo &Bk = bank_of(L.bank, bk);
        const int32_t nl = Bk.n_lights;
        for (int l = 0; l < nl; ++l) {
          const float cl = Nx * Bk.ldir[l][0] + Ny * Bk.ldir[l][1] + Nz * Bk.ldir[l][2];
          if (cl > (float)kLightMin) lv |= 1u << l;
          near0 |= fabsf(cl) <= kKappa;
        }
        if (TRI && k >= S.c_end) {
          // A triangle's normal is the same over the whole face, so a sign
          // decided by FP32 rounding (a normal exactly perpendicular to a
          // light, a zero z component choosing the AO basis, a face seen
          // edge-on) would flip the face as a whole: near zero, the normal
          // and its decisions come from the FP64 vertices instead.
          near0 |= fabsf(nd) <= kKappa || fabsf(Nz) <= kKappa;
          if (near0) {
            if (COUNT) ++l_sg;
            int32_t px = 0, py = 0;
            bank_pixel(Bk, slot & 63, px, py);
            tri_signs_f64(A.jobs[Bk.job], (k - S.c_end) >> kRecShift, kind == kPrimary, px, py, R.dx, R.dy, R.dz,
                          Nx, Ny, Nz, front, lv);
          }
        }
        nr = (uint32_t)Bk.S + (uint32_t)__popc(lv);
        fifo_e = (uint32_t)slot | ((uint32_t)__popc(lv) << 8) | ((uint32_t)Bk.S << 16);
        L.px[slot] = Px;
        L.py[slot] = Py;
        L.pz[slot] = Pz;
        L.nx[slot] = Nx;
        L.ny[slot] = Ny;
        L.nz[slot] = Nz;
        L.prim[slot] = k;
        // A ray leaving a convex surface outward cannot meet it again: skip
        // it.  Leaving from inside, the ray's start is one root of its own
        // primitive; in FP32 that root lands anywhere within the hit
        // point's rounding (which can pass the 1e-4 lower limit at grazing
        // angles), so the walk takes only the other root of its own sphere
        // or cylinder, and never its own (flat) triangle -- the result in
        // exact arithmetic.
        L.pend[slot] = (int32_t)(nr | (front ? 0x80000000u : 0u));
        L.acc[slot] = lv;
        L.aomask[slot] = 0;
        if (nr == 0) finalize = true;
      }
      {  // queue hit slots that have secondary rays: S AO rays, then one per lit light
        const bool enq = fin_prim_hit && nr > 0;
        const uint64_t m = ballot(enq);
        if (enq) L.fifo[(q_tail + (int32_t)lane_rank(m)) % NS] = fifo_e;
        q_tail += __popcll(m);
      }
      if (fin && kind >= kShadow) {  // secondary results
        if (R.bk >= 0) {
          if (kind == kAO) {
            if (ridx < 32) atomicOr(&L.aomask[slot], 1u << ridx);
            atomicAdd(&L.acc[slot], 1u << 16);
          } else {
            atomicOr(&L.acc[slot], 1u << (8 + ridx));
          }
        }
        const int32_t old = atomicSub(&L.pend[slot], 1);
        if ((old & 0x7FFFFFFF) == 1) finalize = true;
      }
      __syncthreads();
      bool cont_next = false;  // the pixel goes on through a transparent surface
      int32_t layer = 0;
      if (!TRANS && finalize) {
        // shaded with the whole tile (shade_tile); a miss is marked here
        if (fin_prim_miss) L.prim[slot] = -1;
        atomicAdd(&bank_of(L.bank, slot >> 6).done, 1);
      }
      if (TRANS && finalize) {
        float alpha = 1.0f;
        const int32_t bk = slot >> 6;
        BankInfo &B = bank_of(L.bank, bk);
        int32_t x, y;
        bank_pixel(B, slot & 63, x, y);
        const int64_t pid = (int64_t)y * B.W + x;
        float cr = B.bg[0], cg = B.bg[1], cb = B.bg[2];
        int32_t hid = -1;
        uint32_t am = 0, lm = 0;
        if (!fin_prim_miss) {
          const int32_t k = L.prim[slot];
          hid = k;
          lm = (L.acc[slot] >> 8) & 0xFFu;
          am = L.aomask[slot];
          float a = 1.0f;
          shade_slot(L, B, slot, k, S.albedo, cr, cg, cb, a);
          if (B.layers > 1) alpha = a;
        }
        layer = L.layer[slot];
        if (layer == 0) {  // hit id and masks: the first surface's
          if (B.hit_id) B.hit_id[pid] = hid >> kRecShift;  // the global id (-1 stays -1)
          if (B.ao_mask) B.ao_mask[pid] = am;
          if (B.light_mask) B.light_mask[pid] = (uint8_t)lm;
        }
        {
          // composite front to back; what is left after the last surface (a
          // miss counts as an opaque background surface) shows the background
          const float T = layer ? L.trn[slot] : 1.0f;
          float ar = layer ? L.acc_r[slot] : 0.0f, ag = layer ? L.acc_g[slot] : 0.0f,
                ab = layer ? L.acc_b[slot] : 0.0f;
          ar += T * alpha * cr;
          ag += T * alpha * cg;
          ab += T * alpha * cb;
          const float Tn = T * (1.0f - alpha);
          if (alpha < 1.0f && layer + 1 < B.layers) {
            // continue through the surface: one more nearest-hit ray from the
            // hit point, skipping the primitive only when leaving it
            L.acc_r[slot] = ar;
            L.acc_g[slot] = ag;
            L.acc_b[slot] = ab;
            L.trn[slot] = Tn;
            L.layer[slot] = (uint8_t)(layer + 1);
            // entering it: its own far side counts, its start does not (the
            // skip rule flips: leaving outward becomes leaving from inside)
            L.pend[slot] = L.pend[slot] < 0 ? 1 : (int32_t)(1u | 0x80000000u);
            cont_next = true;
          } else {
            cr = ar + Tn * B.bg[0];
            cg = ag + Tn * B.bg[1];
            cb = ab + Tn * B.bg[2];
          }
        }
        if (!cont_next) {
          // the colour waits in the slot, whose hit point is spent, until the
          // whole tile goes out at once
          L.px[slot] = cr;
          L.py[slot] = cg;
          L.pz[slot] = cb;
          atomicAdd(&B.done, 1);
        }
      }
      if (TRANS) {  // continuations join the FIFO like slots with secondary rays
        const uint64_t m = ballot(cont_next);
        if (cont_next)  // one continuation ray
          L.fifo[(q_tail + (int32_t)lane_rank(m)) % NS] = (uint32_t)slot | (1u << 8) | (1u << 12);
        q_tail += __popcll(m);
      }
      {  // pixel counters live in LDS (registers are the scarce resource here)
        const uint32_t n_fin = (uint32_t)__popcll(ballot(finalize && !cont_next));
        const uint32_t n_hit = (uint32_t)__popcll(ballot(finalize && !fin_prim_miss && layer == 0));
        if (A.stats && lane == 0) {
          L.cnt[0] += n_fin;
          L.cnt[1] += n_hit;
        }
      }
      if (fin) kind = kIdle;
      __syncthreads();
      // free banks whose pixels are all shaded
      for (int b = 0; b < BANKS; ++b) {
        if (!((bank_busy >> b) & 1u)) continue;
        const int32_t n_b = uni(L.bank[b].n);
        const bool all_issued = issue_bank != b || issue_next == n_b;
        if (all_issued && uni(L.bank[b].done) == n_b) {
          if (!TRANS) shade_tile(L, b, lane, S.albedo);
          write_tile(L, b, lane);
          bank_busy &= ~(1u << b);
          if (issue_bank == b) issue_bank = -1;
        }
      }
    }

    const uint64_t cyc_q0 = COUNT ? clock64() : 0;
    if (COUNT) c_cyc_fin += cyc_q0 - cyc_f0;
    // ================================================================ refill
    {
      const uint64_t idle = ballot(kind == kIdle);
      const int32_t n_idle = __popcll(idle);
      const int32_t rank = (int32_t)lane_rank(idle);
      const bool me_idle = kind == kIdle;
      int32_t assigned = 0;
      // pass 1 -- assignment only: secondary rays from the FIFO, then fresh
      // primary rays; each idle lane learns (kind, slot, ray index)
      int32_t n_ao = 0;    // AO rays among the secondary rays issued this round
      int32_t n_cont = 0;  // continuations through transparent surfaces
      // The FIFO's first entries, one per lane, in one LDS read: the pops
      // below take them with readlane instead of an LDS round trip each.  A
      // round takes at most 64 entries (each has a ray, and at most 64 lanes
      // are idle).
      const int32_t q_n = min(q_tail - q_head, 64);
      uint32_t q_e = 0;
      if (lane < q_n) q_e = L.fifo[(q_head + lane) % NS];
      int32_t q_i = 0;
      while (assigned < n_idle && q_i < q_n) {
        const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int32_t)q_e, q_i);
        const int32_t s = (int32_t)(e & 0xFFu);
        const bool cs = TRANS && ((e >> 12) & 1u) != 0;
        const int32_t S_s = (int32_t)(e >> 16);
        const int32_t nr = S_s + (int32_t)((e >> 8) & 0xFu);
        const int32_t take = min(nr - head_issued, n_idle - assigned);
        if (me_idle && rank >= assigned && rank < assigned + take) {
          slot = s;
          ridx = head_issued + (rank - assigned);
          kind = cs ? kCont : (ridx < S_s ? kAO : kShadow);
        }
        if (cs) n_cont += take;
        n_ao += max(0, min(S_s - head_issued, take));  // ray indices < S are AO
        head_issued += take;
        assigned += take;
        if (head_issued == nr) {
          ++q_i;
          head_issued = 0;
        }
      }
      q_head += q_i;
      if (A.stats && lane == 0 && assigned > 0) {  // ray counters live in LDS
        L.cnt[2] += (uint32_t)n_ao;
        L.cnt[3] += (uint32_t)(assigned - n_ao - n_cont);
      }
      while (assigned < n_idle) {
        if (issue_bank < 0 || issue_next == uni(L.bank[issue_bank].n)) {
          issue_bank = -1;
          const uint32_t free_banks = ~bank_busy & ((1u << BANKS) - 1u);
          if (!free_banks) break;
          if (held_tile < 0) {
            int64_t t = -1;
            while (tiles_left) {
              // the j-th tile of queue xq: tile j mod stripe of the queue's
              // stripe j / stripe, which is stripe (j / stripe) 8 + xq overall
              uint32_t j = 0;
              if (lane == 0) j = atomicAdd(A.tile_counter + xq * kQueueStride, 1u);
              j = (uint32_t)uni((int32_t)j);
              const int32_t sl = A.stripe_log2;
              const int64_t g = ((((int64_t)(j >> sl)) * kQueueXcds + xq) << sl) +
                                (int64_t)(j & ((1u << sl) - 1u));
              if (g < A.n_tiles) {
                t = g;
                break;
              }
              // this queue is drained for good (its tiles only grow with j)
              if (--xq_left == 0) tiles_left = false;
              xq = xq + 1 == kQueueXcds ? 0 : xq + 1;
            }
            if (t < 0) break;
            held_tile = t;
            held_job = uni(find_job((const TR_CONST JobDev *)A.jobs, A.n_jobs, held_tile));
            held_key = uni(A.jobs[held_job].scene_key);
          }
          if (held_key != cur_key) {
            if (bank_busy) break;  // drain this scene's banks before switching
            cur_key = held_key;
            scene_job = held_job;
          }
          const TR_CONST JobDev *J = (const TR_CONST JobDev *)&A.jobs[held_job];
          const int32_t b = __ffs(free_banks) - 1;
          // tile index within its frame (< 2^31: the frame has < 2^31 pixels)
          const uint32_t tl = (uint32_t)(held_tile - J->queue_begin + J->tile_begin);
          const uint32_t txs = (uint32_t)J->tiles_x;
          const int32_t ty = (int32_t)(tl / txs), tx = (int32_t)(tl - (uint32_t)ty * txs);
          const int32_t x0 = tx * TW, y0 = ty * TH;
          const int32_t vw = min(TW, J->W - x0), vh = min(TH, J->H - y0);
          if (lane == 0) {
            BankInfo &B = L.bank[b];
            B.job = held_job;
            B.x0 = x0;
            B.y0 = y0;
            B.vw = vw;
            B.n = vw * vh;
            B.done = 0;
            B.vmagic = (65536 + vw - 1) / vw;
            B.W = J->W;
            B.H = J->H;
            B.th = J->th32;
            B.aspect = J->aspect32;
            B.rw2 = 2.0f / (float)J->W;
            B.rS = J->S > 0 ? 1.0f / (float)J->S : 0.0f;
            B.rh2 = 2.0f / (float)J->H;
            B.rgb = J->rgb;
            B.hit_id = J->hit_id;
            B.ao_mask = J->ao_mask;
            B.light_mask = J->light_mask;
            B.S = J->S;
            B.n_lights = J->n_lights;
            B.key0 = J->key0;
            B.key1 = J->key1;
            B.view = J->view_id;
            B.aa = J->aa;
            B.ks = J->ks32;
            B.shin = J->shin32;
            B.layers = J->layers;
            B.maxd = J->ao_maxdist32;
            B.sky = J->sky32;
          }
          if (lane < 24) {
            const int32_t l = lane / 3, a = lane % 3;
            L.bank[b].ldir[l][a] = J->ldir32[l][a];
            L.bank[b].lcol[l][a] = J->lcol32[l][a];
          } else if (lane < 27) {
            const int32_t a = lane - 24;
            L.bank[b].eye[a] = J->eye32[a];
            L.bank[b].f[a] = J->f32[a];
            L.bank[b].r[a] = J->r32[a];
            L.bank[b].u[a] = J->u32[a];
            L.bank[b].bg[a] = J->bg[a];
          }
          __syncthreads();
          bank_busy |= 1u << b;
          issue_bank = b;
          issue_next = 0;
          held_tile = -1;
        }
        const int32_t nvalid = uni(L.bank[issue_bank].n);
        const int32_t take = min(nvalid - issue_next, n_idle - assigned);
        if (me_idle && rank >= assigned && rank < assigned + take) {
          slot = issue_bank * 64 + issue_next + (rank - assigned);
          kind = kPrimary;
        }
        issue_next += take;
        assigned += take;
      }
      // pass 2 -- build every newly assigned ray once
      bool setup_ok = true;
      if (assigned > 0) {
        const bool fresh = me_idle && kind != kIdle;
        if (fresh) {
          const SceneHot H = load_hot(&A.jobs[uni(scene_job)]);
          const BankInfo &B = bank_of(L.bank, slot >> 6);
          int32_t pi, pj;
          bank_pixel(B, slot & 63, pi, pj);
          // One Philox draw serves both uses (one inlined copy keeps register
          // pressure down): an AO ray's direction, counter (pix, s, view, aa),
          // or an antialiasing sample's position, counter (pix, aa, view,
          // 0xFFFFFFFF); the two uniforms are the top 24 bits of words 0, 1.
          uint32_t b1 = 0, b2 = 0;
          const bool cam_dir = kind == kPrimary || kind == kCont;  // along the camera ray
          if (kind == kAO || (cam_dir && B.aa != 0)) {
            const uint32_t pix = (uint32_t)(pj * B.W + pi);
            const bool ao = kind == kAO;
            // AO streams of later surfaces: word 1 = s + 2^16 * layer
            const uint32_t s_ao = (uint32_t)ridx + (TRANS ? (uint32_t)L.layer[slot] << 16 : 0u);
            const uint4 x = philox4x32_10(
                make_uint4(pix, ao ? s_ao : (uint32_t)B.aa, B.view,
                           ao ? (uint32_t)B.aa : 0xFFFFFFFFu),
                B.key0, B.key1);
            b1 = x.x >> 8;
            b2 = x.y >> 8;
          }
          if (cam_dir) {
            // position inside the pixel: the centre for sample 0
            const float fx = B.aa != 0 ? (float)b1 * 0x1p-24f : 0.5f;
            const float fy = B.aa != 0 ? (float)b2 * 0x1p-24f : 0.5f;
            const float x = fmaf((float)pi + fx, B.rw2, -1.0f) * B.th * B.aspect;
            const float y = fmaf(-((float)pj + fy), B.rh2, 1.0f) * B.th;
            const float vx = B.f[0] + x * B.r[0] + y * B.u[0];
            const float vy = B.f[1] + x * B.r[1] + y * B.u[1];
            const float vz = B.f[2] + x * B.r[2] + y * B.u[2];
            const float inv = __builtin_amdgcn_rsqf(vx * vx + vy * vy + vz * vz);
            R.dx = vx * inv;
            R.dy = vy * inv;
            R.dz = vz * inv;
            R.tmax = INFINITY;
            if (TRANS && kind == kCont) {  // on from the surface it went through
              R.ox = L.px[slot];
              R.oy = L.py[slot];
              R.oz = L.pz[slot];
              R.tmin = kEps;
              R.skip = L.slot_skip(slot);
            } else {
              R.ox = B.eye[0];
              R.oy = B.eye[1];
              R.oz = B.eye[2];
              R.tmin = 0.0f;
              R.skip = -1;
              if (TRANS) L.layer[slot] = 0;
            }
          } else {
            R.ox = L.px[slot];
            R.oy = L.py[slot];
            R.oz = L.pz[slot];
            R.skip = L.slot_skip(slot);
            R.tmin = kEps;
            if (kind == kAO) {
              ao_dir_f32(L.nx[slot], L.ny[slot], L.nz[slot], b1, b2, R.dx, R.dy, R.dz);
              R.tmax = B.maxd;
            } else {
              uint32_t lv = L.acc[slot] & 0xFFu;  // the (ridx - S)-th light with N.L > 0
              for (int32_t n = ridx - B.S; n > 0; --n) lv &= lv - 1;
              const int32_t l = __ffs(lv) - 1;
              ridx = l;
              R.dx = B.ldir[l][0];
              R.dy = B.ldir[l][1];
              R.dz = B.ldir[l][2];
              R.tmax = INFINITY;
            }
          }
          setup_ok = BVH ? bvh_setup(R, H) : ray_setup(R, H);
          st = setup_ok ? kRun : kDone;
        }
      }
      c_rays += (uint64_t)assigned;
      if (COUNT) ++c_refills;
      if (COUNT) {
        const uint32_t entered = (me_idle && kind != kIdle && setup_ok) ? 1u : 0u;
        l_cells += entered;
        l_cells_ao += kind == kAO ? entered : 0u;
        l_cells_sh += kind == kShadow ? entered : 0u;
      }
    }

    if (COUNT) c_cyc_ref += clock64() - cyc_q0;
    // ================================================================ exit
    {
      const uint64_t busy = ballot(kind != kIdle);
      if (!busy) {
        if (!tiles_left && held_tile < 0 && bank_busy == 0 && q_head == q_tail) break;
        if (++idle_rounds > 4) {  // cannot happen when the bookkeeping is right
          if (lane == 0) atomicAdd(A.tile_counter + kQueueXcds * kQueueStride, 1u);
          stalled = true;
          break;
        }
        continue;
      }
      idle_rounds = 0;
    }

    // ============================================================= traverse
    {
      const uint32_t free_banks = ~bank_busy & ((1u << BANKS) - 1u);
      const bool can_refill =
          q_head != q_tail || (issue_bank >= 0 && issue_next < uni(L.bank[issue_bank].n)) ||
          (free_banks && ((held_tile < 0 && tiles_left) || (held_tile >= 0 && (held_key == cur_key || !bank_busy))));
      const SceneHot H = load_hot(&A.jobs[uni(scene_job)]);
      // (>= 1, so the loop also ends when no lane works).  Lanes paused for
      // an FP64 re-solve wait for the loop's end: with a refill pending that
      // comes when fewer than refill_below lanes work, else when none does.
      const int32_t thresh = uni(can_refill ? A.refill_below : 1);
      const bool anyhit = kind >= kShadow;
      const uint64_t near_m = ballot(!anyhit);  // lanes with a nearest-hit ray (or idle)
      // grid-frame offsets of the jump step, held in VGPRs for the whole
      // loop: the step's FMAs take the scale from an SGPR, and one VOP3
      // instruction reads at most one SGPR (else a copy every iteration)
      float gorg0 = H.org32[0], gorg1 = H.org32[1], gorg2 = H.org32[2];
      asm volatile("" : "+v"(gorg0), "+v"(gorg1), "+v"(gorg2));
      const uint64_t cyc0 = COUNT ? clock64() : 0;
      // (the exit test sits at the loop's end, where it is a scalar branch)
      bool work = st == kRun;
      int32_t nwork = __popcll(ballot(work));
      for (int32_t it = 0; nwork >= (it >= kMinIters ? thresh : 1); ++it) {
        if (COUNT) {
          ++c_iters;
          c_lanes += (uint64_t)nwork;
        }
        // The next reference id is already loaded (R.nk, -1 = cell done), so
        // each lane knows its unit of work before touching memory.
        // Working lanes only from here (an if, not a continue: the lanes must
        // meet again at the loop head for its ballot).  Ballots inside count
        // the working lanes.
        if (work) {
        // The entry held: a record offset (a multiple of 16) whose bit 0
        // flags the last entry of its cell's list, or -1 (cell done).
        const int32_t nk = R.nk;
        const int32_t nkr = nk & ~15;  // the record offset (negative stays negative)
        // Each lane's unit of work, one compare each: a sphere test (for a
        // cylinder, first the test of its bounding sphere, in the same code),
        // a triangle test, or a step out of an empty or finished cell.  Every
        // unit some lane wants runs in this iteration; holding a unit back
        // until more lanes want it (thresholds on the lane counts) cost more
        // in scalar decisions per iteration than it saved.
        const bool is_sph = (uint32_t)nk < (uint32_t)H.c_end;  // nk = -1: no
        const bool is_tri = TRI && nk >= H.c_end;
        const bool is_step = !is_sph && !is_tri;  // nk < 0
        // Sphere records are fetched first; the tests run, then the step, which
        // takes both the lanes with no entry left (empty cells) and the lanes
        // that just tested their cell's last entry and go on: a cell costs one
        // iteration per entry, none extra to leave it.  The step's cell load
        // is issued last and consumed next iteration.
        vf4 sdat;  // (read only where is_sph; a cylinder's bounding sphere follows the spheres)
        if (is_sph) sdat = ldgb(H.sph32, (uint32_t)nkr);
        bool enter = false;  // the step moved into a cell inside the grid
        if (BVH && is_step) {
          // ---- BVH node: test both children's boxes against (tmin, min(t1,
          // best t)); go to the nearer hit child, stack the other; with no
          // child hit take the next stacked item, or stop.  Items are node
          // indices, or -(primitive id) - 1 for a leaf.  Every index is
          // checked before use, and a full stack drops the child (counted).
          const bool valid = (uint32_t)R.rc < (uint32_t)(H.bvh_n - 1);
          const uint32_t nb = valid ? 4u * (uint32_t)R.rc : 0u;
          const vf4 n0 = ldg(H.bvh, nb), n1 = ldg(H.bvh, nb + 1u), n2 = ldg(H.bvh, nb + 2u),
                    n3 = ldg(H.bvh, nb + 3u);
          const float tc = vminf(R.t1, R.bt);
          const float la0 = (n0.x - R.ox) * R.hx, lb0 = (n0.w - R.ox) * R.hx;
          const float la1 = (n0.y - R.oy) * R.hy, lb1 = (n1.x - R.oy) * R.hy;
          const float la2 = (n0.z - R.oz) * R.hz, lb2 = (n1.y - R.oz) * R.hz;
          const float ra0 = (n1.z - R.ox) * R.hx, rb0 = (n2.y - R.ox) * R.hx;
          const float ra1 = (n1.w - R.oy) * R.hy, rb1 = (n2.z - R.oy) * R.hy;
          const float ra2 = (n2.x - R.oz) * R.hz, rb2 = (n2.w - R.oz) * R.hz;
          const float tnL = fmaxf(fmaxf(fminf(la0, lb0), fminf(la1, lb1)), fmaxf(fminf(la2, lb2), R.tmin));
          const float tfL = fminf(fminf(fmaxf(la0, lb0), fmaxf(la1, lb1)), fminf(fmaxf(la2, lb2), tc));
          const float tnR = fmaxf(fmaxf(fminf(ra0, rb0), fminf(ra1, rb1)), fmaxf(fminf(ra2, rb2), R.tmin));
          const float tfR = fminf(fminf(fmaxf(ra0, rb0), fmaxf(ra1, rb1)), fminf(fmaxf(ra2, rb2), tc));
          const bool hitL = valid && tnL <= tfL, hitR = valid && tnR <= tfR;
          const int32_t cl = __float_as_int(n3.x), cr = __float_as_int(n3.y);
          const bool lfirst = !hitR || (hitL && tnL <= tnR);
          int32_t sp = R.cx;
          if (hitL && hitR) {
            if (sp < kStack) {
              L.stk[sp * 64 + lane] = lfirst ? cr : cl;
              ++sp;
            } else if (COUNT) {
              ++l_ovf;
            }
          }
          int32_t item = lfirst ? cl : cr;
          bool have = hitL || hitR;
          if (!have && sp > 0) {
            --sp;
            item = L.stk[sp * 64 + lane];
            have = true;
          }
          R.cx = sp;
          R.rc = have && item >= 0 ? item : -1;
          R.nk = have && item < 0 && -item - 1 < H.bvh_n ? (-item - 1) << kRecShift : -1;
          if (R.rc < 0 && R.nk < 0) st = kDone;
          if (COUNT) ++l_cells;
        }
        bool tested = false, hit = false, graze = false;
        float t;  // set by every test; read only on a tested lane
        asm volatile("" : "=v"(t));
        const bool own = nkr == -2 - R.skip;  // the surface this ray leaves from inside
        const bool ball = nkr >= H.s_end;     // (where is_sph) the sphere bounds a cylinder
        bool pass = false;                    // the ray may meet that cylinder
        // the cell's last entry (read only on a tested lane, where nk >= 0)
        const bool last = !BVH & (nk != nkr);
        if (is_sph) {
          tested = true;
          const vf4 s = sdat;
          const float qx = s.x - R.ox, qy = s.y - R.oy, qz = s.z - R.oz;
          const float b = qx * R.dx + qy * R.dy + qz * R.dz;
          const float lx = qx - b * R.dx, ly = qy - b * R.dy, lz = qz - b * R.dz;
          const float ll = lx * lx + ly * ly + lz * lz;
          const float rr = s.w;  // squared radius
          const float disc = rr - ll;
          const float sg = kKappa * (rr + ll);
          graze = RESOLVE & (fabsf(disc) <= sg);
          // decidable real roots: disc >= 0 and not grazing, i.e. disc > sg
          // (disc < 0 gives NaN roots, which no compare accepts)
          const bool ok = RESOLVE ? disc > sg : disc >= 0.0f;
          const float sq = sqrtf_fast(disc);
          const float t0 = b - sq, t1 = b + sq;
          // nearer root if it is past tmin, else the farther (t0 <= t1);
          // only the farther on the ray's own sphere
          t = ((t0 > R.tmin) & !own) ? t0 : t1;
          hit = ok & (t > R.tmin) & (t <= R.t1) & !ball;
          // A bounding sphere passes unless the ray misses it decidably (a
          // cylinder hit lies inside it, and its padding is far above the
          // FP32 rounding); only then is the cylinder itself tested.
          pass = ok | graze;
          graze = graze & !ball;
        }
        // skipped: the surface an outward ray leaves, and the own triangle
        const bool live = (nkr != R.skip) & !(TRI & own & (nkr >= H.c_end));
        if (is_tri) {
          // ---- triangle (two-sided, Moller-Trumbore).  Undecidable in FP32,
          // and so re-solved in FP64: a ray within 2^-12 of the triangle's
          // plane (|det| against |e1 x e2|), or a hit point within 2^-12 of an
          // edge in barycentric terms.
          tested = true;
          const uint32_t m = (uint32_t)(nkr - H.c_end);  // byte offset of its records
          const vf4 V = ldgb(H.triV32, m), E1 = ldgb(H.triE1_32, m), E2 = ldgb(H.triE2_32, m);
          const float Px = R.dy * E2.z - R.dz * E2.y, Py = R.dz * E2.x - R.dx * E2.z,
                      Pz = R.dx * E2.y - R.dy * E2.x;
          const float det = E1.x * Px + E1.y * Py + E1.z * Pz;
          const float Tx = R.ox - V.x, Ty = R.oy - V.y, Tz = R.oz - V.z;
          const float Qx = Ty * E1.z - Tz * E1.y, Qy = Tz * E1.x - Tx * E1.z,
                      Qz = Tx * E1.y - Ty * E1.x;
          const float id = rcpf(det);
          const float u = (Tx * Px + Ty * Py + Tz * Pz) * id;
          const float v = (R.dx * Qx + R.dy * Qy + R.dz * Qz) * id;
          const float w = 1.0f - u - v;
          t = (E2.x * Qx + E2.y * Qy + E2.z * Qz) * id;
          const bool in_t = t > R.tmin && t <= R.t1;
          const bool par = fabsf(det) <= kKappa * V.w;
          const bool edge = u >= -kKappa && v >= -kKappa && w >= -kKappa &&
                            (fabsf(u) <= kKappa || fabsf(v) <= kKappa || fabsf(w) <= kKappa);
          graze = RESOLVE && (par || (edge && in_t));
          hit = !graze && det != 0.0f && u >= 0.0f && v >= 0.0f && w >= 0.0f && in_t;
        } else if (is_sph & ball & pass & live) {
          const vf4 a = ldgb(H.cylA32, (uint32_t)(nkr - H.s_end));
          const vf4 w = ldgb(H.cylW32, (uint32_t)(nkr - H.s_end));
          const float Dx = R.ox - a.x, Dy = R.oy - a.y, Dz = R.oz - a.z;
          const float dw = R.dx * w.x + R.dy * w.y + R.dz * w.z;
          const float Dw = Dx * w.x + Dy * w.y + Dz * w.z;
          const float dpx = R.dx - dw * w.x, dpy = R.dy - dw * w.y, dpz = R.dz - dw * w.z;
          const float Dpx = Dx - Dw * w.x, Dpy = Dy - Dw * w.y, Dpz = Dz - Dw * w.z;
          // |perp(D + t d)|^2 = rho^2 about the closest approach of the
          // perpendicular motion, t_c = -B / A, where the perpendicular
          // offset is l = perp(D) + t_c perp(d): the discriminant (B^2 -
          // A C) / A = rho^2 - |l|^2 then carries no cancellation of the
          // eye's distance (as the sphere test's), and the grazing test
          // compares it with rho^2 + |l|^2.
          const float Aq = dpx * dpx + dpy * dpy + dpz * dpz;
          const float Bq = dpx * Dpx + dpy * Dpy + dpz * Dpz;
          const bool nonpar = Aq > 1e-12f;
          const float iA = rcpf(Aq);
          const float tc = -Bq * iA;
          const float lx = Dpx + tc * dpx, ly = Dpy + tc * dpy, lz = Dpz + tc * dpz;
          const float ll = lx * lx + ly * ly + lz * lz;
          const float rr = a.w;  // squared radius
          const float disc = rr - ll;
          const float sg = kKappa * (rr + ll);
          const bool g0 = RESOLVE & nonpar & (fabsf(disc) <= sg);
          const bool ok = nonpar & (RESOLVE ? disc > sg : disc >= 0.0f);  // (as for spheres)
          const float sq = sqrtf_fast(disc * iA);
          const float tl = tc - sq, th = tc + sq;
          const float kL = kKappa * w.w;
          const float sl = Dw + tl * dw, sh = Dw + th * dw;
          // (predicates combined with & and |: no short-circuit branches)
          const bool inl = ok & !own & (tl > R.tmin) & (tl <= R.t1);  // own: far root only
          const bool inh = ok & (th > R.tmin) & (th <= R.t1);
          const float el0 = fabsf(sl), el1 = fabsf(sl - w.w), eh0 = fabsf(sh), eh1 = fabsf(sh - w.w);
          const bool gl = RESOLVE & inl & ((el0 <= kL) | (el1 <= kL));
          const bool gh = RESOLVE & inh & ((eh0 <= kL) | (eh1 <= kL));
          const bool hl = inl & !gl & (sl >= 0.0f) & (sl <= w.w);
          const bool hh = inh & !gh & (sh >= 0.0f) & (sh <= w.w);
          // the near root decides first; an undecidable root defers to FP64
          graze = g0 | gl | (!hl & gh);
          hit = !graze & (hl | hh);
          t = hl ? tl : th;
        }
        if (tested) {
          hit = hit & live;
          graze = graze & live;
          if (COUNT) {
            l_own += !live;
            l_tests_ao += kind == kAO;
            l_tests_sh += kind == kShadow;
          }
          if (COUNT && live) {
            if (nkr < H.s_end) {
              ++l_st;
              l_sh += hit;
            } else if (TRI && nkr >= H.c_end) {
              ++l_tt;
              l_th += hit;
            } else {
              ++l_ct;
              l_ch += hit;
            }
            l_res += graze;
            if (nkr < H.s_end) l_rs += graze;
            else if (TRI && nkr >= H.c_end) l_rt += graze;
            else l_rc += graze;
            l_rn += graze && !anyhit;
          }
          // nearest hit (ties to the lower id); any hit ends a shadow/AO ray.
          // Most iterations test only shadow and AO rays (about nine rays in
          // ten are), so the nearest-hit order is decided only when a tested
          // lane carries a nearest-hit ray: a wave-uniform branch on the
          // execution mask (the tested lanes) against the phase's mask of
          // such lanes.  (The empty asm statement keeps the compiler from
          // executing the body unconditionally and selecting its result.)
          // A shadow or AO ray reads only bk (hit or not) once it ends, so
          // bt is kept only here too.
          bool take = hit;
          if (__builtin_amdgcn_read_exec() & near_m) {
            asm volatile("");
            take = hit & (anyhit | (t < R.bt) | ((t == R.bt) & (nkr < R.bk)));
            R.bt = take ? t : R.bt;
          }
          R.bk = take ? nkr : R.bk;
          st = (anyhit & hit) ? kDone : st;
          if (RESOLVE) {
            st = graze ? kPaused : st;
            gk = graze ? nkr : gk;
          }
          if (BVH) {  // next stacked item, or the walk is over
            int32_t sp = R.cx;
            int32_t item = -1;
            const bool have = sp > 0;
            if (have) {
              --sp;
              item = L.stk[sp * 64 + lane];
            }
            R.cx = sp;
            R.rc = have && item >= 0 ? item : -1;
            R.nk = have && item < 0 && -item - 1 < H.bvh_n ? (-item - 1) << kRecShift : -1;
            if (R.rc < 0 && R.nk < 0 && st == kRun) st = kDone;
          } else {
            // next entry (after the last use of this one, so the load can land
            // in its register and stay in flight into the next iteration);
            // after the cell's last entry none: the lane steps now, or (paused
            // or done) finds the cell done
            if (last) {
              R.nk = (int32_t)0x80000000u;  // (no block ahead: a unit step)
            } else {
              R.rc += 4;  // (a byte offset into wrefs)
              R.nk = (int32_t)ldgb(H.refs, (uint32_t)R.rc);
            }
          }
        }
        // lanes with nothing left in their cell: stepping on
        if (!BVH && (is_step | (tested & last & (st == kRun)))) {
          // ---- cell exhausted: stop, or leave it.  An empty cell carries the
          // Chebyshev distance k to the nearest occupied cell, so the whole
          // cube of half-size k-1 around it is empty and the walk jumps to
          // where the ray leaves that cube (k = 1: an ordinary DDA step).
          // Branch-free: the k = 1 step is the jump with a cube of size 0.
          // nk1 = -k: rc = -distance in an empty cell, >= 0 otherwise; an
          // empty cell's record also holds, for the ray's octant, the M of the
          // empty block of 2M + 1 cells per axis ahead of it (0 once a cell is
          // done), and the jump takes the larger
          const int32_t mo = (int32_t)__builtin_amdgcn_ubfe((uint32_t)R.nk, (uint32_t)R.o3, 3u);
          const int32_t nk1 = min(min(R.rc, -1), -1 - 2 * mo);
          // cell just beyond the cube on each axis; its near plane is crossed at
          // b_a + i * h_a (b_a is shifted one cell for negative steps at setup);
          // (-sign) (-k) is the offset
          const int32_t ix1 = R.cx + __mul24(R.sx, nk1);
          const int32_t iy1 = R.cy + __mul24(R.sy, nk1);
          const int32_t iz1 = R.cz + __mul24(R.sz, nk1);
          const float tx = fmaf((float)ix1, R.hx, R.bx);  // inf when d_x = 0
          const float ty = fmaf((float)iy1, R.hy, R.by);
          const float tz = fmaf((float)iz1, R.hz, R.bz);
          const float tn = fminf(tx, fminf(ty, tz));
          // Go on unless the plane is the box exit or lies beyond the best hit
          // so far.  Branch-free: a lane that stops computes a cell it never
          // enters (its coordinates are reset when the lane takes a new ray).
          const bool adv = tn < R.bt;  // (bt is at most just above t1)
          const bool ax = tx == tn;
          const bool ay = !ax & (ty == tn);
          const bool az = !ax & !ay;
          // The other axes land in the cell of the exit point, kept within the
          // cube's half ahead of the ray: from the current cell to the last
          // one before i1 (i1 + sign is that cell; the ray moves forward and
          // crosses no other face first, so only rounding could leave it).
          const int32_t nx = med3i(cvt_floor(fmaf(fmaf(tn, R.dx, R.ox), H.inv32[0], gorg0)), R.cx, ix1 + R.sx);
          const int32_t ny = med3i(cvt_floor(fmaf(fmaf(tn, R.dy, R.oy), H.inv32[1], gorg1)), R.cy, iy1 + R.sy);
          const int32_t nz = med3i(cvt_floor(fmaf(fmaf(tn, R.dz, R.oz), H.inv32[2], gorg2)), R.cz, iz1 + R.sz);
          R.cx = ax ? ix1 : nx;
          R.cy = ay ? iy1 : ny;
          R.cz = az ? iz1 : nz;
          // (tn < bt is finite, so the crossed axis has a nonzero step)
          const bool inb = ((uint32_t)R.cx < (uint32_t)H.res[0]) & ((uint32_t)R.cy < (uint32_t)H.res[1]) &
                           ((uint32_t)R.cz < (uint32_t)H.res[2]);
          enter = adv & inb;
          st = enter ? st : kDone;
          if (COUNT) {
            l_jumps += adv & (nk1 < -1);
            l_cells += enter;
            l_cells_ao += enter & (kind == kAO);
            l_cells_sh += enter & (kind == kShadow);
          }
        }
        if (!BVH && enter) load_cell(R, H);
        }  // work
        work = st == kRun;
        nwork = __popcll(ballot(work));
      }
      (void)anyhit;
      if (COUNT) c_cyc_trav += clock64() - cyc0;
    }
  }

  // ---- counters
  if (A.stats) {
    if (COUNT) {
      atomicAdd(&L.cnt[4], l_cells);
      atomicAdd(&L.cnt[5], l_st);
      atomicAdd(&L.cnt[6], l_sh);
      atomicAdd(&L.cnt[7], l_ct);
      atomicAdd(&L.cnt[8], l_ch);
      atomicAdd(&L.cnt[9], l_res);
      atomicAdd(&L.cnt[10], l_jumps);
      if (TRI) {
        atomicAdd(&L.cnt[11], l_tt);
        atomicAdd(&L.cnt[12], l_th);
      }
      if (BVH) atomicAdd(&L.cnt[13], l_ovf);
      if (RESOLVE) {
        atomicAdd(&L.cnt[14], l_rs);
        atomicAdd(&L.cnt[15], l_rc);
        atomicAdd(&L.cnt[16], l_rt);
        atomicAdd(&L.cnt[17], l_rn);
      }
      if (TRI) atomicAdd(&L.cnt[18], l_sg);
      atomicAdd(&L.cnt[19], l_cells_ao);
      atomicAdd(&L.cnt[20], l_tests_ao);
      atomicAdd(&L.cnt[21], l_cells_sh);
      atomicAdd(&L.cnt[22], l_tests_sh);
      atomicAdd(&L.cnt[23], l_own);
    }
    __syncthreads();
    if (lane == 0) {
      unsigned long long *st = (unsigned long long *)A.stats;
      atomicAdd(&st[TR_STAT_PIXELS], (unsigned long long)L.cnt[0]);
      atomicAdd(&st[TR_STAT_HIT_PIXELS], (unsigned long long)L.cnt[1]);
      atomicAdd(&st[TR_STAT_AO_RAYS], (unsigned long long)L.cnt[2]);
      atomicAdd(&st[TR_STAT_SHADOW_RAYS], (unsigned long long)L.cnt[3]);
      atomicAdd(&st[TR_STAT_RAYS_TRACED], (unsigned long long)c_rays);
      if (stalled) atomicAdd(&st[TR_STAT_STALLS], 1ull);
      if (COUNT) {
        atomicAdd(&st[TR_STAT_CELLS], (unsigned long long)L.cnt[4]);
        atomicAdd(&st[TR_STAT_SPH_TESTS], (unsigned long long)L.cnt[5]);
        atomicAdd(&st[TR_STAT_SPH_HITS], (unsigned long long)L.cnt[6]);
        atomicAdd(&st[TR_STAT_CYL_TESTS], (unsigned long long)L.cnt[7]);
        atomicAdd(&st[TR_STAT_CYL_HITS], (unsigned long long)L.cnt[8]);
        atomicAdd(&st[TR_STAT_RESOLVES], (unsigned long long)L.cnt[9]);
        atomicAdd(&st[TR_STAT_WAVE_ITERS], (unsigned long long)c_iters);
        atomicAdd(&st[TR_STAT_LANE_ITERS], (unsigned long long)c_lanes);
        atomicAdd(&st[TR_STAT_REFILLS], (unsigned long long)c_refills);
        atomicAdd(&st[TR_STAT_JUMPS], (unsigned long long)L.cnt[10]);
        atomicAdd(&st[TR_STAT_TRI_TESTS], (unsigned long long)L.cnt[11]);
        atomicAdd(&st[TR_STAT_TRI_HITS], (unsigned long long)L.cnt[12]);
        atomicAdd(&st[TR_STAT_STACK_OVERFLOWS], (unsigned long long)L.cnt[13]);
        atomicAdd(&st[TR_STAT_RESOLVES_SPH], (unsigned long long)L.cnt[14]);
        atomicAdd(&st[TR_STAT_RESOLVES_CYL], (unsigned long long)L.cnt[15]);
        atomicAdd(&st[TR_STAT_RESOLVES_TRI], (unsigned long long)L.cnt[16]);
        atomicAdd(&st[TR_STAT_RESOLVES_NEAREST], (unsigned long long)L.cnt[17]);
        atomicAdd(&st[TR_STAT_SIGNS_F64], (unsigned long long)L.cnt[18]);
        atomicAdd(&st[TR_STAT_CELLS_AO], (unsigned long long)L.cnt[19]);
        atomicAdd(&st[TR_STAT_TESTS_AO], (unsigned long long)L.cnt[20]);
        atomicAdd(&st[TR_STAT_CELLS_SHADOW], (unsigned long long)L.cnt[21]);
        atomicAdd(&st[TR_STAT_TESTS_SHADOW], (unsigned long long)L.cnt[22]);
        atomicAdd(&st[TR_STAT_TESTS_OWN], (unsigned long long)L.cnt[23]);
        atomicAdd(&st[TR_STAT_CYCLES_TRAVERSE], (unsigned long long)c_cyc_trav);
        atomicAdd(&st[TR_STAT_CYCLES_TOTAL], (unsigned long long)(clock64() - c_cyc_start));
        atomicAdd(&st[TR_STAT_CYCLES_RESOLVE], (unsigned long long)c_cyc_res);
        atomicAdd(&st[TR_STAT_CYCLES_FINISH], (unsigned long long)c_cyc_fin);
        atomicAdd(&st[TR_STAT_CYCLES_REFILL], (unsigned long long)c_cyc_ref);
      }
    }
  }
}

__global__ void k_zero_u32(uint32_t *p) { *p = 0u; }

// One job table entry written from a kernel argument (the caller's job needs
// no host staging buffer): the wave copies its 4-byte words.
static_assert(sizeof(JobDev) % 4 == 0, "JobDev is copied as words");
__global__ __launch_bounds__(64) void k_put_job(const JobDev J, JobDev *dst) {
  const uint32_t *src = (const uint32_t *)&J;
  uint32_t *d = (uint32_t *)dst;
  for (uint32_t i = threadIdx.x; i < (uint32_t)(sizeof(JobDev) / 4); i += 64) d[i] = src[i];
}

__global__ void k_debug_philox(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 c = make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
  const uint4 x = philox4x32_10(c, key[2 * i], key[2 * i + 1]);
  out[4 * i] = x.x;
  out[4 * i + 1] = x.y;
  out[4 * i + 2] = x.z;
  out[4 * i + 3] = x.w;
}

__global__ void k_debug_ao_dirs(int64_t n, const float *nrm, const uint32_t *pix, const uint32_t *smp,
                                uint32_t view, uint32_t k0, uint32_t k1, float *w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t b1, b2;
  ao_uniform_bits(pix[i], smp[i], view, 0u, k0, k1, b1, b2);
  ao_dir_f32(nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2], b1, b2, w[3 * i], w[3 * i + 1], w[3 * i + 2]);
}

}  // namespace

namespace trh {

template <int BANKS, bool RES, bool CNT, bool TRANS, bool TRI, bool BVH = false>
static hipError_t launch_t(const WaveLaunch &L, hipStream_t st) {
  WaveArgs a;
  a.jobs = L.jobs;
  a.n_jobs = L.n_jobs;
  a.n_tiles = L.n_tiles;
  a.tile_counter = L.tile_counter;
  a.stats = L.stats;
  a.tile_w = L.tile_w;
  a.refill_below = L.refill_below;
  a.stripe_log2 = __builtin_ctz((unsigned)L.stripe);
  k_render_wave<BANKS, RES, CNT, TRANS, TRI, BVH><<<L.n_waves, 64, 0, st>>>(a);
  return hipGetLastError();
}

template <int BANKS, bool TRANS, bool TRI>
static hipError_t launch_bt(const WaveLaunch &L, hipStream_t st) {
  const bool cnt = L.count_ops != 0 && L.stats != nullptr;
  if (L.resolve)
    return cnt ? launch_t<BANKS, true, true, TRANS, TRI>(L, st)
               : launch_t<BANKS, true, false, TRANS, TRI>(L, st);
  return cnt ? launch_t<BANKS, false, true, TRANS, TRI>(L, st)
             : launch_t<BANKS, false, false, TRANS, TRI>(L, st);
}

// Variants: compositing (transparency) and triangles are compiled in only
// for launches that need them, so the common kernel keeps its registers.
// BVH walk: two banks, opaque rendering
template <bool TRI>
static hipError_t launch_bvh_walk(const WaveLaunch &L, hipStream_t st) {
  const bool cnt = L.count_ops != 0 && L.stats != nullptr;
  if (L.resolve)
    return cnt ? launch_t<2, true, true, false, TRI, true>(L, st)
               : launch_t<2, true, false, false, TRI, true>(L, st);
  return cnt ? launch_t<2, false, true, false, TRI, true>(L, st)
             : launch_t<2, false, false, false, TRI, true>(L, st);
}

template <int BANKS>
static hipError_t launch_b(const WaveLaunch &L, hipStream_t st) {
  if (L.trans) return L.tri ? launch_bt<BANKS, true, true>(L, st) : launch_bt<BANKS, true, false>(L, st);
  return L.tri ? launch_bt<BANKS, false, true>(L, st) : launch_bt<BANKS, false, false>(L, st);
}

hipError_t launch_render_wave(const WaveLaunch &L, hipStream_t st) {
  if (L.bvh) return L.tri ? launch_bvh_walk<true>(L, st) : launch_bvh_walk<false>(L, st);
  if (L.banks == 3) return launch_b<3>(L, st);
  return launch_b<2>(L, st);
}

hipError_t launch_put_job(const JobDev &J, JobDev *dst, hipStream_t st) {
  k_put_job<<<1, 64, 0, st>>>(J, dst);
  return hipGetLastError();
}

hipError_t launch_zero_counter(uint32_t *p, hipStream_t st) {
  k_zero_u32<<<1, 1, 0, st>>>(p);
  return hipGetLastError();
}

hipError_t launch_debug_philox(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_debug_philox<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, ctr, key, out);
  return hipGetLastError();
}

hipError_t launch_debug_ao_dirs(int64_t n, const float *nrm, const uint32_t *pix,
                                const uint32_t *smp, uint32_t view, uint32_t k0, uint32_t k1,
                                float *w, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_debug_ao_dirs<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, nrm, pix, smp, view, k0, k1, w);
  return hipGetLastError();
}

}  // namespace trh
