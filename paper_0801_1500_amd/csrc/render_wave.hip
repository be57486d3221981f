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
//            and writes the frame;
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
// pixel.  Intersection and shading run in FP32; a sphere or cylinder test
// whose discriminant is within 2^-12 of its scale, or whose axial hit is
// within 2^-12 L of a cylinder end, is re-solved in FP64 with the FP64
// primitive (primary rays are regenerated in FP64 from their pixel).
#include "tr_internal.h"

namespace {

using namespace trd;

constexpr float kEps = 1e-4f;
constexpr float kKappa = 1.0f / 4096.0f;
constexpr double kEpsD = 1e-4;

enum : int32_t { kIdle = 0, kPrimary = 1, kShadow = 2, kAO = 3 };

template <int BANKS>
struct Lds {
  static constexpr int NS = BANKS * 64;
  float px[NS], py[NS], pz[NS];
  float nx[NS], ny[NS], nz[NS];
  int32_t prim[NS];     // hit primitive
  int32_t skip[NS];     // primitive skipped by secondary rays (-1 = none)
  int32_t pending[NS];  // secondary rays not yet finished
  int32_t nrays[NS];    // secondary rays of the slot
  uint32_t lvalid[NS];  // lights with N.L > 0
  uint32_t aomask[NS];
  int32_t aocnt[NS];
  uint32_t lmask[NS];
  uint8_t fifo[NS];
  int32_t bank_job[BANKS], bank_x0[BANKS], bank_y0[BANKS], bank_vw[BANKS], bank_n[BANKS];
  int32_t bank_done[BANKS];
};

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrtf_fast(float x) { return __builtin_amdgcn_sqrtf(x); }

// Per-lane ray and traversal state.
struct Ray {
  float ox, oy, oz, dx, dy, dz;
  float tmin, tmax;  // t interval of accepted hits
  float t1;          // exit of the grid box (clipped to tmax)
  float bx, by, bz;  // plane t = base + plane_index * hid  (per axis)
  float hx, hy, hz;
  float tnx, tny, tnz;
  int32_t cx, cy, cz;
  int32_t sx, sy, sz;  // step signs
  uint32_t rc, re;     // reference cursor / end in the current cell
  float bt;            // best t
  int32_t bk;          // best id (-1 = none)
  int32_t skip;
};

// Clip to the grid box and position the walk at the entry cell.
// Returns false when the ray misses the box.
template <class SC>
__device__ __forceinline__ bool ray_setup(Ray &R, const SC &S) {
  const float ix = rcpf(R.dx), iy = rcpf(R.dy), iz = rcpf(R.dz);
  float t0 = R.tmin, t1 = R.tmax;
  {
    const float a = (S.lo32[0] - R.ox) * ix, b = (S.hi32[0] - R.ox) * ix;
    t0 = fmaxf(t0, fminf(a, b));
    t1 = fminf(t1, fmaxf(a, b));
  }
  {
    const float a = (S.lo32[1] - R.oy) * iy, b = (S.hi32[1] - R.oy) * iy;
    t0 = fmaxf(t0, fminf(a, b));
    t1 = fminf(t1, fmaxf(a, b));
  }
  {
    const float a = (S.lo32[2] - R.oz) * iz, b = (S.hi32[2] - R.oz) * iz;
    t0 = fmaxf(t0, fminf(a, b));
    t1 = fminf(t1, fmaxf(a, b));
  }
  R.t1 = t1;
  R.bt = INFINITY;
  R.bk = -1;
  if (!(t0 <= t1)) return false;
  const float ex = R.ox + t0 * R.dx, ey = R.oy + t0 * R.dy, ez = R.oz + t0 * R.dz;
  R.cx = min(max((int32_t)floorf((ex - S.lo32[0]) * S.inv32[0]), 0), S.res[0] - 1);
  R.cy = min(max((int32_t)floorf((ey - S.lo32[1]) * S.inv32[1]), 0), S.res[1] - 1);
  R.cz = min(max((int32_t)floorf((ez - S.lo32[2]) * S.inv32[2]), 0), S.res[2] - 1);
  R.sx = R.dx > 0.0f ? 1 : (R.dx < 0.0f ? -1 : 0);
  R.sy = R.dy > 0.0f ? 1 : (R.dy < 0.0f ? -1 : 0);
  R.sz = R.dz > 0.0f ? 1 : (R.dz < 0.0f ? -1 : 0);
  R.bx = (S.lo32[0] - R.ox) * ix;
  R.by = (S.lo32[1] - R.oy) * iy;
  R.bz = (S.lo32[2] - R.oz) * iz;
  R.hx = S.h32[0] * ix;
  R.hy = S.h32[1] * iy;
  R.hz = S.h32[2] * iz;
  R.tnx = R.sx ? fmaf((float)(R.cx + (R.sx > 0)), R.hx, R.bx) : INFINITY;
  R.tny = R.sy ? fmaf((float)(R.cy + (R.sy > 0)), R.hy, R.by) : INFINITY;
  R.tnz = R.sz ? fmaf((float)(R.cz + (R.sz > 0)), R.hz, R.bz) : INFINITY;
  const uint32_t cell = ((uint32_t)R.cz * (uint32_t)S.res[1] + (uint32_t)R.cy) * (uint32_t)S.res[0] +
                        (uint32_t)R.cx;
  R.rc = S.cell_begin[cell];
  R.re = S.cell_begin[cell + 1];
  return true;
}

// FP64 re-solve of one sphere / cylinder test.
__device__ __noinline__ int resolve_f64(const SceneDev &S, int32_t k, const double o[3],
                                        const double d[3], double tmin, double tmax, double &t) {
  if (k < S.n_s) return hit_sphere_f64(S.sph64[k], o, d, tmin, tmax, t);
  return hit_cylinder_f64(S.cylA64[k - S.n_s], S.cylW64[k - S.n_s], o, d, tmin, tmax, t);
}

// The lane's ray promoted to FP64: primary rays are regenerated exactly from
// their pixel; secondary rays promote the FP32 origin and renormalise the
// direction.
__device__ __noinline__ void ray_f64(const Ray &R, bool primary, const JobDev *job, int32_t pi,
                                     int32_t pj, double o[3], double d[3]) {
  if (primary) {
    primary_ray_f64(*job, pi, pj, o, d);
    return;
  }
  o[0] = R.ox;
  o[1] = R.oy;
  o[2] = R.oz;
  const double v[3] = {(double)R.dx, (double)R.dy, (double)R.dz};
  const double n = sqrt(dot3d(v, v));
  d[0] = v[0] / n;
  d[1] = v[1] / n;
  d[2] = v[2] / n;
}

struct WaveArgs {
  const JobDev *jobs;
  int32_t n_jobs;
  int64_t n_tiles;
  uint32_t *tile_counter;
  uint64_t *stats;
  int32_t tile_w, refill_below;
};

__device__ __forceinline__ int32_t find_job(const JobDev *jobs, int32_t n, int64_t tile) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (jobs[mid].queue_begin <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Scene fields used by the traversal, loaded (wave-uniform) from the job
// table at the start of each phase.
struct SceneHot {
  const uint32_t *refs, *cell_begin;
  const float4 *sph32, *cylA32, *cylW32;
  int32_t n_s;
  int32_t res[3];
  float lo32[3], hi32[3], inv32[3], h32[3];
};

__device__ __forceinline__ SceneHot load_hot(const JobDev *J) {
  SceneHot H;
  H.refs = J->sc.refs;
  H.cell_begin = J->sc.cell_begin;
  H.sph32 = J->sc.sph32;
  H.cylA32 = J->sc.cylA32;
  H.cylW32 = J->sc.cylW32;
  H.n_s = J->sc.n_s;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    H.res[q] = J->sc.res[q];
    H.lo32[q] = J->sc.lo32[q];
    H.hi32[q] = J->sc.hi32[q];
    H.inv32[q] = J->sc.inv32[q];
    H.h32[q] = J->sc.h32[q];
  }
  return H;
}

template <int BANKS, bool RESOLVE, bool COUNT>
__global__ __launch_bounds__(64) void k_render_wave(const WaveArgs A) {
  __shared__ Lds<BANKS> L;
  __shared__ uint32_t cnt_sh[4];
  constexpr int NS = BANKS * 64;
  constexpr int kMinIters = 2;
  const int32_t lane = threadIdx.x;
  const int32_t TW = A.tile_w;
  const int32_t TH = 64 / TW;
  if (lane < 4) cnt_sh[lane] = 0;

  // ---- wave-uniform control state
  int32_t q_head = 0, q_tail = 0, head_issued = 0;
  int32_t issue_bank = -1, issue_next = 0;
  uint32_t bank_busy = 0;
  bool tiles_left = true;
  int64_t held_tile = -1;
  int32_t held_job = 0, held_key = -1;
  int32_t cur_key = -1;   // scene loaded in this wave
  int32_t scene_job = 0;  // a job whose scene is the current one
  int32_t issue_job = 0;  // job of issue_bank
  int32_t idle_rounds = 0;

  // ---- counters
  uint64_t c_cells = 0, c_st = 0, c_sh = 0, c_ct = 0, c_ch = 0, c_res = 0, c_rays = 0;
  uint32_t l_pix = 0, l_hit = 0, l_ao = 0, l_shadow = 0;  // per lane

  // ---- per-lane state
  int32_t kind = kIdle;
  bool done = false;
  int32_t slot = 0, ridx = 0;
  int32_t pi = 0, pj = 0;  // pixel of the lane's ray
  Ray R;
  R.bk = -1;
  R.rc = R.re = 0;
  __syncthreads();

  for (;;) {
    // ================================================================ finish
    if (__ballot(kind != kIdle && done)) {
      const bool fin = kind != kIdle && done;
      const bool fin_prim_hit = fin && kind == kPrimary && R.bk >= 0;
      const bool fin_prim_miss = fin && kind == kPrimary && R.bk < 0;
      bool finalize = fin_prim_miss;
      uint32_t nr = 0;
      if (fin_prim_hit) {
        const JobDev *jb = &A.jobs[L.bank_job[slot >> 6]];
        const SceneDev &S = jb->sc;
        const int32_t k = R.bk;
        const float t = R.bt;
        const float Px = R.ox + t * R.dx, Py = R.oy + t * R.dy, Pz = R.oz + t * R.dz;
        float Nx, Ny, Nz;
        if (k < S.n_s) {
          const float4 s = S.sph32[k];
          Nx = Px - s.x;
          Ny = Py - s.y;
          Nz = Pz - s.z;
        } else {
          const float4 a = S.cylA32[k - S.n_s], w = S.cylW32[k - S.n_s];
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
        const bool front = (Nx * R.dx + Ny * R.dy + Nz * R.dz) < 0.0f;
        if (!front) {
          Nx = -Nx;
          Ny = -Ny;
          Nz = -Nz;
        }
        uint32_t lv = 0;
        const int32_t nl = jb->n_lights;
        for (int l = 0; l < nl; ++l) {
          const float cl = Nx * jb->ldir32[l][0] + Ny * jb->ldir32[l][1] + Nz * jb->ldir32[l][2];
          if (cl > 0.0f) lv |= 1u << l;
        }
        nr = (uint32_t)jb->S + (uint32_t)__popc(lv);
        L.px[slot] = Px;
        L.py[slot] = Py;
        L.pz[slot] = Pz;
        L.nx[slot] = Nx;
        L.ny[slot] = Ny;
        L.nz[slot] = Nz;
        L.prim[slot] = k;
        L.skip[slot] = front ? k : -1;
        L.pending[slot] = (int32_t)nr;
        L.nrays[slot] = (int32_t)nr;
        L.lvalid[slot] = lv;
        L.aomask[slot] = 0;
        L.aocnt[slot] = 0;
        L.lmask[slot] = 0;
        if (nr == 0) finalize = true;
      }
      {  // queue hit slots that have secondary rays
        const bool enq = fin_prim_hit && nr > 0;
        const uint64_t m = __ballot(enq);
        if (enq) L.fifo[(q_tail + (int32_t)lane_rank(m)) % NS] = (uint8_t)slot;
        q_tail += __popcll(m);
      }
      if (fin && kind >= kShadow) {  // secondary results
        if (R.bk >= 0) {
          if (kind == kAO) {
            if (ridx < 32) atomicOr(&L.aomask[slot], 1u << ridx);
            atomicAdd(&L.aocnt[slot], 1);
          } else {
            atomicOr(&L.lmask[slot], 1u << ridx);
          }
        }
        const int32_t old = atomicSub(&L.pending[slot], 1);
        if (old == 1) finalize = true;
      }
      __syncthreads();
      if (finalize) {
        const int32_t bk = slot >> 6;
        const int32_t q = slot & 63;
        const int32_t vw = L.bank_vw[bk];
        const int32_t x = L.bank_x0[bk] + q % vw;
        const int32_t y = L.bank_y0[bk] + q / vw;
        const JobDev *J = &A.jobs[L.bank_job[bk]];
        const int64_t pid = (int64_t)y * J->W + x;
        float cr = J->bg[0], cg = J->bg[1], cb = J->bg[2];
        int32_t hid = -1;
        uint32_t am = 0, lm = 0;
        ++l_pix;
        if (!fin_prim_miss) {
          const int32_t k = L.prim[slot];
          hid = k;
          const float Nx = L.nx[slot], Ny = L.ny[slot], Nz = L.nz[slot];
          const uint32_t lv = L.lvalid[slot];
          lm = L.lmask[slot];
          am = L.aomask[slot];
          float Dr = 0.0f, Dg = 0.0f, Db = 0.0f;
          for (int l = 0; l < J->n_lights; ++l) {
            if (!((lv >> l) & 1u) || ((lm >> l) & 1u)) continue;
            const float cl = Nx * J->ldir32[l][0] + Ny * J->ldir32[l][1] + Nz * J->ldir32[l][2];
            Dr += J->lcol32[l][0] * cl;
            Dg += J->lcol32[l][1] * cl;
            Db += J->lcol32[l][2] * cl;
          }
          float ao = 1.0f;
          if (J->S > 0) ao = (float)(J->S - L.aocnt[slot]) / (float)J->S;
          const float4 alb = J->sc.albedo[k];
          const float sk = J->sky32 * ao;
          cr = fminf(fmaxf(alb.x * (Dr + sk), 0.0f), 1.0f);
          cg = fminf(fmaxf(alb.y * (Dg + sk), 0.0f), 1.0f);
          cb = fminf(fmaxf(alb.z * (Db + sk), 0.0f), 1.0f);
          ++l_hit;
          l_ao += (uint32_t)J->S;
          l_shadow += (uint32_t)__popc(lv);
        }
        J->rgb[pid * 3 + 0] = cr;
        J->rgb[pid * 3 + 1] = cg;
        J->rgb[pid * 3 + 2] = cb;
        if (J->hit_id) J->hit_id[pid] = hid;
        if (J->ao_mask) J->ao_mask[pid] = am;
        if (J->light_mask) J->light_mask[pid] = (uint8_t)lm;
        atomicAdd(&L.bank_done[bk], 1);
      }
      if (fin) kind = kIdle;
      __syncthreads();
      // free banks whose pixels are all shaded
      for (int b = 0; b < BANKS; ++b) {
        if (!((bank_busy >> b) & 1u)) continue;
        const bool all_issued = issue_bank != b || issue_next == L.bank_n[b];
        if (all_issued && uni(L.bank_done[b]) == uni(L.bank_n[b])) {
          bank_busy &= ~(1u << b);
          if (issue_bank == b) issue_bank = -1;
        }
      }
    }

    // ================================================================ refill
    {
      const uint64_t idle = __ballot(kind == kIdle);
      const int32_t n_idle = __popcll(idle);
      const int32_t rank = (int32_t)lane_rank(idle);
      const bool me_idle = kind == kIdle;
      int32_t assigned = 0;
      bool setup_ok = true;
      // secondary rays from the FIFO
      if (q_head != q_tail && n_idle > 0) {
        const SceneHot H = load_hot(&A.jobs[scene_job]);
        while (assigned < n_idle && q_head != q_tail) {
          const int32_t s = uni((int32_t)L.fifo[q_head % NS]);
          const int32_t nr = uni(L.nrays[s]);
          const int32_t take = min(nr - head_issued, n_idle - assigned);
          if (me_idle && rank >= assigned && rank < assigned + take) {
            slot = s;
            ridx = head_issued + (rank - assigned);
            const int32_t bk = s >> 6;
            const JobDev *J = &A.jobs[L.bank_job[bk]];
            const int32_t q = s & 63;
            const int32_t vw = L.bank_vw[bk];
            pi = L.bank_x0[bk] + q % vw;
            pj = L.bank_y0[bk] + q / vw;
            R.ox = L.px[s];
            R.oy = L.py[s];
            R.oz = L.pz[s];
            R.skip = L.skip[s];
            R.tmin = kEps;
            const int32_t S_ao = J->S;
            if (ridx < S_ao) {
              kind = kAO;
              uint32_t b1, b2;
              ao_uniform_bits((uint32_t)((int64_t)pj * J->W + pi), (uint32_t)ridx, J->view_id,
                              J->key0, J->key1, b1, b2);
              ao_dir_f32(L.nx[s], L.ny[s], L.nz[s], b1, b2, R.dx, R.dy, R.dz);
              R.tmax = J->ao_maxdist32;
            } else {
              kind = kShadow;
              uint32_t lv = L.lvalid[s];  // the (ridx - S)-th light with N.L > 0
              for (int32_t n = ridx - S_ao; n > 0; --n) lv &= lv - 1;
              const int32_t l = __ffs(lv) - 1;
              ridx = l;
              R.dx = J->ldir32[l][0];
              R.dy = J->ldir32[l][1];
              R.dz = J->ldir32[l][2];
              R.tmax = INFINITY;
            }
            setup_ok = ray_setup(R, H);
            done = !setup_ok;
          }
          head_issued += take;
          assigned += take;
          if (head_issued == nr) {
            ++q_head;
            head_issued = 0;
          }
        }
      }
      // primary rays
      while (assigned < n_idle) {
        if (issue_bank < 0 || issue_next == uni(L.bank_n[issue_bank])) {
          issue_bank = -1;
          const uint32_t free_banks = ~bank_busy & ((1u << BANKS) - 1u);
          if (!free_banks) break;
          if (held_tile < 0) {
            if (!tiles_left) break;
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(A.tile_counter, 1u);
            t = (uint32_t)uni((int32_t)t);
            if ((int64_t)t >= A.n_tiles) {
              tiles_left = false;
              break;
            }
            held_tile = t;
            held_job = uni(find_job(A.jobs, A.n_jobs, held_tile));
            held_key = uni(A.jobs[held_job].scene_key);
          }
          if (held_key != cur_key) {
            if (bank_busy) break;  // drain this scene's banks before switching
            cur_key = held_key;
            scene_job = held_job;
          }
          const JobDev *J = &A.jobs[held_job];
          const int32_t b = __ffs(free_banks) - 1;
          const int64_t tl = held_tile - J->queue_begin + J->tile_begin;
          const int32_t tx = (int32_t)(tl % J->tiles_x), ty = (int32_t)(tl / J->tiles_x);
          const int32_t x0 = tx * TW, y0 = ty * TH;
          const int32_t vw = min(TW, J->W - x0), vh = min(TH, J->H - y0);
          if (lane == 0) {
            L.bank_job[b] = held_job;
            L.bank_x0[b] = x0;
            L.bank_y0[b] = y0;
            L.bank_vw[b] = vw;
            L.bank_n[b] = vw * vh;
            L.bank_done[b] = 0;
          }
          __syncthreads();
          bank_busy |= 1u << b;
          issue_bank = b;
          issue_job = held_job;
          issue_next = 0;
          held_tile = -1;
        }
        const int32_t nvalid = uni(L.bank_n[issue_bank]);
        const int32_t take = min(nvalid - issue_next, n_idle - assigned);
        if (me_idle && rank >= assigned && rank < assigned + take) {
          const int32_t q = issue_next + (rank - assigned);
          slot = issue_bank * 64 + q;
          const JobDev *J = &A.jobs[issue_job];
          const SceneHot H = load_hot(J);
          const int32_t vw = L.bank_vw[issue_bank];
          pi = L.bank_x0[issue_bank] + q % vw;
          pj = L.bank_y0[issue_bank] + q / vw;
          kind = kPrimary;
          const float x = ((2.0f * ((float)pi + 0.5f)) / (float)J->W - 1.0f) * J->th32 * J->aspect32;
          const float y = (1.0f - (2.0f * ((float)pj + 0.5f)) / (float)J->H) * J->th32;
          const float vx = J->f32[0] + x * J->r32[0] + y * J->u32[0];
          const float vy = J->f32[1] + x * J->r32[1] + y * J->u32[1];
          const float vz = J->f32[2] + x * J->r32[2] + y * J->u32[2];
          const float inv = __builtin_amdgcn_rsqf(vx * vx + vy * vy + vz * vz);
          R.dx = vx * inv;
          R.dy = vy * inv;
          R.dz = vz * inv;
          R.ox = J->eye32[0];
          R.oy = J->eye32[1];
          R.oz = J->eye32[2];
          R.tmin = 0.0f;
          R.tmax = INFINITY;
          R.skip = -1;
          setup_ok = ray_setup(R, H);
          done = !setup_ok;
        }
        issue_next += take;
        assigned += take;
      }
      c_rays += (uint64_t)assigned;
      if (COUNT) c_cells += __popcll(__ballot(me_idle && kind != kIdle && setup_ok));
    }

    // ================================================================ exit
    {
      const uint64_t busy = __ballot(kind != kIdle);
      if (!busy) {
        if (!tiles_left && held_tile < 0 && bank_busy == 0 && q_head == q_tail) break;
        if (++idle_rounds > 4) {  // cannot happen when the bookkeeping is right
          if (lane == 0) atomicAdd(A.tile_counter + 1, 1u);
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
          q_head != q_tail || (issue_bank >= 0 && issue_next < uni(L.bank_n[issue_bank])) ||
          (free_banks && ((held_tile < 0 && tiles_left) || (held_tile >= 0 && (held_key == cur_key || !bank_busy))));
      const SceneHot H = load_hot(&A.jobs[scene_job]);
      const JobDev *const jobs = A.jobs;
      for (int32_t it = 0;; ++it) {
        const bool work = kind != kIdle && !done;
        const int32_t nwork = __popcll(__ballot(work));
        if (nwork == 0) break;
        if (it >= kMinIters) {
          if (can_refill && nwork < A.refill_below) break;
          // finished primaries would queue new rays
          if (nwork < A.refill_below && __ballot(kind == kPrimary && done)) break;
        }
        if (work) {
          if (R.rc < R.re) {
            // ---- test one primitive reference
            const int32_t k = (int32_t)H.refs[R.rc];
            ++R.rc;
            if (k != R.skip) {
              float t = 0.0f;
              bool hit = false;
              bool graze = false;
              if (k < H.n_s) {
                if (COUNT) c_st += __popcll(__ballot(true));
                const float4 s = H.sph32[k];
                const float qx = s.x - R.ox, qy = s.y - R.oy, qz = s.z - R.oz;
                const float b = qx * R.dx + qy * R.dy + qz * R.dz;
                const float lx = qx - b * R.dx, ly = qy - b * R.dy, lz = qz - b * R.dz;
                const float ll = lx * lx + ly * ly + lz * lz;
                const float rr = s.w * s.w;
                const float disc = rr - ll;
                if (RESOLVE && fabsf(disc) <= kKappa * (rr + ll)) {
                  graze = true;
                } else if (disc >= 0.0f) {
                  const float sq = sqrtf_fast(disc);
                  const float t0 = b - sq, t1 = b + sq;
                  if (t0 > R.tmin && t0 <= R.tmax) {
                    t = t0;
                    hit = true;
                  } else if (t1 > R.tmin && t1 <= R.tmax) {
                    t = t1;
                    hit = true;
                  }
                }
                if (COUNT) c_sh += __popcll(__ballot(hit));
              } else {
                if (COUNT) c_ct += __popcll(__ballot(true));
                const float4 a = H.cylA32[k - H.n_s];
                const float4 w = H.cylW32[k - H.n_s];
                const float Dx = R.ox - a.x, Dy = R.oy - a.y, Dz = R.oz - a.z;
                const float dw = R.dx * w.x + R.dy * w.y + R.dz * w.z;
                const float Dw = Dx * w.x + Dy * w.y + Dz * w.z;
                const float dpx = R.dx - dw * w.x, dpy = R.dy - dw * w.y, dpz = R.dz - dw * w.z;
                const float Dpx = Dx - Dw * w.x, Dpy = Dy - Dw * w.y, Dpz = Dz - Dw * w.z;
                const float Aq = dpx * dpx + dpy * dpy + dpz * dpz;
                const float Bq = dpx * Dpx + dpy * Dpy + dpz * Dpz;
                const float Cq = (Dpx * Dpx + Dpy * Dpy + Dpz * Dpz) - a.w * a.w;
                if (Aq > 1e-12f) {
                  const float disc = Bq * Bq - Aq * Cq;
                  if (RESOLVE && fabsf(disc) <= kKappa * (Bq * Bq + fabsf(Aq * Cq))) {
                    graze = true;
                  } else if (disc >= 0.0f) {
                    const float sq = sqrtf_fast(disc);
                    const float qq = -(Bq + __builtin_copysignf(sq, Bq));
                    if (qq != 0.0f) {
                      const float r0 = qq * rcpf(Aq), r1 = Cq * rcpf(qq);
                      const float tl = fminf(r0, r1), th = fmaxf(r0, r1);
                      const float kL = kKappa * w.w;
                      if (tl > R.tmin && tl <= R.tmax) {
                        const float sa = Dw + tl * dw;
                        if (RESOLVE && (fabsf(sa) <= kL || fabsf(sa - w.w) <= kL)) {
                          graze = true;
                        } else if (sa >= 0.0f && sa <= w.w) {
                          t = tl;
                          hit = true;
                        }
                      }
                      if (!hit && !graze && th > R.tmin && th <= R.tmax) {
                        const float sa = Dw + th * dw;
                        if (RESOLVE && (fabsf(sa) <= kL || fabsf(sa - w.w) <= kL)) {
                          graze = true;
                        } else if (sa >= 0.0f && sa <= w.w) {
                          t = th;
                          hit = true;
                        }
                      }
                    }
                  }
                }
                if (COUNT) c_ch += __popcll(__ballot(hit));
              }
              if (RESOLVE && graze) {
                if (COUNT) c_res += __popcll(__ballot(true));
                double o64[3], d64[3], t64 = 0.0;
                const JobDev *jr = &jobs[L.bank_job[slot >> 6]];
                ray_f64(R, kind == kPrimary, jr, pi, pj, o64, d64);
                const double tmin64 = kind == kPrimary ? 0.0 : kEpsD;
                const double tmax64 = kind == kAO ? jr->ao_maxdist : INFINITY;
                if (resolve_f64(jr->sc, k, o64, d64, tmin64, tmax64, t64)) {
                  hit = true;
                  t = (float)t64;
                }
              }
              if (hit) {
                if (kind != kPrimary) {
                  R.bk = k;
                  R.bt = t;
                  done = true;
                } else if (t < R.bt || (t == R.bt && k < R.bk)) {
                  R.bt = t;
                  R.bk = k;
                }
              }
            }
          } else {
            // ---- cell exhausted: stop, or step to the next cell
            const float tn = fminf(R.tnx, fminf(R.tny, R.tnz));
            const float t_exit = fminf(tn, R.t1);
            if ((R.bk >= 0 && R.bt <= t_exit) || !(tn < R.t1)) {
              done = true;
            } else {
              int32_t st;
              if (R.tnx == tn) {
                st = R.sx;
                R.cx += R.sx;
                R.tnx = fmaf((float)(R.cx + (R.sx > 0)), R.hx, R.bx);
              } else if (R.tny == tn) {
                st = R.sy;
                R.cy += R.sy;
                R.tny = fmaf((float)(R.cy + (R.sy > 0)), R.hy, R.by);
              } else {
                st = R.sz;
                R.cz += R.sz;
                R.tnz = fmaf((float)(R.cz + (R.sz > 0)), R.hz, R.bz);
              }
              if (st == 0 || (uint32_t)R.cx >= (uint32_t)H.res[0] ||
                  (uint32_t)R.cy >= (uint32_t)H.res[1] || (uint32_t)R.cz >= (uint32_t)H.res[2]) {
                done = true;
              } else {
                if (COUNT) c_cells += __popcll(__ballot(true));
                const uint32_t cell =
                    ((uint32_t)R.cz * (uint32_t)H.res[1] + (uint32_t)R.cy) * (uint32_t)H.res[0] +
                    (uint32_t)R.cx;
                R.rc = H.cell_begin[cell];
                R.re = H.cell_begin[cell + 1];
              }
            }
          }
        }
      }
    }
  }

  // ---- counters
  if (A.stats) {
    atomicAdd(&cnt_sh[0], l_pix);
    atomicAdd(&cnt_sh[1], l_hit);
    atomicAdd(&cnt_sh[2], l_ao);
    atomicAdd(&cnt_sh[3], l_shadow);
    __syncthreads();
    if (lane == 0) {
      unsigned long long *st = (unsigned long long *)A.stats;
      atomicAdd(&st[TR_STAT_PIXELS], (unsigned long long)cnt_sh[0]);
      atomicAdd(&st[TR_STAT_HIT_PIXELS], (unsigned long long)cnt_sh[1]);
      atomicAdd(&st[TR_STAT_AO_RAYS], (unsigned long long)cnt_sh[2]);
      atomicAdd(&st[TR_STAT_SHADOW_RAYS], (unsigned long long)cnt_sh[3]);
      atomicAdd(&st[TR_STAT_RAYS_TRACED], (unsigned long long)c_rays);
      if (COUNT) {
        atomicAdd(&st[TR_STAT_CELLS], (unsigned long long)c_cells);
        atomicAdd(&st[TR_STAT_SPH_TESTS], (unsigned long long)c_st);
        atomicAdd(&st[TR_STAT_SPH_HITS], (unsigned long long)c_sh);
        atomicAdd(&st[TR_STAT_CYL_TESTS], (unsigned long long)c_ct);
        atomicAdd(&st[TR_STAT_CYL_HITS], (unsigned long long)c_ch);
        atomicAdd(&st[TR_STAT_RESOLVES], (unsigned long long)c_res);
      }
    }
  }
}

__global__ void k_zero_u32(uint32_t *p) { *p = 0u; }

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
  ao_uniform_bits(pix[i], smp[i], view, k0, k1, b1, b2);
  ao_dir_f32(nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2], b1, b2, w[3 * i], w[3 * i + 1], w[3 * i + 2]);
}

}  // namespace

namespace trh {

template <int BANKS, bool RES, bool CNT>
static hipError_t launch_t(const WaveLaunch &L, hipStream_t st) {
  WaveArgs a;
  a.jobs = L.jobs;
  a.n_jobs = L.n_jobs;
  a.n_tiles = L.n_tiles;
  a.tile_counter = L.tile_counter;
  a.stats = L.stats;
  a.tile_w = L.tile_w;
  a.refill_below = L.refill_below;
  k_render_wave<BANKS, RES, CNT><<<L.n_waves, 64, 0, st>>>(a);
  return hipGetLastError();
}

template <int BANKS>
static hipError_t launch_b(const WaveLaunch &L, hipStream_t st) {
  const bool cnt = L.count_ops != 0 && L.stats != nullptr;
  if (L.resolve) return cnt ? launch_t<BANKS, true, true>(L, st) : launch_t<BANKS, true, false>(L, st);
  return cnt ? launch_t<BANKS, false, true>(L, st) : launch_t<BANKS, false, false>(L, st);
}

hipError_t launch_render_wave(const WaveLaunch &L, hipStream_t st) {
  if (L.banks == 3) return launch_b<3>(L, st);
  return launch_b<2>(L, st);
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
