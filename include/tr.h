/*
 * tr.h -- C ABI of the MI355X (gfx950) ambient-occlusion ray caster.
 *
 * The calls follow the paper's statement of the problem (McGuigan, "Toward
 * the Graphics Turing Scale on a Blue Gene Supercomputer", Sec. 2, Strong
 * scaling): a molecular scene of spheres and cylinders, an image resolution
 * given as width x height (the -res option), a rescale factor for the
 * scene's direct lights (-rescale_lights), the strength of ambient-occlusion
 * sky lighting computed by Monte Carlo sampling (-add_skylight), and an RGB
 * frame out (the "Image I/O" phase of Table 5).  The acceleration build is
 * the "Preprocess" phase and rendering is the "Ray Tracing" phase (Table 5).
 *
 * Conventions for every call:
 *  - Plain C types only; no exception crosses the ABI.  Every call returns a
 *    tr_status (or a value documented below) and records a message readable
 *    through tr_last_error() on the calling thread.
 *  - Host pointers are read only during the call and are copied; the caller
 *    keeps ownership.  Device pointers (frame buffers, stats) are owned by
 *    the caller, must be allocated on the current HIP device, and must stay
 *    valid until the work enqueued on the given stream has completed.
 *  - `hip_stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Render calls validate synchronously, enqueue, and return without
 *    waiting; a device fault surfaces as TR_EDEVICE on a later call or on a
 *    stream synchronisation.
 *  - Results depend only on (scene, camera, params, pixel): never on batch
 *    composition, tile shape, queue depth, cells per primitive, or the
 *    order of primitive references (a determinism contract).
 */
#ifndef TR_H
#define TR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TR_ABI_VERSION 4

typedef enum {
  TR_OK = 0,
  TR_EINVAL = -1,        /* an argument failed validation; nothing enqueued */
  TR_ENOMEM = -2,        /* device or host allocation failed                */
  TR_EDEVICE = -3,       /* a HIP call failed (message has the HIP error)   */
  TR_EUNSUPPORTED = -4   /* a valid request this build does not implement   */
} tr_status;

/* Arithmetic of the render.  The paper's renderer computes in double
 * precision throughout (Sec. 2).  TR_PREC_FP64 is that plain FP64 path on
 * the GPU (one thread per pixel).  TR_PREC_FP32 intersects and shades in
 * FP32 in the persistent-wavefront kernel; TR_PREC_FP32_RESOLVE adds an
 * FP64 re-solve of near-grazing sphere/cylinder tests (the default). */
typedef enum {
  TR_PREC_FP64 = 0,
  TR_PREC_FP32 = 1,
  TR_PREC_FP32_RESOLVE = 2
} tr_precision;

/* Opaque scene: primitives, albedo, lights and the uniform grid, resident on
 * the device it was built on.  Immutable after build except through
 * tr_scene_rebuild (which rebuilds the grid from the resident arrays). */
typedef struct tr_scene tr_scene;

/* Scene description (Sec. 2: the 26,318 "objects" of the molecular scene
 * are spheres and cylinders; triangles carry surface representations).
 * Global primitive id: spheres [0, n_spheres), cylinders [n_spheres,
 * n_spheres + n_cylinders), then triangles.  Arrays are row-major xyz
 * triples.  Any count may be 0 (an empty scene renders background). */
typedef struct {
  int64_t n_spheres;
  const double *sph_center;  /* [n_spheres*3]                               */
  const double *sph_radius;  /* [n_spheres], > 0                            */
  const float *sph_rgb;      /* [n_spheres*3] albedo                        */
  int64_t n_cylinders;
  const double *cyl_a;       /* [n_cylinders*3] first end point             */
  const double *cyl_b;       /* [n_cylinders*3] second end point, != cyl_a  */
  const double *cyl_radius;  /* [n_cylinders], > 0                          */
  const float *cyl_rgb;      /* [n_cylinders*3] albedo                      */
  int32_t n_lights;          /* 0..8 directional lights                     */
  const double *light_dir;   /* [n_lights*3] toward the light; normalised by the library */
  const double *light_rgb;   /* [n_lights*3] intensity                      */
  double cells_per_prim;     /* grid density lambda; 0 => 24.  Speed only.  */
  const float *sph_opacity;  /* [n_spheres] opacity in (0, 1], or NULL = opaque */
  const float *cyl_opacity;  /* [n_cylinders] opacity in (0, 1], or NULL = opaque;
                                used only by renders with tr_params.max_layers > 1 */
  int64_t n_triangles;       /* triangles (surface representations), ids
                                n_spheres + n_cylinders + [0, n_triangles);
                                n_spheres + n_cylinders + n_triangles < 2^27   */
  const double *tri_v0;      /* [n_triangles*3] vertices, finite; two-sided,
                                hit by the Moller-Trumbore test with the edges
                                inside; a zero-area triangle is never hit     */
  const double *tri_v1;
  const double *tri_v2;
  const float *tri_rgb;      /* [n_triangles*3] albedo                      */
  const float *tri_opacity;  /* [n_triangles] opacity in (0, 1], or NULL     */
  int32_t max_skip;          /* empty-space skipping: the walk jumps over empty
                                cells using each empty cell's Chebyshev distance
                                to the nearest occupied cell, stored up to this
                                cap, 1..32; 0 => 32; 1 => no jumps (a plain
                                3D-DDA).  Speed only.                          */
} tr_scene_desc;

/* Pinhole camera, one ray through each pixel centre (more with
 * tr_params.aa_samples).  width = horizontal
 * pixel count, height = vertical (the -res W H option, Sec. 2).  Row 0 of
 * the frame is the top of the image, column 0 the left. */
typedef struct {
  double eye[3], lookat[3], up[3];
  double fovy_deg;           /* vertical field of view, (0, 180)            */
  int32_t width, height;     /* > 0, width*height <= 2^31 - 1               */
} tr_camera;

typedef struct {
  double light_rescale;      /* -rescale_lights (paper: 0.3)                */
  double skylight;           /* -add_skylight   (paper: 1.0); AO is cast only if > 0 */
  int32_t ao_samples;        /* AO rays per hit pixel, 0..65535             */
  double ao_maxdist;         /* AO ray length, > 0; INFINITY = unbounded    */
  uint64_t seed;             /* Philox key (low word, high word)            */
  uint32_t view_id;          /* third Philox counter word (frame / view)    */
  int32_t precision;         /* tr_precision                                */
  float background[3];       /* colour of pixels whose primary ray misses   */
  int32_t aa_samples;        /* primary samples per pixel (antialiasing), 0..256;
                                0 and 1 = the pixel centre only.  With A > 1,
                                sample 0 is the centre and sample a >= 1 a point
                                (i + x, j + y) of the pixel square, x and y the top
                                24 bits of words 0 and 1 of Philox counter (pix, a,
                                view_id, 0xFFFFFFFF) times 2^-24; AO sample s of
                                sample a uses counter (pix, s, view_id, a).  rgb is
                                the mean of the A clamped colours (summed in
                                sample order, then divided by A); hit_id and the
                                masks are sample 0's.  Costs (A - 1) * W * H * 12
                                bytes of library workspace per frame (kept per
                                stream, grown on demand with a synchronising
                                hipMalloc); not with tile ranges or graphs.  A
                                zero-filled struct of ABI 1 means one sample.  */
  double specular;           /* Phong highlight strength k_s, finite, >= 0 (0 = none) */
  double shininess;          /* Phong exponent n, finite, > 0 (read only if k_s > 0).
                                The highlight (a shading option of the renderer
                                the paper drives, not used in its runs) adds
                                light_rescale * sum_l I_l V_l k_s max(0, R_l.V)^n,
                                white, to the albedo-scaled colour before the
                                clamp; R_l is the light direction mirrored about
                                N, V the unit direction back to the eye, and the
                                sum runs over the lights with N.L_l > 2^-40. */
  int32_t max_layers;        /* transparency (the -trans_vmd option, Sec. 2),
                                0..64; 0 and 1 = opaque rendering.  With L > 1 a
                                primary ray that hits a primitive of opacity
                                alpha < 1 continues through it from the hit
                                point (t > 1e-4, same line, skipping it only when
                                leaving it), up to L surfaces; each surface is
                                shaded as an opaque one (shadow and AO rays see
                                all primitives as opaque; AO counter word 1 =
                                s + 2^16 * layer) and the pixel is
                                sum_i (prod_{j<i} (1 - alpha_j)) alpha_i C_i plus
                                the remaining transmittance times background.
                                hit_id and the masks are the first surface's. */
} tr_params;

/* Device output buffers, caller-owned.  Only rgb is required.
 *  rgb        float  [height][width][3], linear, clamped to [0, 1]
 *  hit_id     int32  [height][width], global primitive id or -1 (miss)
 *  ao_mask    uint32 [height][width], bit s = AO sample s occluded (needs
 *             ao_samples <= 32 when non-NULL)
 *  light_mask uint8  [height][width], bit l = light l cast a shadow ray and
 *             it was blocked
 *  stats      uint64 [TR_STAT_COUNT], counts ADDED atomically (zero it
 *             first); NULL = no counting. */
typedef struct {
  float *rgb;
  int32_t *hit_id;
  uint32_t *ao_mask;
  uint8_t *light_mask;
  uint64_t *stats;
} tr_frame;

/* Indices into tr_frame.stats.  The first five are always exact; the
 * traversal counters (cells onward) are filled only by precise-counting
 * renders (tr_tune.count_ops = 1 or the FP64 path). */
enum {
  TR_STAT_PIXELS = 0,        /* primary rays                                */
  TR_STAT_HIT_PIXELS,        /* primary rays that hit                       */
  TR_STAT_AO_RAYS,           /* AO rays cast                                */
  TR_STAT_SHADOW_RAYS,       /* light shadow rays cast (N.L > 2^-40)        */
  TR_STAT_RAYS_TRACED,       /* all rays handed to a traversal              */
  TR_STAT_CELLS,             /* grid cells visited (the FP32 walk skips runs of empty cells) */
  TR_STAT_SPH_TESTS,
  TR_STAT_SPH_HITS,
  TR_STAT_CYL_TESTS,
  TR_STAT_CYL_HITS,
  TR_STAT_RESOLVES,          /* FP64 re-solves of near-grazing tests        */
  TR_STAT_WAVE_ITERS,        /* wavefront kernel: traversal-loop iterations (per wave) */
  TR_STAT_LANE_ITERS,        /* wavefront kernel: busy lanes summed over those iterations */
  TR_STAT_REFILLS,           /* wavefront kernel: finish/refill rounds (per wave) */
  TR_STAT_JUMPS,             /* wavefront kernel: empty-space jumps over more than one cell */
  TR_STAT_CYCLES_TRAVERSE,   /* wavefront kernel: shader clocks in the traversal loop (summed over waves) */
  TR_STAT_CYCLES_TOTAL,      /* wavefront kernel: shader clocks from wave start to end (summed) */
  TR_STAT_TRI_TESTS,
  TR_STAT_TRI_HITS,
  TR_STAT_STACK_OVERFLOWS,   /* BVH walk: children dropped on a full stack (0 unless the tree is too deep) */
  TR_STAT_STALLS,            /* wavefront kernel: waves that left with work outstanding (an
                                internal-error guard: always 0 unless the queue bookkeeping broke,
                                and then the frame is incomplete) */
  TR_STAT_RESOLVES_SPH,      /* FP64 re-solves split by primitive kind ... */
  TR_STAT_RESOLVES_CYL,
  TR_STAT_RESOLVES_TRI,
  TR_STAT_RESOLVES_NEAREST,  /* ... and those of nearest-hit (primary, continuation) rays;
                                the rest are shadow and AO rays */
  TR_STAT_SIGNS_F64,         /* triangle hits whose facing, N.L and AO-basis signs were
                                decided from the FP64 vertices (a sign within 2^-12 of 0) */
  TR_STAT_CELLS_AO,          /* wavefront kernel: cells entered and primitive tests (with the */
  TR_STAT_TESTS_AO,          /*   skipped ones) by AO rays ...                               */
  TR_STAT_CELLS_SHADOW,      /* ... and by light shadow rays (the rest: nearest-hit rays)   */
  TR_STAT_TESTS_SHADOW,
  TR_STAT_TESTS_OWN,         /* tests that met the primitive a secondary ray leaves (skipped) */
  TR_STAT_CYCLES_RESOLVE,    /* wavefront kernel: shader clocks (summed over waves) in the FP64 */
  TR_STAT_CYCLES_FINISH,     /*   re-solve, finish (shading, write) and refill (queue, ray */
  TR_STAT_CYCLES_REFILL,     /*   setup) phases; the traversal loop is TR_STAT_CYCLES_TRAVERSE */
  TR_STAT_COUNT
};

/* Launch shape of the persistent-wavefront kernel.  Any valid choice of the
 * shape fields gives bit-identical frames; only speed changes.  accel picks
 * the acceleration structure instead (see there).  Zero fields take
 * defaults. */
typedef struct {
  int32_t tile_w;            /* tile width in pixels: 4, 8, 16, 32 or 64; tiles hold 64
                                pixels (default 64: one row segment per tile) */
  int32_t banks;             /* pixel banks (tiles in flight) per wave: 2 or 3 (queue depth) */
  int32_t waves_per_cu;      /* persistent waves launched per compute unit, 1..32 */
  int32_t refill_below;      /* refill when fewer than this many lanes are busy, 1..64 */
  int32_t count_ops;         /* 1 = also fill the traversal counters of tr_frame.stats */
  int32_t accel;             /* 0 = walk the uniform grid; 1 = walk the scene's
                                BVH (tr_scene_build_bvh first; FP32 precisions,
                                opaque rendering, two banks).  Both walks meet
                                the same FP32 bar against the FP64 reference;
                                they test primitives in different orders, so a
                                near-tie in FP32 can settle differently (tested:
                                >= 99.99% of pixels with the same hit and masks,
                                the same colour wherever they agree). */
  int32_t stripe;            /* tiles per stripe of the tile queue, a power of two 1..1024:
                                stripe s of the frame's row-major tiles goes to XCD s mod 8,
                                whose waves take it before the other XCDs' stripes */
} tr_tune;

/* ---------------------------------------------------------------- scenes */

/* Validate the description, copy the arrays to the device (FP64 and packed
 * FP32 structure-of-arrays), and build the uniform grid on the GPU: bounds
 * reduction, per-cell counting, exclusive prefix scan, scatter of primitive
 * references and an in-cell sort (the "Preprocess" phase, Table 5).  Blocks
 * on the stream once to read back the scene bounds.  *out receives the new
 * scene; TR_EINVAL on a NULL required pointer, negative count, non-finite
 * coordinate, radius <= 0, zero-length cylinder, n_lights outside 0..8, an
 * opacity outside (0, 1], cells_per_prim < 0 or n_spheres + n_cylinders +
 * n_triangles >= 2^27; TR_EUNSUPPORTED when the grid's primitive
 * references and cells together would pass 2^29 - 1. */
tr_status tr_scene_build(const tr_scene_desc *desc, void *hip_stream, tr_scene **out);

/* Rebuild the grid from the resident device arrays (same result as the
 * build's grid), with cells_per_prim (0 = keep the current value).  After a
 * failed rebuild the scene renders nothing (TR_EINVAL) until a rebuild
 * succeeds. */
tr_status tr_scene_rebuild(tr_scene *scene, double cells_per_prim, void *hip_stream);

/* Set the empty-space skipping cap (tr_scene_desc.max_skip, 0..32) and
 * rebuild the grid as tr_scene_rebuild does.  Rendered results do not
 * depend on it; 1 gives the plain uniform-grid walk for comparison.
 * TR_EINVAL on a NULL scene or a cap outside 0..32. */
tr_status tr_scene_set_max_skip(tr_scene *scene, int32_t max_skip, void *hip_stream);

/* Build (or rebuild) a linear BVH over the scene's primitives for the BVH
 * walk (tr_tune.accel = 1), the alternative to the uniform grid: primitives
 * ordered by the 30-bit Morton code of their box centres over the grid box,
 * the hierarchy of Karras (HPG 2012), node boxes bottom-up (widened by the
 * grid's insertion margin, rounded outwards to FP32).  Synchronises the
 * stream.  TR_EINVAL on a NULL scene or an invalid grid; TR_EUNSUPPORTED from
 * 2^26 primitives on.  The walk keeps one deferred sibling per level on a
 * 48-entry stack per ray: rendering through a tree deeper than 48 internal
 * nodes (tr_scene_bvh_nodes reports the depth) fails with TR_EUNSUPPORTED
 * before any launch. */
tr_status tr_scene_build_bvh(tr_scene *scene, void *hip_stream);

/* Copy the BVH's records to a HOST buffer (may be NULL) of 16 floats per
 * internal node: left child box (lo xyz, hi xyz), right child box, then the
 * two children as int32 bit patterns (node index >= 0, or -(primitive id) - 1
 * for a leaf) and two zero words.  Boxes are in the FP32 frame (relative to
 * the grid box centre).  *n_nodes = primitives - 1 (0 below two); *depth
 * (may be NULL) = internal nodes on the longest root-to-leaf path (0 when no
 * BVH is built).  TR_EINVAL on a NULL scene or n_nodes. */
tr_status tr_scene_bvh_nodes(const tr_scene *scene, float *nodes, int64_t *n_nodes,
                             int32_t *depth, void *hip_stream);

/* Device bytes held by the scene (arrays + grid). */
tr_status tr_scene_footprint(const tr_scene *scene, size_t *bytes);

/* Grid shape: lo/hi bounds, resolution, reference count, and the grid's
 * cells-per-primitive value. */
tr_status tr_scene_grid_info(const tr_scene *scene, double lo[3], double hi[3], int32_t res[3],
                             int64_t *n_refs);

/* Copy the grid arrays to HOST buffers: cell_begin [n_cells+1] and refs
 * [n_refs] (either may be NULL).  Synchronises the stream. */
tr_status tr_scene_grid_arrays(const tr_scene *scene, uint32_t *cell_begin, uint32_t *refs,
                               void *hip_stream);

/* Binary scene files (the "Parse" phase of Table 5, for which the paper gives
 * no format).  Little-endian: char magic[8] = "TRSCENE1"; int64 n_spheres,
 * n_cylinders; int32 n_lights, int32 flags; double cells_per_prim; then the
 * arrays of tr_scene_desc in its order (sph_center, sph_radius, sph_rgb,
 * cyl_a, cyl_b, cyl_radius, cyl_rgb, light_dir, light_rgb), each padded to a
 * multiple of 8 bytes; with flags bit 1 (written when there are triangles)
 * then int64 n_triangles, tri_v0, tri_v1, tri_v2, tri_rgb; with flags bit 0
 * (written when some opacity is below 1) then sph_opacity, cyl_opacity and,
 * with bit 1, tri_opacity, padded likewise.  Other flag bits must be 0.
 * tr_scene_save writes the description the scene was built from (the FP64
 * arrays, albedo, the lights as given, the grid density); synchronises the
 * stream; TR_EINVAL on a NULL argument or a failed write.
 * tr_scene_load reads a file and builds it with tr_scene_build (same scene as
 * building that description directly); TR_EINVAL on a NULL argument, an
 * unreadable file, a bad magic, bad counts or a size that does not match the
 * counts, and tr_scene_build's errors otherwise. */
tr_status tr_scene_save(const tr_scene *scene, const char *path, void *hip_stream);
tr_status tr_scene_load(const char *path, void *hip_stream, tr_scene **out);

/* Copy the FP32 walk's view of the grid to HOST buffers (either may be NULL):
 * cellinfo [2 * n_cells], per cell (byte offset of its list in wrefs, the
 * list's first entry), or for an empty cell (-d, x): d the Chebyshev
 * distance in cells to the nearest occupied cell, capped at the scene's
 * max_skip (32 by default), and x with bit 31 set and, in bits 3o..3o+2, M_o
 * for octant o of a ray's direction (bit a of o set when the direction is
 * negative on axis a): the largest m <= min(7, (max_skip - 1) / 2) such that
 * for every m' in 1..m the cell m' steps along the octant's diagonal lies in
 * the grid with distance >= m' + 1, i.e. the block of 2m + 1 cells per axis
 * ahead of the cell in that octant is empty (a ray in that octant jumps
 * max(d, 2 M_o + 1) cells); and wrefs
 * [*n_walk], per occupied cell in cell order its references in ascending id,
 * each stored as 16 x id (the byte offset of the primitive's 16-byte FP32
 * records) with bit 0 set on the list's last entry, then 0xFFFFFFFF.  *n_walk (required) receives the wrefs length.  Derived
 * from the canonical grid of tr_scene_grid_arrays; synchronises the stream. */
tr_status tr_scene_walk_arrays(const tr_scene *scene, int32_t *cellinfo, uint32_t *wrefs,
                               int64_t *n_walk, void *hip_stream);

/* Free the scene's device memory.  The caller guarantees no enqueued work
 * still uses it (the call synchronises the device before freeing). */
void tr_scene_destroy(tr_scene *scene);

/* ---------------------------------------------------------------- render */

/* Render one frame (the "Ray Tracing" phase, Table 5): per pixel, the
 * nearest hit of the camera ray; on a hit, the viewer-facing normal, one
 * shadow ray per light with N.L > 2^-40 (at or below, N.L is rounding noise of
 * a light in the plane of the surface, and the light adds nothing), and
 * params->ao_samples AO rays drawn
 * from the cosine-weighted hemisphere with Philox4x32-10 uniforms keyed by
 * (pixel, sample, view_id) and seed; colour = clamp(albedo * (light_rescale
 * * sum_l I_l (N.L_l) V_l + skylight * AO) + highlight, 0, 1) (highlight:
 * tr_params.specular).  Enqueued on the
 * stream.  TR_EINVAL on a NULL scene/camera/params/frame->rgb, width or
 * height <= 0 or width*height >= 2^31, fovy outside (0, 180), eye == lookat,
 * up parallel to the view direction, non-finite camera, ao_samples outside
 * 0..65535, ao_maxdist <= 0, ao_mask requested with ao_samples > 32,
 * aa_samples outside 0..256, specular negative or not finite, shininess not
 * finite and > 0 while specular > 0, or an unknown precision; TR_ENOMEM when the
 * antialiasing workspace cannot be allocated. */
tr_status tr_render(const tr_scene *scene, const tr_camera *cam, const tr_params *params,
                    const tr_frame *frame, void *hip_stream);

/* tr_render with an explicit launch shape (NULL = the tuned or default
 * shape).  TR_EINVAL on an invalid tune field. */
tr_status tr_render_tuned(const tr_scene *scene, const tr_camera *cam, const tr_params *params,
                          const tr_frame *frame, const tr_tune *tune, void *hip_stream);

/* Render n frames in ONE persistent launch whose tile queue spans all n
 * jobs (scenes may differ; job i uses scenes[i], cams[i], params[i],
 * frames[i]).  The FP32 jobs share one launch: they must all use the first
 * FP32 job's precision and its stats buffer (which may be NULL), and that
 * job picks the launch shape.  TR_PREC_FP64 jobs are rendered one launch
 * each.  Every job is checked before anything is enqueued: on an error
 * nothing is rendered.  Each frame equals the same job rendered alone.
 * 1 <= n <= 4096. */
tr_status tr_render_batch(int32_t n, const tr_scene *const *scenes, const tr_camera *cams,
                          const tr_params *params, const tr_frame *frames, void *hip_stream);

/* tr_render_batch for callers that cannot allocate memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same frames as tr_render_batch, bit for bit (same kernels, same rules: one
 * FP32 precision and one stats buffer for the FP32 jobs, the first FP32 job's
 * tuning or `tune` when non-NULL; FP64 jobs are rendered one launch each).
 * The job table and tile queue live in a fixed array of the library's
 * static device memory, about 22 KB per device (TR_NOALLOC_MAX_JOBS job
 * records and the queue's counters), held until the process
 * ends; its address is looked up on the first call on each device.  The
 * call allocates nothing (no hipMalloc, hipFree, host staging or library
 * workspace): the table is written by kernels from their arguments, the
 * counter cleared by a kernel.  Every call on one device shares that array
 * and leaves its contents behind: calls ordered on one stream are safe;
 * calls that overlap on one device (unordered streams) race.
 * TR_EINVAL: n outside 1..TR_NOALLOC_MAX_JOBS, or tr_render_batch's errors;
 * TR_EUNSUPPORTED: aa_samples > 1 (antialiasing needs a workspace).  Every
 * job is checked before anything is enqueued. */
#define TR_NOALLOC_MAX_JOBS 16
tr_status tr_render_batch_noalloc(int32_t n, const tr_scene *const *scenes, const tr_camera *cams,
                                  const tr_params *params, const tr_frame *frames,
                                  const tr_tune *tune, void *hip_stream);

/* Number of 64-pixel tiles of a width x height frame for tile width tile_w
 * (0 = default).  Returns -1 on invalid arguments. */
int64_t tr_tile_count(int32_t width, int32_t height, int32_t tile_w);

/* Batch render restricted to tiles [tile_begin[i], tile_end[i]) of each
 * job (row-major tile order for the given tile width), so a serving loop can
 * advance many frames a bounded step at a time.  Pixels outside the ranges
 * are left untouched.  FP32 precisions only. */
tr_status tr_render_batch_tiles(int32_t n, const tr_scene *const *scenes, const tr_camera *cams,
                                const tr_params *params, const tr_frame *frames,
                                const int64_t *tile_begin, const int64_t *tile_end,
                                const tr_tune *tune, void *hip_stream);

/* Bytes of device memory a frame of this camera needs for the outputs named
 * by frame_flags (bit 0 rgb, bit 1 hit_id, bit 2 ao_mask, bit 3 light_mask);
 * 0 on invalid arguments. */
size_t tr_frame_footprint(const tr_camera *cam, const tr_params *params, uint32_t frame_flags);

/* ---------------------------------------------------------- frame output */

/* 8-bit output of a rendered frame, on the GPU (the "Image I/O" phase of
 * Table 5, whose conversion the paper does not state): out[i] =
 * floor(min(max(values[i], 0), 1) * 255 + 1/2), computed exactly, NaN -> 0.
 * values: n device floats (a frame's rgb is n = 3 * W * H, row-major
 * [H][W][3]); out: n device bytes, same order (an 8-bit RGB image).  Any
 * alignment (16-byte aligned values and 4-byte aligned out take the
 * vectorised path).  Enqueued on the stream; the caller owns both buffers.
 * TR_EINVAL on n < 0 or a NULL pointer with n > 0; n = 0 does nothing. */
tr_status tr_frame_quantize(const float *values, int64_t n, uint8_t *out, void *hip_stream);

/* A Targa (TGA 2.0) file of an 8-bit RGB image, encoded on the GPU (the
 * "Image I/O" phase of Table 5; the paper names no format).  rgb8: device
 * bytes [height][width][3], R G B, row 0 at the top (tr_frame_quantize's
 * output for a frame).  The file: an 18-byte header (image type 10,
 * run-length true colour; 24 bits per pixel; descriptor 0x20, rows stored
 * top first), each row's packets, and the 26-byte TGA 2.0 footer (zero
 * extension and developer offsets, "TRUEVISION-XFILE." and a zero byte).
 * Pixels are stored B G R.  Packets never cross a row: a maximal run of two
 * or more equal pixels becomes run packets (header 0x80 | (count - 1), then
 * the pixel) of 128 pixels and a last one of the rest; a maximal stretch of
 * pixels equal to neither neighbour becomes raw packets (header count - 1,
 * then the pixels) of 128 and a last one of the rest.
 * out: device buffer of capacity bytes (tr_tga_max_bytes is always enough).
 * The call waits for the size pass on the stream and sets *size to the file
 * length; the file itself is written asynchronously on the stream.
 * TR_EINVAL when width or height is outside 1..65535, on a NULL image or
 * size, or when the file needs more than capacity bytes (then *size still
 * holds the length and nothing is written). */
tr_status tr_frame_encode_tga(const uint8_t *rgb8, int32_t width, int32_t height, uint8_t *out,
                              int64_t capacity, int64_t *size, void *hip_stream);

/* Bytes that always hold tr_frame_encode_tga's file of a width x height
 * image (4 per pixel plus header and footer), or -1 when either side is
 * outside 1..65535.  Host only. */
int64_t tr_tga_max_bytes(int32_t width, int32_t height);

/* ------------------------------------------------ graphs (batched views) */

/* A captured, replayable batch render: the tile-counter reset and the
 * persistent launch recorded once into a hipGraph.  Cameras and parameters
 * live in a device job table, so tr_graph_update changes views without
 * re-capturing.  The jobs follow tr_render_batch's rules, and in addition
 * need an FP32 precision, aa_samples <= 1 and max_layers <= 1 (else
 * TR_EUNSUPPORTED).  The tuning (tune may be NULL) is fixed at capture;
 * tune->accel = 1 walks the scenes' BVHs (tr_scene_build_bvh first).
 * The graph reads its scenes' device arrays as they were at creation or at
 * the last tr_graph_update: after tr_scene_rebuild, tr_scene_set_max_skip
 * or tr_scene_build_bvh on one of its scenes, call tr_graph_update before
 * the next launch.  Scenes and frames must outlive the graph. */
typedef struct tr_graph tr_graph;

tr_status tr_graph_create(int32_t n, const tr_scene *const *scenes, const tr_camera *cams,
                          const tr_params *params, const tr_frame *frames, const tr_tune *tune,
                          void *hip_stream, tr_graph **out);
/* Update the n cameras (same resolutions as at creation) and/or params
 * (either may be NULL; both NULL re-reads the scenes only).  The job table
 * upload is enqueued on the stream after every replay already enqueued, on
 * any stream, and every later tr_graph_launch, on any stream, waits for it.
 * TR_EINVAL on a changed resolution or precision or an invalid camera or
 * params (the graph is then unchanged). */
tr_status tr_graph_update(tr_graph *g, const tr_camera *cams, const tr_params *params,
                          void *hip_stream);
/* Replay the graph on the stream (after the latest tr_graph_update). */
tr_status tr_graph_launch(tr_graph *g, void *hip_stream);
/* Waits for the device to finish, then frees the graph.  NULL is a no-op. */
void tr_graph_destroy(tr_graph *g);

/* ----------------------------------------------------------- autotuning */

/* Time the candidate launch shapes on this (scene, camera, params)
 * (coordinate descent over the shape fields, then the winner re-timed against
 * the default shape, interleaved, median of 7 each) and keep the faster in a
 * process-wide cache keyed by (device, primitive-count
 * bucket, resolution, AO samples, precision); later renders with a NULL tune
 * use it.  Checks that every candidate gives a bit-identical frame
 * (TR_EDEVICE with a message if not).  *best (may be NULL) receives the
 * choice; *best_ms (may be NULL) its time.  Synchronises the stream. */
tr_status tr_autotune(const tr_scene *scene, const tr_camera *cam, const tr_params *params,
                      void *hip_stream, tr_tune *best, double *best_ms);

/* Tune a captured graph on itself (all its views, as it replays): the
 * scenes' grid density, which changes speed only (the paper leaves the grid
 * resolution free, Sec. 2), then the launch shape.  Each density in
 * lambdas[0 .. n_lambdas) (cells per primitive, finite and > 0; n_lambdas
 * 0..64) is tried by rebuilding every scene of the graph at it (a density
 * whose grid cannot be built is skipped); the fastest is kept, or the
 * scenes' own densities when none beats them.  Then one pass of coordinate
 * descent over tile width {8, 16, 64}, banks {2, 3}, waves per compute unit
 * {12, 16, 20, 24}, refill threshold {24, 32, 40, 48} and queue stripe {16,
 * 32, 64, 128, 256}, and the winner re-timed against the default shape,
 * interleaved, median of 5 each; the faster is kept.  Every candidate is
 * timed as the median of 3 replays after a warm-up and must leave the first
 * and last frames bit-identical to the starting graph's (else TR_EDEVICE).
 * Afterwards the graph is re-captured with the choice and its scenes are at
 * the chosen density; the frames hold the last replay's images and the stats
 * buffer (if any) has accumulated every replay.  Nothing else may use the
 * graph's scenes meanwhile.  *best (the shape), *best_lambda (0 = the
 * scenes' own densities kept) and *best_ms (its replay time) may be NULL.
 * Synchronises the stream; TR_EINVAL on a NULL graph or a bad density list.
 * On any later error the scenes are rebuilt at their own densities and the
 * graph re-captured with its starting shape before the error is returned. */
tr_status tr_graph_autotune(tr_graph *g, int32_t n_lambdas, const double *lambdas,
                            void *hip_stream, tr_tune *best, double *best_lambda, double *best_ms);

/* Default launch shape for the current device. */
tr_status tr_default_tune(tr_tune *out);

/* ---------------------------------------------------------- measurement */

/* Measured FP32 multiply-add rate of the current device, in TFLOP/s (FMA = 2
 * flops): every lane of 32 waves per compute unit runs 16 independent chains
 * of non-packed FMAs (the form the render kernel issues; packed FP32 is
 * disabled in all of the library's device code), best of 5 timed launches
 * after a warm-up.  Not part of the paper's method: the measured peak that
 * the render kernel's FP32 throughput is reported against, beside the chip's
 * published 157.3 (packed) and 78.6 (non-packed) TFLOP/s.  *clock_mhz (may
 * be NULL) receives the device's reported peak engine clock and *n_cus its
 * compute units (may be NULL).  Synchronises the stream; allocates and frees
 * a small device buffer.  TR_EINVAL on a NULL tflops. */
tr_status tr_measure_fp32_peak(void *hip_stream, double *tflops, double *clock_mhz,
                               int32_t *n_cus);

/* ---------------------------------------------------------------- debug */

/* Philox4x32-10 on the device, for bit-identity checks: out[4i..4i+3] =
 * Philox(ctr[4i..4i+3], key[2i..2i+1]).  Device pointers, n >= 0. */
tr_status tr_debug_philox(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out,
                          void *hip_stream);

/* AO directions as the FP32 kernel draws them: for each i, normal
 * n[3i..3i+2] (unit), pixel pix[i], sample s[i] -> w[3i..3i+2].  Device
 * pointers. */
tr_status tr_debug_ao_dirs(int64_t n, const float *normals, const uint32_t *pix,
                           const uint32_t *sample, uint32_t view_id, uint64_t seed, float *w,
                           void *hip_stream);

/* Thread-local message for the last failing call on this thread. */
const char *tr_last_error(void);
int32_t tr_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TR_H */
