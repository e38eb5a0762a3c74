/*
 * rich.h - C ABI of librich.so: Cherenkov optical-photon propagation through a
 * RICH-like detector on AMD MI355X (gfx950).
 *
 * What the calls compute comes from arxiv 2309.12496 ("Optical Photon
 * Simulation with Mitsuba3"):
 *   - photons are emitted on the Cherenkov cone cos(theta) = 1/(n beta),
 *     azimuth-independent (Section 3), or handed over one by one as origin,
 *     direction and wavelength arrays (Section 4.2, the photon emitter);
 *   - they fly straight through a scene reduced to mirrors, absorbing walls
 *     and a detector plane (Section 4.1, windows and casing removed);
 *   - mirror reflectivity and detector quantum efficiency depend on the
 *     wavelength (Section 4.3) and are applied where the photon meets the
 *     surface, the kill-or-propagate treatment proposed in Section 7;
 *   - detected photons are reported as global hit coordinates and pixel ids
 *     (Section 4.4), optionally as a compact list of hits (Section 7).
 * rich_propagate_batch and rich_propagate_adjoint extend the paper: one
 * persistent launch over many tracks, and the reverse-mode derivative of the
 * detector hits with respect to mirror-segment alignment parameters.
 *
 * Units: mm, nm, rad.  Conventions shared by every call:
 *   - Pointers named dev_* are device pointers owned by the caller.  A scene
 *     is owned by the library (rich_build_scene / rich_destroy_scene).
 *   - Every call returns a rich_status.  No C++ exception crosses the ABI.
 *     rich_last_error() returns a thread-local message for the last failure.
 *   - Argument checks are synchronous; the propagation work is enqueued on
 *     the given stream and returns immediately.  Flags raised on the device
 *     (hit-list or traversal-stack overflow, a batch size that is not the
 *     tracks' photon total) are read by rich_get_status.
 *   - NULL output pointers mean "do not write".  The histogram, fate counts
 *     and hit-list counter accumulate: the caller zeroes them.
 *   - Each stream that launches on a scene has its own device workspace
 *     on it (batch work counters, fate-count slots, adjoint partial sums,
 *     forward and batch processing orders, captured batch graph), so
 *     launches on one scene from different streams may run at the same
 *     time.  A stream takes one of the scene's 64 workspace slots at its
 *     first launch and keeps it for the scene's life (a launch from a 65th
 *     stream fails with RICH_ESTATE); the counters and fate-count slots of
 *     every slot are made with the scene, while the calls grow their
 *     stream's buffers with hipMalloc: rich_propagate on a meshed scene (or
 *     with the pre-filter) its photon order, 4 bytes per photon up to 2^24
 *     photons, and the batch and adjoint calls theirs (run a call once on a
 *     stream, at its largest size, before capturing that stream into a
 *     graph; rich_propagate on an analytic scene allocates nothing).  A launch
 *     captured into a graph uses the slot of the stream it was captured on.
 *     Calls on one scene from one stream are ordered.  The scene's host
 *     state is locked: host threads may call on one scene at once (the
 *     calls take turns).  Parameter changes (rich_set_mirror_params,
 *     rich_fit_step) are ordered on their stream only: launches on other
 *     streams see them once the caller orders the streams.
 */
#ifndef RICH_H
#define RICH_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rich_status;
#define RICH_OK         0
#define RICH_EINVAL    -1   /* bad argument: NaN, n*beta <= 1, bad table, bad sizes */
#define RICH_ENOMEM    -2   /* host or device allocation failed */
#define RICH_EDEVICE   -3   /* HIP runtime error */
#define RICH_ERANGE    -4   /* photon id range beyond 2^64 or beyond the batch */
#define RICH_EOVERFLOW -5   /* device flag: hit list or traversal stack overflowed */
#define RICH_ESTATE    -6   /* wrong call order (e.g. no parameters to differentiate) */

/* Photon fates (per-photon output). */
#define RICH_DETECTED        0   /* reached the detector front inside the pixel grid and passed QE */
#define RICH_QE_REJECTED     1   /* reached the pixel grid but failed the QE roulette */
#define RICH_ABSORBED_MIRROR 2   /* failed a mirror reflectivity roulette */
#define RICH_ABSORBED        3   /* absorber, back face, or detector dead border */
#define RICH_ESCAPED         4   /* left the scene without hitting anything */
#define RICH_MAX_BOUNCES     5   /* still flying after max_bounces surfaces */
#define RICH_PREFILTERED     6   /* rejected by the pre-propagation efficiency filter */
#define RICH_N_FATES         7

/* Device status flags returned by rich_get_status. */
#define RICH_FLAG_HITLIST_OVERFLOW 0x1u
#define RICH_FLAG_STACK_OVERFLOW   0x2u
#define RICH_FLAG_PATH_OVERFLOW    0x4u   /* adjoint: more surfaces than it records */
#define RICH_FLAG_BATCH_SIZE       0x8u   /* batch: n_photons differs from offsets[n_tracks] */

#define RICH_MAX_TABLE 32           /* nodes of a piecewise-linear efficiency table */
#define RICH_MAX_SEGMENTS 256       /* parametrised mirror segments */

#define RICH_MAT_MIRROR   0
#define RICH_MAT_ABSORBER 1

/* ---------------------------------------------------------------- scene ---- */

/* Material: mirrors reflect with probability refl(lambda), a piecewise-linear
 * table clamped to its end values (Section 4.3); absorbers end the photon. */
typedef struct rich_material {
    int32_t kind;                 /* RICH_MAT_MIRROR or RICH_MAT_ABSORBER */
    int32_t n_refl;               /* 1..RICH_MAX_TABLE nodes, lambda increasing */
    const double *refl_lambda;    /* host */
    const double *refl_value;     /* host, in [0,1] */
} rich_material;

/* A parametrised mirror segment.  Its 6 parameters p = (tilt_x, tilt_y, R,
 * dx, dy, dz) place a sphere of radius R with centre
 *     C = pivot + (dx,dy,dz) + R * Rot(tilt_x, tilt_y) * u0,
 * Rot = rotation about e2 by tilt_y after rotation about e1 by tilt_x.
 * A meshed segment moves rigidly and scales about its pivot:
 *     v = pivot + (dx,dy,dz) + Rot * (R/radius0) * (v_nominal - pivot). */
typedef struct rich_segment {
    double pivot[3];              /* a point of the nominal sphere */
    double u0[3];                 /* unit vector pivot -> centre at zero tilt */
    double e1[3], e2[3];          /* unit tilt axes, fixed */
    double radius0;               /* nominal radius (scales meshed segments) */
} rich_segment;

/* Analytic spherical cap of a segment: the part of the segment's sphere on the
 * pivot's side of the plane through C normal to Rot*u0, whose coordinates
 * a = (P-origin).axis_a, b = (P-origin).axis_b lie in the half-open cell
 * [bounds[0], bounds[1]) x [bounds[2], bounds[3]).  The active (reflecting)
 * side is the concave one. */
typedef struct rich_cap {
    int32_t segment;              /* 0..n_segments-1 */
    int32_t material;
    double origin[3], axis_a[3], axis_b[3];
    double bounds[4];
} rich_cap;

/* Flat rectangle |u| <= half[0], |v| <= half[1] about center; normal marks the active side. */
typedef struct rich_rect {
    int32_t material;
    int32_t reserved;
    double center[3], normal[3], axis_u[3], axis_v[3];
    double half[2];
} rich_rect;

/* Triangle mesh.  The geometric normal (v1-v0)x(v2-v0) marks the active side.
 * segment = -1: fixed; otherwise the mesh follows that segment's parameters. */
typedef struct rich_mesh {
    const double *vertices;       /* host [n_tri][3][3] */
    int64_t n_tri;
    int32_t material;
    int32_t segment;
} rich_mesh;

/* Photodetector plane: a rectangle |u| <= half[0], |v| <= half[1]; the active
 * side faces along normal.  Pixels of size pitch tile a centred nx*pitch by
 * ny*pitch area; pixel = j*nx + i with i = floor((u + nx*pitch/2)/pitch).
 * Hits outside the pixel grid are ABSORBED.  qe is a piecewise-linear table. */
typedef struct rich_detector {
    double center[3], normal[3], axis_u[3], axis_v[3];
    double half[2];
    double pitch;
    int32_t nx, ny;
    int32_t n_qe;
    const double *qe_lambda;      /* host */
    const double *qe_value;       /* host */
} rich_detector;

typedef struct rich_scene_desc {
    int32_t n_materials;  const rich_material *materials;
    int32_t n_segments;   const rich_segment *segments;
    const double *params;         /* host [n_segments][6] initial parameters, or NULL = (0,0,radius0,0,0,0) */
    int32_t n_caps;       const rich_cap *caps;
    int32_t n_rects;      const rich_rect *rects;
    int32_t n_meshes;     const rich_mesh *meshes;
    rich_detector detector;
    int32_t has_box;              /* 1: absorbing axis-aligned box surface */
    double box_lo[3], box_hi[3];
    int32_t max_bounces;          /* surfaces a photon may meet; 16 by default */
    double t_min;                 /* self-intersection guard, mm (1e-2) */
} rich_scene_desc;

typedef struct rich_scene rich_scene;

/* Scene statistics (rich_scene_info). */
typedef struct rich_scene_stats {
    int64_t n_triangles;
    int64_t n_nodes;              /* BVH4 nodes, all instances plus the top level */
    int32_t n_instances;
    int32_t max_depth;            /* deepest BVH4 path, top level included */
    int64_t device_bytes;
    double build_seconds;         /* host time of rich_build_scene */
} rich_scene_stats;

/* --------------------------------------------------------------- sources ---- */

/* Optional pre-propagation efficiency filter, as the paper's Section 4.3
 * applies it: each photon is kept with probability
 *     QE(lambda) * refl_{materials[0]}(lambda) * ... * refl_{materials[n-1]}(lambda)
 * (one factor per mirror the photons are expected to meet; Section 4.3 uses
 * two), drawn from word 0 of Philox block 0x7FFFFFFF of the photon.  Rejected
 * photons get fate RICH_PREFILTERED and are not traced; kept photons are
 * traced with every efficiency equal to one (no roulette on mirrors or the
 * detector).  enabled = 0 (the default) traces every photon with the
 * efficiencies applied at the surfaces. */
typedef struct rich_prefilter {
    int32_t enabled;
    int32_t n_materials;          /* 0..4 */
    int32_t materials[4];         /* mirror materials whose reflectivity enters the product */
} rich_prefilter;

/* Wavelength dependence of the radiator's refractive index (Section 3: the
 * cone angle is set by n).  n_nodes = 0 (the default) uses the constant
 * n_radiator.  Otherwise n(lambda) is piecewise linear through the host
 * arrays (lambda strictly increasing, n >= 1, 1..32 nodes), clamped outside,
 * and
 *   - wavelengths follow the Frank-Tamm spectrum (1 - 1/(beta n)^2)/lambda^2:
 *     the 1/lambda^2 draw (Philox block 0, word 1) is accepted with
 *     probability w(lambda)/w_max, w = 1 - 1/(beta n)^2 and w_max its largest
 *     value over [lambda_min, lambda_max]; its acceptance uniform is word 0
 *     of block 0x7FFFFFFE; retry k >= 1 draws both from words 1 and 0 of
 *     block 0x7FFFFFFE - k; after 64 rejections the last draw stands;
 *   - the cone follows the photon's own index, cos(theta) = 1/(n(lambda) beta);
 *   - light travels at c/n_g, n_g = n - lambda dn/dlambda (the table
 *     segment's slope, 0 outside the table).
 * Without a table n_g = n_radiator.  The arrays are read during the call
 * only; a table with one index everywhere gives the plain photons. */
typedef struct rich_dispersion {
    int32_t n_nodes;
    int32_t reserved;
    const double *lambda;         /* [n_nodes] nm, host */
    const double *index;          /* [n_nodes] refractive index, host */
} rich_dispersion;

#define RICH_SRC_TRACK    0       /* Cherenkov photons from a straight track segment (length 0: a point) */
#define RICH_SRC_EXPLICIT 2       /* photons given one by one (Section 4.2) */

typedef struct rich_source {
    int32_t kind;
    int32_t reserved;
    /* RICH_SRC_TRACK: photon g is emitted at origin + s*length*dir, s uniform */
    double origin[3], direction[3];
    double length, beta;
    /* RICH_SRC_EXPLICIT: device arrays indexed by g - first_photon_id */
    const float *dev_o;           /* [N][3] */
    const float *dev_d;           /* [N][3] unit */
    const float *dev_lambda;      /* [N] nm */
    /* spectrum and radiator (TRACK) */
    double n_radiator, lambda_min, lambda_max;
    rich_prefilter prefilter;
    rich_dispersion dispersion;   /* TRACK and EXPLICIT (group index for hit_time) */
} rich_source;

/* One track of a batch (32 bytes). */
typedef struct rich_track {
    float origin[3];
    float direction[3];
    float length;
    float beta;
} rich_track;

/* Many tracks in one launch.  Track k owns global photon ids
 * [offsets[k], offsets[k+1]); offsets is the exclusive scan of the counts
 * (non-decreasing; the caller draws the counts, e.g. Poisson of the track
 * length times rich_cherenkov_yield).  The tracks live on the device, so the
 * host does not check them: a track with n beta <= 1 (n_max beta <= 1 with a
 * dispersion table) has no cone, and its photons come out RICH_ESCAPED
 * without being traced. */
typedef struct rich_batch {
    const rich_track *dev_tracks; /* [n_tracks] */
    const uint64_t *dev_offsets;  /* [n_tracks + 1], offsets[0] = 0 */
    int32_t n_tracks;
    int32_t reserved;
    double n_radiator, lambda_min, lambda_max;
    rich_prefilter prefilter;
    rich_dispersion dispersion;
} rich_batch;

/* --------------------------------------------------------------- outputs ---- */

typedef struct rich_hit {
    uint64_t photon;              /* global photon id */
    int32_t pixel;
    float xyz[3];
} rich_hit;

/* Per-photon arrays are indexed by g - first_photon_id (batch: by g). */
typedef struct rich_outputs {
    uint8_t *fate;                /* [N] RICH_DETECTED.. */
    int32_t *pixel;               /* [N] -1 unless DETECTED / QE_REJECTED */
    float *hit_xyz;               /* [N][3] global hit, NaN unless DETECTED / QE_REJECTED */
    float *hit_uv;                /* [N][2] detector coordinates, NaN likewise */
    uint32_t *histogram;          /* [nx*ny] DETECTED photons per pixel, accumulated */
    unsigned long long *fate_counts;  /* [RICH_N_FATES], accumulated */
    rich_hit *hit_list;           /* [capacity] DETECTED photons, in no particular order */
    uint64_t hit_list_capacity;
    unsigned long long *hit_count;    /* [1] accumulated; may exceed capacity (flag raised) */
    float *hit_time;              /* [N] ns: emission s/(beta c) after the track start (0 for explicit
                                     photons) plus path length x n_g / c to the detector hit; NaN
                                     unless DETECTED / QE_REJECTED */
} rich_outputs;

/* Launch shape of the persistent batch kernel. */
typedef struct rich_tuning {
    int32_t block;                /* threads per block: 64, 128, 256 or 512 */
    int32_t chunk;                /* photon ids fetched per wave at a time, multiple of 64 */
    int32_t blocks_per_cu;        /* resident blocks per compute unit in the persistent grid */
    int32_t reserved;
} rich_tuning;

/* ----------------------------------------------------------------- calls ---- */

/* Build a scene on `device` from host FP64 data (paper Section 4.1: the
 * detector reduced to mirrors, absorbing walls and the photodetector plane,
 * meshed surfaces given as triangles): validates, builds SAH BVH4s (one per
 * mesh instance, in that instance's local frame, with facet normals computed
 * in FP64) and a top-level BVH4, and uploads FP32 copies.  Every fixed mesh
 * (segment -1) goes into one instance; each parametrised segment's meshes
 * into one instance of their own.  The desc arrays
 * are read during the call only; the scene owns its device memory until
 * rich_destroy_scene.  Synchronous.  *out is NULL on failure.
 * Errors: RICH_EINVAL for a NULL pointer, a bad table, an unknown material,
 * a non-finite or non-unit frame, an empty cell or rectangle, a segment or
 * material index out of range, 2^26 or more triangles, or a BVH of 2^25 or
 * more nodes, or a device that does not exist; RICH_ENOMEM / RICH_EDEVICE when host or
 * device memory cannot be had. */
rich_status rich_build_scene(const rich_scene_desc *desc, int device, rich_scene **out);

/* Free the scene and everything it holds on the device.  The caller makes
 * sure no launch on the scene is still running.  RICH_EINVAL for NULL. */
rich_status rich_destroy_scene(rich_scene *s);

/* Copy the scene's statistics into *out (host).  RICH_EINVAL for NULL. */
rich_status rich_scene_info(const rich_scene *s, rich_scene_stats *out);

/* Mirror-segment alignment (an extension beyond the paper, which keeps its
 * mirrors fixed): replace the segment parameters from a device array
 * [n_segments][6] (FP32, the caller's, read on the stream) and refresh the
 * derived cap centres, instance transforms and top-level BVH boxes on the
 * stream.  Meshed segments move as instances, so no triangle is rebuilt and
 * no parameter range is refused.  Errors: RICH_EINVAL (NULL pointers),
 * RICH_ESTATE (the scene has no segments), RICH_EDEVICE (launch failed). */
rich_status rich_set_mirror_params(rich_scene *s, const float *dev_params, hipStream_t stream);

/* Propagate photons first_photon_id .. first_photon_id + n_photons - 1 of a
 * single source, seeded by `seed` (Philox4x32-10, counter = photon id):
 * generation on the Cherenkov cone (Section 3) or the given arrays (Section
 * 4.2), straight flight to the closest surface, specular reflection with the
 * reflectivity roulette and the QE roulette at the detector (Section 4.3, at
 * the surface as Section 7 proposes), and the detector hit as global point,
 * (u, v) and pixel (Section 4.4); the compact hit list is Section 7's list of
 * global hits.  Every output array is the caller's device memory, indexed by
 * g - first_photon_id; NULL skips it.  Asynchronous on `stream`.  On meshed
 * scenes and with the pre-filter the photons are traced in an order sorted
 * by cone azimuth within windows of 32,768 ids (8192 with the pre-filter; a
 * sort kernel runs first, into the stream's order buffer), in launches of
 * at most 2^24 photons; results do not depend on the order.
 * Errors (synchronous, nothing launched): RICH_EINVAL for NULL scene or
 * source, an unknown source kind, n beta <= 1, a bad table or prefilter
 * material, a hit list without its counter; RICH_ERANGE when the id range
 * wraps 2^64 or n_photons > 2^40; RICH_ENOMEM when the stream's order buffer
 * cannot grow; RICH_EDEVICE when the launch fails.
 * Traversal-stack and hit-list overflow raise device flags
 * (rich_get_status). */
rich_status rich_propagate(rich_scene *s, const rich_source *src, uint64_t n_photons, uint64_t seed,
                           uint64_t first_photon_id, const rich_outputs *out, hipStream_t stream);

/* The computation of rich_propagate for many tracks in one launch (an
 * extension: the paper instantiates one emitter for all the photons it is
 * handed, Section 4.2).  Propagate every photon of a batch (n_photons =
 * offsets[n_tracks], else the device raises RICH_FLAG_BATCH_SIZE; ids
 * n_photons.. are then left out, or photons beyond the last track's count
 * are drawn from it) in one persistent launch replayed from a captured HIP
 * graph.  Outputs are indexed by the global id g.  Errors as rich_propagate,
 * plus RICH_EINVAL for a bad tuning and RICH_ENOMEM when autotuning or graph
 * capture fails.  tune = NULL picks the
 * launch shape with the autotuner (cached per scene and in the JSON file named
 * by RICH_TUNE_CACHE, if set; tuning synchronises the stream).  The call
 * captures and launches its own graph, so it is not itself meant to be
 * captured into a caller's graph. */
rich_status rich_propagate_batch(rich_scene *s, const rich_batch *batch, uint64_t n_photons, uint64_t seed,
                                 const rich_outputs *out, const rich_tuning *tune, hipStream_t stream);

/* Time the batch kernel over a grid of launch shapes (block 64..512 threads,
 * chunk 64..1024 ids, 1..16 resident blocks per CU as LDS allows) on the
 * first min(n_photons, 4e6) photons, into scratch outputs, and return the
 * fastest (synchronous; allocates and frees its scratch buffers). */
rich_status rich_autotune(rich_scene *s, const rich_batch *batch, uint64_t n_photons, uint64_t seed,
                          rich_tuning *out);

/* Reverse-mode derivative (an extension beyond the paper, which does not
 * differentiate; the DrJit engine its Section 2 builds on is a compiler for
 * differentiable rendering) of detector hit coordinates (u, v) with respect to
 * the segment parameters, at the scene's current parameters, for the photons
 * of either `src` (ids first_photon_id..) or `batch` (ids 0..), exactly one
 * non-NULL.  Interior derivative: visibility changes at edges are ignored.
 * Only photons with dev_mask[i] != 0 (dev_mask NULL: every photon) whose path
 * ends on the pixel grid count.
 *   dev_grad_uv != NULL: dev_grad_params = sum_i J_i^T dev_grad_uv[i];
 *   dev_targets != NULL (fused loss): L = (1/N) sum_i |uv_i - target_i|^2 over
 *     the N counted photons, dev_grad_params = dL/dp, *dev_loss = L.
 *     dev_residual_cut (fused mode only, NULL = no cut) points to one float
 *     on the device, read when the kernel runs: photons whose residual
 *     |uv_i - target_i| exceeds it are not counted (outlier rejection for
 *     fits; a negative or NaN cut leaves every photon out).  Giving it in dev_grad_uv
 *     mode is RICH_EINVAL.
 * dev_grad_params [n_segments][6] is overwritten (zeros, and a zero loss, when
 * no photon counts, n_photons = 0 included).  The sums are deterministic
 * (fixed reduction order).  The first call, and a call with more photons than
 * any before, allocates the scene's partial-sum buffer: a caller that
 * captures this call in a graph makes one such call first.
 * Errors: RICH_EINVAL (both or neither of src/batch or of
 * dev_grad_uv/dev_targets, a cut without targets, NULL dev_grad_params, a
 * batch not starting at id 0), RICH_ESTATE (no segments), RICH_ERANGE (id
 * range), RICH_ENOMEM (partial sums), RICH_EDEVICE (launch).  A path that
 * meets more surfaces than the adjoint records raises
 * RICH_FLAG_PATH_OVERFLOW and is left out. */
rich_status rich_propagate_adjoint(rich_scene *s, const rich_source *src, const rich_batch *batch,
                                   uint64_t n_photons, uint64_t seed, uint64_t first_photon_id,
                                   const float *dev_grad_uv, const float *dev_targets, const uint8_t *dev_mask,
                                   const float *dev_residual_cut, float *dev_grad_params, float *dev_loss,
                                   hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or fitting loops, harnesses that forbid hipMalloc):
 * rich_propagate_adjoint with the same arguments, results and errors, except
 * that its device work buffer lives in a static device array that the
 * library holds on every device it runs on (8 MiB, kept until the process
 * ends) instead of the scene's buffer, so it never calls hipMalloc or hipFree.
 * The work buffer holds B x (6 n_segments + 2) floats of block partial sums
 * per 2^32 photons (B = min(ceil(n / 4096), the blocks the device holds at
 * once)) and, with a mask, 12 bytes per 4096 photons of mask counts, each
 * part rounded up to 256 bytes; a call that needs more than 8 MiB returns
 * RICH_ERANGE before launching anything (on MI355X: up to 256 segments with
 * up to 1.7e9 masked-call photons, or 2^32 without a mask).  Every call on
 * one device shares that device's array: calls that overlap on one device
 * (different streams, or different host threads) race and give wrong sums;
 * order them on one stream.  The array needs no clearing: each launch writes
 * every value it later reads. */
rich_status rich_propagate_adjoint_noalloc(rich_scene *s, const rich_source *src, const rich_batch *batch,
                                           uint64_t n_photons, uint64_t seed, uint64_t first_photon_id,
                                           const float *dev_grad_uv, const float *dev_targets,
                                           const uint8_t *dev_mask, const float *dev_residual_cut,
                                           float *dev_grad_params, float *dev_loss, hipStream_t stream);

/* Optimiser of the alignment fit (extension beyond the paper, built on
 * rich_propagate_adjoint): one Adam step (Kingma and Ba, ICLR 2015) over the
 * segment parameters in normalised coordinates z = (p - p0) / scale, with
 * the step size decaying from lr (step 1) towards lr_final along a cosine:
 *   size_t = lr_final + (lr - lr_final) (1 + cos(pi (t - 1) / n_steps)) / 2,
 *   g = dL/dp * scale (0 in columns not free),
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   z -= size_t (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps),
 *   p = p0 + z * scale,
 * written into the scene (cap centres, instance transforms and top-level
 * boxes refreshed on the stream, as by rich_set_mirror_params). */
typedef struct rich_fit {
    int32_t n_steps;          /* length of the step-size schedule, >= 1 */
    int32_t reserved;
    double lr, lr_final;      /* step sizes in normalised units, >= 0 */
    double beta1, beta2;      /* moment decay rates in [0, 1) */
    double eps;               /* > 0 */
    double scale[6];          /* > 0: column units of z (tx, ty [rad], R, dx, dy, dz [mm]) */
    int32_t free[6];          /* nonzero: the column is fitted */
    double outlier_cut;       /* residual cut after the step: outlier_cut sqrt(loss) + cut_floor (mm) */
    double cut_floor;
} rich_fit;

/* One fit step on `stream`, after the step's rich_propagate_adjoint (fused
 * loss mode) has written dev_grad [n_segments][6] and dev_loss [1]:
 *   dev_p0 [n_segments][6]   parameters at z = 0 (read);
 *   dev_state [3 * 6 * n_segments + 1]   z, m, v, then the number of steps
 *            taken (FP32), zeroed by the caller before the first step and
 *            updated in place;
 *   dev_params [n_segments][6] or NULL   receives the new parameters;
 *   dev_losses [n_steps] or NULL   dev_losses[t - 1] = *dev_loss at step t;
 *   dev_cut [1] or NULL   becomes outlier_cut sqrt(loss) + cut_floor, or
 *            +inf when the loss is 0 (no photon counted), for the next
 *            adjoint's dev_residual_cut.
 * Nothing is allocated and nothing waits for the host, so the adjoint and
 * this call can be captured together in a graph and replayed. */
rich_status rich_fit_step(rich_scene *s, const rich_fit *fit, const float *dev_p0, const float *dev_grad,
                          const float *dev_loss, float *dev_state, float *dev_params, float *dev_losses,
                          float *dev_cut, hipStream_t stream);

/* Film read-out emulation (Section 4.4): the paper detects photons by
 * imaging the detector plane with a pinhole camera onto a film and counting
 * pixels above an intensity threshold (which spreads one photon over several
 * pixels).  The camera sits on the detector normal through its centre,
 * `distance` from it, with a full field of view `fov` across `width` pixels:
 * a hit at detector coordinates (u, v) lands at film coordinates
 *   x = width/2 + f u / distance,  y = height/2 + f v / distance,
 *   f = (width/2) / tan(fov/2).
 * Every DETECTED photon adds 255 exp(-(dx^2 + dy^2) / (2 sigma^2)) to each
 * pixel (i, j) whose centre (i + 1/2, j + 1/2) lies within 4 sigma of (x, y)
 * in x and in y, so one photon centred on a pixel gives it 255. */
typedef struct rich_film {
    int32_t width, height;        /* film pixels; width * height <= 2^31 */
    double distance;              /* mm, > 0 */
    double fov;                   /* rad, 0 < fov < pi */
    double sigma;                 /* reconstruction filter std dev in film pixels, 0 < sigma < 64 */
    double threshold;             /* hit when min(image, 255) >= threshold */
} rich_film;

/* Splat the DETECTED photons among dev_fate[n] / dev_hit_uv[n][2] (as
 * written by the propagate calls) into dev_image[height][width] (FP32,
 * accumulated: the caller zeroes it; atomic additions, so the last bits
 * depend on their order), then, if dev_hits is not NULL, set
 * dev_hits[height][width] to 1 where min(image, 255) >= threshold, else 0.
 * Asynchronous on `stream`, on the current device. */
rich_status rich_film_readout(const rich_film *film, const uint8_t *dev_fate, const float *dev_hit_uv,
                              uint64_t n_photons, float *dev_image, uint8_t *dev_hits, hipStream_t stream);

/* Cherenkov photons emitted per mm of track at velocity beta (Frank-Tamm,
 * the step before the paper's Section 3 cone, which Geant4 supplies there):
 * 2 pi alpha times the integral over [lambda_min, lambda_max] of
 * (1 - 1/(beta n(lambda))^2)^+ / lambda^2, lambda in mm, alpha the fine
 * structure constant; n from `dispersion` (NULL or 0 nodes: n_radiator).
 * The expected photon count of a track of length L is L times this; the
 * caller draws the counts (offsets of a batch).  Host only, synchronous. */
rich_status rich_cherenkov_yield(const rich_dispersion *dispersion, double n_radiator, double beta,
                                 double lambda_min, double lambda_max, double *photons_per_mm);

/* Synchronise the stream, return the device flags raised since the last call
 * (RICH_FLAG_*) in *flags (host; NULL: not returned) and clear them.  Returns
 * RICH_EOVERFLOW when any is set, RICH_EDEVICE when the stream reports an
 * error (a fault of an earlier launch surfaces here). */
rich_status rich_get_status(rich_scene *s, hipStream_t stream, uint32_t *flags);

/* Thread-local description of the last error ("" if none). */
const char *rich_last_error(void);

/* Library version string. */
const char *rich_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RICH_H */
