/*
 * FP64 CPU oracle for Cherenkov photon propagation in a RICH-like scene.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the plain, slow reference that the
 * HIP library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * links, imports or calls it.  It shares no code with the HIP library.
 *
 * What it computes (per photon id g, independently):
 *   - a Cherenkov photon on a track: cos(theta) = 1/(n beta), azimuth uniform
 *     (paper, Section 3), wavelength drawn from dN/dlambda ~ 1/lambda^2;
 *   - straight-line propagation to the closest surface (no refraction, the
 *     casing and windows are removed as in Section 4.1);
 *   - specular reflection on mirrors with wavelength-dependent reflectivity
 *     roulette, detection on the photodetector plane with quantum-efficiency
 *     roulette applied at the surface (the improvement proposed in Section 7
 *     over the pre-propagation accept-reject of Section 4.3);
 *   - global hit coordinates and pixel id of photons that reach the detector
 *     (Section 4.4 and the list-of-hits read-out proposed in Section 7).
 * Everything is double precision.  Random numbers come from Philox4x32-10
 * (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the seed, with the photon id
 * in the counter, so any photon can be recomputed alone.
 */
#ifndef RICH_ORACLE_H
#define RICH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_TABLE 32
#define ORC_MAX_PATH_SEGS 4   /* distinct parametrised segments whose Jacobians one path reports */

enum { ORC_DETECTED = 0, ORC_QE_REJECTED = 1, ORC_ABSORBED_MIRROR = 2,
       ORC_ABSORBED = 3, ORC_ESCAPED = 4, ORC_MAX_BOUNCES = 5, ORC_PREFILTERED = 6 };
enum { ORC_MIRROR = 0, ORC_ABSORBER = 1 };
enum { ORC_SRC_TRACK = 0, ORC_SRC_BATCH = 1, ORC_SRC_EXPLICIT = 2 };

typedef struct {
    int32_t n_mat;
    const int32_t *mat_kind;       /* [n_mat] */
    const int32_t *mat_nrefl;      /* [n_mat] */
    const double *mat_refl_x;      /* [n_mat][ORC_MAX_TABLE] */
    const double *mat_refl_y;      /* [n_mat][ORC_MAX_TABLE] */

    int32_t n_seg;
    const double *seg_pivot, *seg_u0, *seg_e1, *seg_e2;   /* [n_seg][3] */
    const double *seg_r0;                                  /* [n_seg] */
    const double *params;                                  /* [n_seg][6] */

    int32_t n_cap;
    const int32_t *cap_seg, *cap_mat;                      /* [n_cap] */
    const double *cap_origin, *cap_a, *cap_b;              /* [n_cap][3] */
    const double *cap_bounds;                              /* [n_cap][4] */

    int32_t n_rect;
    const int32_t *rect_mat;
    const double *rect_c, *rect_n, *rect_u, *rect_v;      /* [n_rect][3] */
    const double *rect_half;                               /* [n_rect][2] */

    int64_t n_tri;
    const double *tri_v;           /* [n_tri][3][3] nominal vertices */
    const int32_t *tri_mat, *tri_seg;

    double det_c[3], det_n[3], det_u[3], det_v[3], det_half[2], det_pitch;
    int32_t det_nx, det_ny, n_qe;
    double qe_x[ORC_MAX_TABLE], qe_y[ORC_MAX_TABLE];

    int32_t has_box;
    double box_lo[3], box_hi[3];

    int32_t max_bounces;
    double t_min;
} orc_scene_desc;

typedef struct {
    int32_t kind;
    /* ORC_SRC_TRACK */
    double origin[3], dir[3], length, beta;
    /* ORC_SRC_BATCH: rows (ox,oy,oz,tx,ty,tz,length,beta) and exclusive scan of counts */
    int64_t n_tracks;
    const double *tracks;          /* [n_tracks][8] */
    const uint64_t *offsets;       /* [n_tracks+1] */
    /* ORC_SRC_EXPLICIT */
    const double *ex_o, *ex_d, *ex_lambda;
    /* common */
    double n_radiator, lambda_min, lambda_max;
    /* pre-propagation filter (Section 4.3): keep with probability QE * prod refl(mats) */
    int32_t prefilter, pf_n, pf_mats[4];
    /* dispersion of the radiator (0 nodes: n = n_radiator for every wavelength):
     * n(lambda) piecewise linear through (disp_x, disp_n), clamped outside */
    int32_t n_disp;
    double disp_x[ORC_MAX_TABLE], disp_n[ORC_MAX_TABLE];
} orc_source;

typedef struct orc_scene orc_scene;

/* Per-photon outputs; any pointer may be NULL.  Arrays are indexed by i = g - first_id. */
typedef struct {
    uint8_t *fate;
    int32_t *pixel;            /* -1 unless DETECTED / QE_REJECTED */
    double *hit_xyz;           /* [n][3], NaN unless DETECTED / QE_REJECTED */
    double *hit_uv;            /* [n][2] */
    double *edge_margin;       /* smallest distance (mm) to a mirror/detector edge or facet edge on the path */
    double *pixel_margin;      /* distance (mm) of the detector hit to the nearest pixel boundary */
    double *roulette_margin;   /* smallest |u - p| over roulette decisions on the path */
    int32_t *n_bounce;         /* surfaces hit */
    int32_t *segment;          /* parametrised segment hit (-1 none, -2 more than one, -3 more than ORC_MAX_PATH_SEGS) */
    double *jac;               /* [n][2][6] d(u,v)/d(segment params), NaN when undefined (also for -2 and -3) */
    double *hit_time;          /* [n] ns from the track origin to the detector hit, NaN unless DETECTED / QE_REJECTED */
    /* Every parametrised segment on the path, in the order first met, and the
     * Jacobian of (u,v) with respect to each one's six parameters, all other
     * segments held fixed; the total derivative of (u,v) is the sum over k of
     * jacs[i][k] applied to segments[i][k]'s parameter change.  Unused slots:
     * segment -1, Jacobian NaN.  Set only for DETECTED / QE_REJECTED. */
    int32_t *segments;         /* [n][ORC_MAX_PATH_SEGS] */
    double *jacs;              /* [n][ORC_MAX_PATH_SEGS][2][6] */
} orc_outputs;

/* Cherenkov photons per mm of track (Frank-Tamm): 2 pi alpha times the
 * integral over [lambda_min, lambda_max] of (1 - 1/(beta n(lambda))^2)^+ / lambda^2,
 * lambda in mm; n from the source's dispersion table or n_radiator. */
int orc_cherenkov_yield(const orc_source *src, double beta, double *photons_per_mm);

/* Film read-out emulation (Section 4.4: camera, film and an intensity
 * threshold instead of recorded hits).  A pinhole camera on the detector
 * normal through its centre, `distance` from it, with a full field of view
 * `fov` across `width` film pixels, maps a detector hit (u, v) to film
 * coordinates x = width/2 + f u / distance, y = height/2 + f v / distance,
 * f = (width/2) / tan(fov/2).  Each DETECTED photon adds
 * 255 exp(-(dx^2 + dy^2) / (2 sigma^2)) to every pixel whose centre
 * (i + 1/2, j + 1/2) lies within 4 sigma in x and in y (dx, dy from the
 * projected point), so a photon centred on a pixel gives that pixel 255.
 * image[j][i] accumulates; hits[j][i] = 1 where min(image, 255) >= threshold. */
typedef struct {
    int32_t width, height;
    double distance, fov, sigma, threshold;
} orc_film;

int orc_film_readout(const orc_film *film, const uint8_t *fate, const double *hit_uv, uint64_t n, double *image,
                     uint8_t *hits);

/* Philox4x32-10: ctr[4], key[2] -> out[4]. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Same with an explicit round count (rounds >= 0), for structural tests. */
void orc_philox4x32_r(const uint32_t ctr[4], const uint32_t key[2], int rounds, uint32_t out[4]);

/* Scene setup: applies the segment parameters, builds the optional BVH. Returns NULL on bad input. */
orc_scene *orc_scene_create(const orc_scene_desc *d, int build_bvh);
void orc_scene_free(orc_scene *s);
const char *orc_last_error(void);

/* Photon generation only: origin, direction and wavelength of photons first_id .. first_id+n-1. */
int orc_generate(const orc_scene *s, const orc_source *src, uint64_t n, uint64_t seed,
                 uint64_t first_id, double *o, double *d, double *lambda);

/* Propagate photons first_id .. first_id+n-1 (batch sources: global ids into the offsets).
 * use_bvh = 0: brute force over every triangle; 1: the oracle's own BVH.
 * with_jacobian = 1 also fills jac and segment. n_threads >= 1. */
int orc_propagate(const orc_scene *s, const orc_source *src, uint64_t n, uint64_t seed,
                  uint64_t first_id, int use_bvh, int with_jacobian, int n_threads,
                  const orc_outputs *out);

/* Same for an arbitrary list of photon ids (not for explicit sources); outputs indexed by list position. */
int orc_propagate_ids(const orc_scene *s, const orc_source *src, const uint64_t *ids, uint64_t n, uint64_t seed,
                      int use_bvh, int with_jacobian, int n_threads, const orc_outputs *out);

/* Closest hit of explicit rays (o, d) over the whole scene: prim index (-1 = none) and t. */
int orc_closest_hit(const orc_scene *s, uint64_t n, const double *o, const double *d,
                    int use_bvh, int64_t *prim, double *t);

/* Index layout of primitives: caps, rects, detector, box, then triangles. */
int64_t orc_prim_base_triangles(const orc_scene *s);

#ifdef __cplusplus
}
#endif
#endif
