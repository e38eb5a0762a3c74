/*
 * FP64 CPU oracle for Cherenkov photon propagation (see rich_oracle.h).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It is kept
 * deliberately plain: every photon is traced on its own, every surface is a
 * textbook formula in double precision, and the closest hit is the minimum
 * over all primitives (optionally found through a simple median-split BVH
 * that must return exactly the same primitive as the brute-force scan).
 *
 * Paper anchors:
 *   Section 3    Cherenkov angle cos(theta_c) = 1/(n beta), azimuth-independent.
 *   Section 4.1  geometry reduced to mirrors and a detector plane, no windows:
 *                photons fly straight between surfaces.
 *   Section 4.2  photons enter as explicit (position, direction) arrays.
 *   Section 4.3  wavelength-dependent mirror reflectivity and detector QE.
 *   Section 4.4  hits reported in global coordinates on the detector front face.
 *   Section 7    efficiencies applied at the surface during tracing and hits
 *                written to a list, instead of image read-out.
 */
#include "rich_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Errors                                                                    */
/* ------------------------------------------------------------------------ */

static __thread char g_err[256];

static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }

const char *orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------ */
/* Philox4x32 (Salmon et al., SC'11): a Feistel-like bijection of a 128-bit  */
/* counter under a 64-bit key.  Each round multiplies words 0 and 2 by fixed */
/* odd constants, swaps the halves around and mixes the high product halves */
/* with the key and the other two words; the key gets a Weyl increment      */
/* between rounds.                                                           */
/* ------------------------------------------------------------------------ */

#define PHILOX_M0 0xD2511F53u          /* multipliers published for Philox4x32 */
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u          /* floor(2^32 (golden ratio - 1)) */
#define PHILOX_W1 0xBB67AE85u          /* floor(2^32 (sqrt(3) - 1)) */

#define RICH_STREAM_TAG 0x52494348u    /* fourth counter word: "RICH" */

void orc_philox4x32_r(const uint32_t ctr[4], const uint32_t key[2], int rounds, uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < rounds; ++r) {
        if (r > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    orc_philox4x32_r(ctr, key, 10, out);
}

/* Block `blk` of the random stream of photon g. */
static void photon_block(uint64_t seed, uint64_t g, uint32_t blk, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(g >> 32), blk, RICH_STREAM_TAG};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Uniform on [0,1) from the top 24 bits: exact in binary32 and binary64. */
static double u24(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* ------------------------------------------------------------------------ */
/* Small vector algebra                                                      */
/* ------------------------------------------------------------------------ */

typedef struct { double x, y, z; } v3;

static v3 V(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 vload(const double *p) { return V(p[0], p[1], p[2]); }
static v3 vadd(v3 a, v3 b) { return V(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 vsub(v3 a, v3 b) { return V(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 vmul(v3 a, double s) { return V(a.x * s, a.y * s, a.z * s); }
static double vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 vcross(v3 a, v3 b) { return V(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static double vlen(v3 a) { return sqrt(vdot(a, a)); }
static v3 vunit(v3 a) { return vmul(a, 1.0 / vlen(a)); }
static double vget(v3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

/* Rotation of v by angle th about unit axis k (Rodrigues' formula). */
static v3 rodrigues(v3 k, double th, v3 v)
{
    double c = cos(th), s = sin(th);
    return vadd(vadd(vmul(v, c), vmul(vcross(k, v), s)), vmul(k, vdot(k, v) * (1.0 - c)));
}

/* Segment rotation: first about e1 by tilt_x, then about e2 by tilt_y. */
static v3 seg_rot(v3 e1, v3 e2, double tx, double ty, v3 v)
{
    return rodrigues(e2, ty, rodrigues(e1, tx, v));
}

/* Piecewise-linear table, clamped to the end values outside its range. */
static double table(int n, const double *x, const double *y, double l)
{
    if (l <= x[0]) return y[0];
    if (l >= x[n - 1]) return y[n - 1];
    int i = 0;
    while (i + 1 < n - 1 && l >= x[i + 1]) ++i;
    return y[i] + (y[i + 1] - y[i]) * (l - x[i]) / (x[i + 1] - x[i]);
}

/* ------------------------------------------------------------------------ */
/* Scene                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    double lo[3], hi[3];
    int64_t left, right;     /* children, or -1 for a leaf */
    int64_t first, count;    /* leaf range in bvh_idx */
} bnode;

struct orc_scene {
    orc_scene_desc d;        /* scalar fields; array pointers are replaced by copies below */
    /* materials */
    int32_t *mat_kind, *mat_nrefl;
    double *mat_refl_x, *mat_refl_y;
    /* segments */
    double *seg_pivot, *seg_u0, *seg_e1, *seg_e2, *seg_r0, *params;
    /* caps with the current sphere centre, radius and axis */
    int32_t *cap_seg, *cap_mat;
    double *cap_origin, *cap_a, *cap_b, *cap_bounds;
    double *cap_C, *cap_R, *cap_axis;
    /* rects */
    int32_t *rect_mat;
    double *rect_c, *rect_n, *rect_u, *rect_v, *rect_half;
    /* triangles at the current parameters: vertices and unit normal */
    double *tri_v0;          /* nominal vertices (for Jacobians of moving meshes) */
    double *tri;             /* [n][9] */
    double *tri_nrm;         /* [n][3] */
    int32_t *tri_mat, *tri_seg;
    /* BVH */
    bnode *nodes;
    int64_t n_nodes;
    int64_t *bvh_idx;
};

static void *dup(const void *p, size_t bytes)
{
    if (bytes == 0) return calloc(1, 1);
    void *q = malloc(bytes);
    if (q && p) memcpy(q, p, bytes);
    return q;
}

int64_t orc_prim_base_triangles(const orc_scene *s) { return (int64_t)s->d.n_cap + s->d.n_rect + 2; }

static void apply_params(orc_scene *s)
{
    for (int i = 0; i < s->d.n_cap; ++i) {
        int k = s->cap_seg[i];
        const double *p = s->params + 6 * k;
        v3 ax = seg_rot(vload(s->seg_e1 + 3 * k), vload(s->seg_e2 + 3 * k), p[0], p[1], vload(s->seg_u0 + 3 * k));
        v3 C = vadd(vadd(vload(s->seg_pivot + 3 * k), V(p[3], p[4], p[5])), vmul(ax, p[2]));
        s->cap_C[3 * i] = C.x; s->cap_C[3 * i + 1] = C.y; s->cap_C[3 * i + 2] = C.z;
        s->cap_axis[3 * i] = ax.x; s->cap_axis[3 * i + 1] = ax.y; s->cap_axis[3 * i + 2] = ax.z;
        s->cap_R[i] = p[2];
    }
    for (int64_t j = 0; j < s->d.n_tri; ++j) {
        int k = s->tri_seg[j];
        v3 w[3];
        for (int m = 0; m < 3; ++m) {
            v3 v0 = vload(s->tri_v0 + 9 * j + 3 * m);
            if (k >= 0) {
                const double *p = s->params + 6 * k;
                v3 piv = vload(s->seg_pivot + 3 * k);
                double sc = p[2] / s->seg_r0[k];
                v3 r = seg_rot(vload(s->seg_e1 + 3 * k), vload(s->seg_e2 + 3 * k), p[0], p[1], vmul(vsub(v0, piv), sc));
                w[m] = vadd(vadd(piv, V(p[3], p[4], p[5])), r);
            } else {
                w[m] = v0;
            }
            s->tri[9 * j + 3 * m] = w[m].x;
            s->tri[9 * j + 3 * m + 1] = w[m].y;
            s->tri[9 * j + 3 * m + 2] = w[m].z;
        }
        v3 n = vunit(vcross(vsub(w[1], w[0]), vsub(w[2], w[0])));
        s->tri_nrm[3 * j] = n.x; s->tri_nrm[3 * j + 1] = n.y; s->tri_nrm[3 * j + 2] = n.z;
    }
}

/* --- oracle BVH: binary, split at the median centroid of the longest axis --- */

typedef struct { const double *cen; int axis; } sel_ctx;

static int key_less(const double *cen, int axis, int64_t a, int64_t b)
{
    double ka = cen[3 * a + axis], kb = cen[3 * b + axis];
    return ka < kb || (ka == kb && a < b);
}

/* Reorder idx[lo..hi) so that position m holds the m-th smallest key (quickselect). */
static void select_nth(int64_t *idx, int64_t lo, int64_t hi, int64_t m, const double *cen, int axis)
{
    while (hi - lo > 1) {
        int64_t pv = idx[lo + (hi - lo) / 2];
        int64_t i = lo, j = hi - 1;
        while (i <= j) {
            while (key_less(cen, axis, idx[i], pv)) ++i;
            while (key_less(cen, axis, pv, idx[j])) --j;
            if (i <= j) {
                int64_t t = idx[i]; idx[i] = idx[j]; idx[j] = t;
                ++i; --j;
            }
        }
        if (m <= j) hi = j + 1;
        else if (m >= i) lo = i;
        else return;
    }
}

static int64_t build_node(orc_scene *s, const double *cen, int64_t first, int64_t count)
{
    int64_t me = s->n_nodes++;
    bnode *nd = &s->nodes[me];
    for (int a = 0; a < 3; ++a) { nd->lo[a] = INFINITY; nd->hi[a] = -INFINITY; }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t q = first; q < first + count; ++q) {
        int64_t j = s->bvh_idx[q];
        for (int m = 0; m < 3; ++m)
            for (int a = 0; a < 3; ++a) {
                double x = s->tri[9 * j + 3 * m + a];
                if (x < nd->lo[a]) nd->lo[a] = x;
                if (x > nd->hi[a]) nd->hi[a] = x;
            }
        for (int a = 0; a < 3; ++a) {
            double c = cen[3 * j + a];
            if (c < clo[a]) clo[a] = c;
            if (c > chi[a]) chi[a] = c;
        }
    }
    for (int a = 0; a < 3; ++a) {      /* pad so that box tests never cut a triangle */
        double pad = 1e-6 + 1e-12 * (fabs(nd->lo[a]) + fabs(nd->hi[a]));
        nd->lo[a] -= pad;
        nd->hi[a] += pad;
    }
    if (count <= 4) {
        nd->left = nd->right = -1;
        nd->first = first;
        nd->count = count;
        return me;
    }
    int axis = 0;
    for (int a = 1; a < 3; ++a)
        if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    int64_t half = count / 2;
    select_nth(s->bvh_idx, first, first + count, first + half, cen, axis);
    nd->first = first;
    nd->count = 0;
    int64_t l = build_node(s, cen, first, half);
    int64_t r = build_node(s, cen, first + half, count - half);
    s->nodes[me].left = l;
    s->nodes[me].right = r;
    return me;
}

static int build_bvh(orc_scene *s)
{
    int64_t n = s->d.n_tri;
    if (n == 0) return 1;
    double *cen = malloc(sizeof(double) * 3 * n);
    s->bvh_idx = malloc(sizeof(int64_t) * n);
    s->nodes = malloc(sizeof(bnode) * (2 * n + 1));
    if (!cen || !s->bvh_idx || !s->nodes) { free(cen); return 0; }
    for (int64_t j = 0; j < n; ++j) {
        s->bvh_idx[j] = j;
        for (int a = 0; a < 3; ++a)
            cen[3 * j + a] = (s->tri[9 * j + a] + s->tri[9 * j + 3 + a] + s->tri[9 * j + 6 + a]) / 3.0;
    }
    s->n_nodes = 0;
    build_node(s, cen, 0, n);
    free(cen);
    return 1;
}

static int finite_arr(const double *p, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(p[i])) return 0;
    return 1;
}

orc_scene *orc_scene_create(const orc_scene_desc *d, int build)
{
    if (!d) { set_err("null scene description"); return NULL; }
    if (d->n_qe < 1 || d->n_qe > ORC_MAX_TABLE || d->det_nx <= 0 || d->det_ny <= 0 || !(d->det_pitch > 0)) {
        set_err("bad detector description");
        return NULL;
    }
    for (int i = 0; i < d->n_mat; ++i)
        if (d->mat_nrefl[i] < 1 || d->mat_nrefl[i] > ORC_MAX_TABLE) { set_err("bad reflectivity table"); return NULL; }
    if (!finite_arr(d->tri_v, 9 * d->n_tri)) { set_err("non-finite vertex"); return NULL; }
    for (int i = 0; i < d->n_cap; ++i)
        if (d->cap_seg[i] < 0 || d->cap_seg[i] >= d->n_seg) { set_err("cap without a segment"); return NULL; }
    for (int64_t j = 0; j < d->n_tri; ++j)
        if (d->tri_seg[j] >= d->n_seg) { set_err("triangle segment out of range"); return NULL; }

    orc_scene *s = calloc(1, sizeof *s);
    if (!s) { set_err("out of memory"); return NULL; }
    s->d = *d;
    int nm = d->n_mat, ns = d->n_seg, nc = d->n_cap, nr = d->n_rect;
    int64_t nt = d->n_tri;
    s->mat_kind = dup(d->mat_kind, sizeof(int32_t) * nm);
    s->mat_nrefl = dup(d->mat_nrefl, sizeof(int32_t) * nm);
    s->mat_refl_x = dup(d->mat_refl_x, sizeof(double) * nm * ORC_MAX_TABLE);
    s->mat_refl_y = dup(d->mat_refl_y, sizeof(double) * nm * ORC_MAX_TABLE);
    s->seg_pivot = dup(d->seg_pivot, sizeof(double) * 3 * ns);
    s->seg_u0 = dup(d->seg_u0, sizeof(double) * 3 * ns);
    s->seg_e1 = dup(d->seg_e1, sizeof(double) * 3 * ns);
    s->seg_e2 = dup(d->seg_e2, sizeof(double) * 3 * ns);
    s->seg_r0 = dup(d->seg_r0, sizeof(double) * ns);
    s->params = dup(d->params, sizeof(double) * 6 * ns);
    s->cap_seg = dup(d->cap_seg, sizeof(int32_t) * nc);
    s->cap_mat = dup(d->cap_mat, sizeof(int32_t) * nc);
    s->cap_origin = dup(d->cap_origin, sizeof(double) * 3 * nc);
    s->cap_a = dup(d->cap_a, sizeof(double) * 3 * nc);
    s->cap_b = dup(d->cap_b, sizeof(double) * 3 * nc);
    s->cap_bounds = dup(d->cap_bounds, sizeof(double) * 4 * nc);
    s->cap_C = dup(NULL, sizeof(double) * 3 * nc);
    s->cap_R = dup(NULL, sizeof(double) * nc);
    s->cap_axis = dup(NULL, sizeof(double) * 3 * nc);
    s->rect_mat = dup(d->rect_mat, sizeof(int32_t) * nr);
    s->rect_c = dup(d->rect_c, sizeof(double) * 3 * nr);
    s->rect_n = dup(d->rect_n, sizeof(double) * 3 * nr);
    s->rect_u = dup(d->rect_u, sizeof(double) * 3 * nr);
    s->rect_v = dup(d->rect_v, sizeof(double) * 3 * nr);
    s->rect_half = dup(d->rect_half, sizeof(double) * 2 * nr);
    s->tri_v0 = dup(d->tri_v, sizeof(double) * 9 * nt);
    s->tri = dup(NULL, sizeof(double) * 9 * nt);
    s->tri_nrm = dup(NULL, sizeof(double) * 3 * nt);
    s->tri_mat = dup(d->tri_mat, sizeof(int32_t) * nt);
    s->tri_seg = dup(d->tri_seg, sizeof(int32_t) * nt);
    if (!s->tri || !s->tri_v0 || !s->tri_nrm) { orc_scene_free(s); set_err("out of memory"); return NULL; }
    apply_params(s);
    if (build && !build_bvh(s)) { orc_scene_free(s); set_err("out of memory (bvh)"); return NULL; }
    return s;
}

void orc_scene_free(orc_scene *s)
{
    if (!s) return;
    void *ptrs[] = {s->mat_kind, s->mat_nrefl, s->mat_refl_x, s->mat_refl_y, s->seg_pivot, s->seg_u0,
                    s->seg_e1, s->seg_e2, s->seg_r0, s->params, s->cap_seg, s->cap_mat, s->cap_origin,
                    s->cap_a, s->cap_b, s->cap_bounds, s->cap_C, s->cap_R, s->cap_axis, s->rect_mat,
                    s->rect_c, s->rect_n, s->rect_u, s->rect_v, s->rect_half, s->tri_v0, s->tri,
                    s->tri_nrm, s->tri_mat, s->tri_seg, s->nodes, s->bvh_idx};
    for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; ++i) free(ptrs[i]);
    free(s);
}

/* ------------------------------------------------------------------------ */
/* Intersections (all double precision, textbook forms)                      */
/* ------------------------------------------------------------------------ */

/* Spherical cap: the sphere |P - C| = R restricted to the pivot's hemisphere,
 * (P - C).axis < 0, and to the half-open aperture cell of the fixed frame.
 * Roots of t^2 + 2 (f.d) t + |f|^2 - R^2 = 0 with f = o - C; the smaller root
 * beyond t_min that lies on the cap wins. */
static int hit_cap(const orc_scene *s, int i, v3 o, v3 d, double tmin, double *t_out, int *root_out)
{
    v3 C = vload(s->cap_C + 3 * i), ax = vload(s->cap_axis + 3 * i);
    double R = s->cap_R[i];
    v3 f = vsub(o, C);
    double b = vdot(f, d), c = vdot(f, f) - R * R;
    double disc = b * b - c;
    if (disc < 0) return 0;
    double sq = sqrt(disc);
    double ts[2] = {-b - sq, -b + sq};
    const double *bd = s->cap_bounds + 4 * i;
    v3 O = vload(s->cap_origin + 3 * i), A = vload(s->cap_a + 3 * i), B = vload(s->cap_b + 3 * i);
    for (int r = 0; r < 2; ++r) {
        double t = ts[r];
        if (!(t > tmin)) continue;
        v3 P = vadd(o, vmul(d, t));
        if (vdot(vsub(P, C), ax) >= 0) continue;
        double a = vdot(vsub(P, O), A), bb = vdot(vsub(P, O), B);
        if (a >= bd[0] && a < bd[1] && bb >= bd[2] && bb < bd[3]) {
            *t_out = t;
            *root_out = r;
            return 1;
        }
    }
    return 0;
}

/* Plane rectangle |u| <= hu, |v| <= hv around c. */
static int hit_rect(v3 c, v3 n, v3 U, v3 W, double hu, double hv, v3 o, v3 d, double tmin, double *t_out)
{
    double dn = vdot(d, n);
    if (dn == 0) return 0;
    double t = vdot(vsub(c, o), n) / dn;
    if (!(t > tmin)) return 0;
    v3 P = vadd(o, vmul(d, t));
    double u = vdot(vsub(P, c), U), v = vdot(vsub(P, c), W);
    if (fabs(u) <= hu && fabs(v) <= hv) { *t_out = t; return 1; }
    return 0;
}

/* Axis-aligned box surface: entry or exit point, whichever is first beyond tmin. */
static int hit_box(const double *lo, const double *hi, v3 o, v3 d, double tmin, double *t_out)
{
    double tn = -INFINITY, tf = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double oa = vget(o, a), da = vget(d, a);
        if (da == 0) {
            if (oa < lo[a] || oa > hi[a]) return 0;
            continue;
        }
        double t1 = (lo[a] - oa) / da, t2 = (hi[a] - oa) / da;
        double tlo = t1 < t2 ? t1 : t2, thi = t1 < t2 ? t2 : t1;
        if (tlo > tn) tn = tlo;
        if (thi < tf) tf = thi;
    }
    if (tn > tf) return 0;
    if (tn > tmin) { *t_out = tn; return 1; }
    if (tf > tmin) { *t_out = tf; return 1; }
    return 0;
}

/* Moller-Trumbore ray/triangle test from either side.  The barycentric range is
 * closed and widened by BARY_EPS so that a ray through a shared edge or vertex
 * of a closed mesh hits at least one of the triangles despite rounding (the
 * overlap is ~1e-8 mm on the meshes used here). */
#define BARY_EPS 1e-10
static int hit_tri(const double *w, v3 o, v3 d, double tmin, double *t_out)
{
    v3 v0 = vload(w), v1 = vload(w + 3), v2 = vload(w + 6);
    v3 e1 = vsub(v1, v0), e2 = vsub(v2, v0);
    v3 p = vcross(d, e2);
    double det = vdot(e1, p);
    if (det == 0) return 0;
    double inv = 1.0 / det;
    v3 sv = vsub(o, v0);
    double u = vdot(sv, p) * inv;
    if (u < -BARY_EPS || u > 1 + BARY_EPS) return 0;
    v3 q = vcross(sv, e1);
    double v = vdot(d, q) * inv;
    if (v < -BARY_EPS || u + v > 1 + BARY_EPS) return 0;
    double t = vdot(e2, q) * inv;
    if (!(t > tmin)) return 0;
    *t_out = t;
    return 1;
}

typedef struct { double t; int64_t prim; int root; } hitrec;

static void offer_tri(const orc_scene *s, int64_t j, v3 o, v3 d, hitrec *h, int64_t base)
{
    double t;
    if (!hit_tri(s->tri + 9 * j, o, d, s->d.t_min, &t)) return;
    int64_t id = base + j;
    if (t < h->t || (t == h->t && id < h->prim)) { h->t = t; h->prim = id; h->root = 0; }
}

/* Slab test against a node box; returns 1 and the entry distance when the ray can reach it. */
static int node_entry(const bnode *nd, v3 o, v3 d, double tmax, double *t_entry)
{
    double tn = -INFINITY, tf = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double oa = vget(o, a), da = vget(d, a);
        if (da == 0) {
            if (oa < nd->lo[a] || oa > nd->hi[a]) return 0;
            continue;
        }
        double t1 = (nd->lo[a] - oa) / da, t2 = (nd->hi[a] - oa) / da;
        double tlo = t1 < t2 ? t1 : t2, thi = t1 < t2 ? t2 : t1;
        if (tlo > tn) tn = tlo;
        if (thi < tf) tf = thi;
    }
    if (tn > tf || tf < 0 || tn > tmax) return 0;
    *t_entry = tn;
    return 1;
}

static void closest_hit(const orc_scene *s, v3 o, v3 d, int use_bvh, hitrec *h)
{
    const double tmin = s->d.t_min;
    h->t = INFINITY;
    h->prim = -1;
    h->root = 0;
    double t;
    int root;
    int64_t id = 0;
    for (int i = 0; i < s->d.n_cap; ++i, ++id)
        if (hit_cap(s, i, o, d, tmin, &t, &root) && t < h->t) { h->t = t; h->prim = id; h->root = root; }
    for (int i = 0; i < s->d.n_rect; ++i, ++id)
        if (hit_rect(vload(s->rect_c + 3 * i), vload(s->rect_n + 3 * i), vload(s->rect_u + 3 * i),
                     vload(s->rect_v + 3 * i), s->rect_half[2 * i], s->rect_half[2 * i + 1], o, d, tmin, &t) &&
            t < h->t) { h->t = t; h->prim = id; h->root = 0; }
    if (hit_rect(vload(s->d.det_c), vload(s->d.det_n), vload(s->d.det_u), vload(s->d.det_v),
                 s->d.det_half[0], s->d.det_half[1], o, d, tmin, &t) && t < h->t) {
        h->t = t; h->prim = id; h->root = 0;
    }
    ++id;
    if (s->d.has_box && hit_box(s->d.box_lo, s->d.box_hi, o, d, tmin, &t) && t < h->t) {
        h->t = t; h->prim = id; h->root = 0;
    }
    ++id;
    int64_t base = id;
    if (s->d.n_tri == 0) return;
    if (!use_bvh || !s->nodes) {
        for (int64_t j = 0; j < s->d.n_tri; ++j) offer_tri(s, j, o, d, h, base);
        return;
    }
    int64_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const bnode *nd = &s->nodes[stack[--sp]];
        double te;
        if (!node_entry(nd, o, d, h->t, &te)) continue;
        if (nd->left < 0) {
            for (int64_t q = nd->first; q < nd->first + nd->count; ++q) offer_tri(s, s->bvh_idx[q], o, d, h, base);
        } else {
            stack[sp++] = nd->right;
            stack[sp++] = nd->left;
        }
    }
}

int orc_closest_hit(const orc_scene *s, uint64_t n, const double *o, const double *d, int use_bvh,
                    int64_t *prim, double *t)
{
    for (uint64_t i = 0; i < n; ++i) {
        hitrec h;
        closest_hit(s, vload(o + 3 * i), vload(d + 3 * i), use_bvh, &h);
        prim[i] = h.prim;
        t[i] = h.prim >= 0 ? h.t : INFINITY;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Photon generation                                                         */
/* ------------------------------------------------------------------------ */

/* Orthonormal basis around unit n (Duff, Burgess, Christensen, Hery, Kensler,
 * Liani, Villemin, "Building an Orthonormal Basis, Revisited", JCGT 2017). */
static void onb(v3 n, v3 *b1, v3 *b2)
{
    double sign = copysign(1.0, n.z);
    double a = -1.0 / (sign + n.z);
    double b = n.x * n.y * a;
    *b1 = V(1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x);
    *b2 = V(b, sign + n.y * n.y * a, -n.y);
}

/* t0: emission time (ns after the track origin passes P0); ng: group index
 * of the radiator at the photon's wavelength; margin: smallest |u - p| over
 * the wavelength accept-reject decisions. */
typedef struct { v3 o, d; double lambda; double u_qe; double t0, ng, margin; } photon;

#define C_MM_PER_NS 299.792458            /* speed of light in vacuum */
#define FINE_STRUCTURE (1.0 / 137.035999084)
#define DISP_BLOCK 0x7FFFFFFEu            /* Philox blocks of the wavelength retries count down from here */
#define DISP_MAX_TRIES 64

/* Refractive index of the radiator at lambda (Section 3: the cone angle
 * follows n); piecewise linear through the dispersion table, clamped. */
static double index_at(const orc_source *src, double lambda)
{
    return src->n_disp > 0 ? table(src->n_disp, src->disp_x, src->disp_n, lambda) : src->n_radiator;
}

/* Group index n - lambda dn/dlambda: the speed c/n_g at which the photon's
 * light travels.  dn/dlambda is the table segment's slope (0 outside). */
static double group_index_at(const orc_source *src, double lambda)
{
    if (src->n_disp < 2) return index_at(src, lambda);
    const double *x = src->disp_x, *y = src->disp_n;
    int n = src->n_disp;
    if (lambda < x[0] || lambda >= x[n - 1]) return index_at(src, lambda);
    int i = 0;
    while (i + 1 < n - 1 && lambda >= x[i + 1]) ++i;
    double slope = (y[i + 1] - y[i]) / (x[i + 1] - x[i]);
    return index_at(src, lambda) - lambda * slope;
}

/* Frank-Tamm spectral weight 1 - 1/(beta n)^2, zero below threshold. */
static double ft_weight(double n, double beta)
{
    double w = 1.0 - 1.0 / (beta * beta * n * n);
    return w > 0.0 ? w : 0.0;
}

/* Largest refractive index over [lambda_min, lambda_max] (at a table node or an end). */
static double max_index(const orc_source *src)
{
    double m = fmax(index_at(src, src->lambda_min), index_at(src, src->lambda_max));
    for (int k = 0; k < src->n_disp; ++k)
        if (src->disp_x[k] > src->lambda_min && src->disp_x[k] < src->lambda_max) m = fmax(m, src->disp_n[k]);
    return m;
}

#define PREFILTER_BLOCK 0x7FFFFFFFu

/* Section 4.3: one accept-reject per photon with probability
 * QE(lambda) * product of the listed mirrors' reflectivities. */
static int prefilter_keep(const orc_scene *s, const orc_source *src, uint64_t seed, uint64_t g, double lambda,
                          double *margin)
{
    double p = table(s->d.n_qe, s->d.qe_x, s->d.qe_y, lambda);
    for (int k = 0; k < src->pf_n; ++k) {
        int m = src->pf_mats[k];
        p *= table(s->mat_nrefl[m], s->mat_refl_x + ORC_MAX_TABLE * m, s->mat_refl_y + ORC_MAX_TABLE * m, lambda);
    }
    uint32_t w[4];
    photon_block(seed, g, PREFILTER_BLOCK, w);
    double u = u24(w[0]);
    *margin = fabs(u - p);
    return u < p;
}

static int find_track(const orc_source *src, uint64_t g)
{
    /* last k with offsets[k] <= g */
    int64_t lo = 0, hi = src->n_tracks;   /* answer in [lo, hi) */
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (src->offsets[mid] <= g) lo = mid; else hi = mid;
    }
    return (int)lo;
}

static void make_photon(const orc_source *src, uint64_t seed, uint64_t g, uint64_t i, photon *ph)
{
    uint32_t w[4];
    photon_block(seed, g, 0, w);
    double u_phi = u24(w[0]), u_lam = u24(w[1]), u_s = u24(w[2]);
    ph->u_qe = u24(w[3]);
    if (src->kind == ORC_SRC_EXPLICIT) {
        ph->o = vload(src->ex_o + 3 * i);
        ph->d = vload(src->ex_d + 3 * i);
        ph->lambda = src->ex_lambda[i];
        ph->t0 = 0.0;
        ph->ng = group_index_at(src, ph->lambda);
        ph->margin = INFINITY;
        return;
    }
    v3 P0, T;
    double L, beta;
    if (src->kind == ORC_SRC_BATCH) {
        const double *r = src->tracks + 8 * find_track(src, g);
        P0 = vload(r);
        T = vload(r + 3);
        L = r[6];
        beta = r[7];
    } else {
        P0 = vload(src->origin);
        T = vload(src->dir);
        L = src->length;
        beta = src->beta;
    }
    T = vunit(T);
    /* wavelength: inverse CDF of dN/dlambda ~ 1/lambda^2 on [lambda_min, lambda_max] */
    double a = 1.0 / src->lambda_min, b = 1.0 / src->lambda_max;
    ph->lambda = 1.0 / (a - u_lam * (a - b));
    ph->margin = INFINITY;
    if (src->n_disp > 0) {
        /* With dispersion the Frank-Tamm spectrum is (1 - 1/(beta n)^2)/lambda^2:
         * accept the 1/lambda^2 draw with probability w(lambda)/w_max, else draw
         * again.  Attempt 0 keeps the draw above (its acceptance uniform is word
         * 0 of block DISP_BLOCK); attempt k >= 1 takes words 1 (wavelength) and
         * 0 (acceptance) of block DISP_BLOCK - k.  After DISP_MAX_TRIES
         * rejections the last draw stands. */
        double wmax = ft_weight(max_index(src), beta);
        for (int k = 0; k < DISP_MAX_TRIES; ++k) {
            uint32_t wb[4];
            photon_block(seed, g, DISP_BLOCK - (uint32_t)k, wb);
            if (k > 0) ph->lambda = 1.0 / (a - u24(wb[1]) * (a - b));
            double p = ft_weight(index_at(src, ph->lambda), beta) / wmax;
            double u = u24(wb[0]);
            ph->margin = fmin(ph->margin, fabs(u - p));
            if (u < p) break;
        }
    }
    /* Cherenkov cone (Section 3) at the photon's own refractive index */
    double ct = 1.0 / (index_at(src, ph->lambda) * beta);
    double st = sqrt(1.0 - ct * ct);
    double phi = 2.0 * M_PI * u_phi;
    v3 e1, e2;
    onb(T, &e1, &e2);
    ph->d = vadd(vmul(T, ct), vmul(vadd(vmul(e1, cos(phi)), vmul(e2, sin(phi))), st));
    ph->o = vadd(P0, vmul(T, u_s * L));
    /* the track moves at beta c from P0 */
    ph->t0 = u_s * L / (beta * C_MM_PER_NS);
    ph->ng = group_index_at(src, ph->lambda);
}

int orc_generate(const orc_scene *s, const orc_source *src, uint64_t n, uint64_t seed, uint64_t first_id,
                 double *o, double *d, double *lambda)
{
    (void)s;
    for (uint64_t i = 0; i < n; ++i) {
        photon ph;
        make_photon(src, seed, first_id + i, i, &ph);
        if (o) { o[3 * i] = ph.o.x; o[3 * i + 1] = ph.o.y; o[3 * i + 2] = ph.o.z; }
        if (d) { d[3 * i] = ph.d.x; d[3 * i + 1] = ph.d.y; d[3 * i + 2] = ph.d.z; }
        if (lambda) lambda[i] = ph.lambda;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Forward-mode duals for the Jacobian of (u,v) w.r.t. one segment's params   */
/* ------------------------------------------------------------------------ */

#define NT 6
typedef struct { double v, g[NT]; } dn;
typedef struct { dn x, y, z; } dv;

static dn dc(double v) { dn r; r.v = v; memset(r.g, 0, sizeof r.g); return r; }
static dn dvar(double v, int k) { dn r = dc(v); r.g[k] = 1.0; return r; }
static dn dadd(dn a, dn b) { dn r; r.v = a.v + b.v; for (int k = 0; k < NT; ++k) r.g[k] = a.g[k] + b.g[k]; return r; }
static dn dsub(dn a, dn b) { dn r; r.v = a.v - b.v; for (int k = 0; k < NT; ++k) r.g[k] = a.g[k] - b.g[k]; return r; }
static dn dmul(dn a, dn b) { dn r; r.v = a.v * b.v; for (int k = 0; k < NT; ++k) r.g[k] = a.g[k] * b.v + a.v * b.g[k]; return r; }
static dn ddiv(dn a, dn b)
{
    dn r;
    r.v = a.v / b.v;
    for (int k = 0; k < NT; ++k) r.g[k] = (a.g[k] * b.v - a.v * b.g[k]) / (b.v * b.v);
    return r;
}
static dn dsqrt_(dn a) { dn r; r.v = sqrt(a.v); for (int k = 0; k < NT; ++k) r.g[k] = a.g[k] / (2.0 * r.v); return r; }
static dn dsin_(dn a) { dn r; r.v = sin(a.v); double c = cos(a.v); for (int k = 0; k < NT; ++k) r.g[k] = c * a.g[k]; return r; }
static dn dcos_(dn a) { dn r; r.v = cos(a.v); double s = -sin(a.v); for (int k = 0; k < NT; ++k) r.g[k] = s * a.g[k]; return r; }
static dn dneg(dn a) { return dsub(dc(0.0), a); }

static dv DV(dn x, dn y, dn z) { dv r = {x, y, z}; return r; }
static dv dvc(v3 a) { return DV(dc(a.x), dc(a.y), dc(a.z)); }
static dv dvadd(dv a, dv b) { return DV(dadd(a.x, b.x), dadd(a.y, b.y), dadd(a.z, b.z)); }
static dv dvsub(dv a, dv b) { return DV(dsub(a.x, b.x), dsub(a.y, b.y), dsub(a.z, b.z)); }
static dv dvscale(dv a, dn s) { return DV(dmul(a.x, s), dmul(a.y, s), dmul(a.z, s)); }
static dn dvdot(dv a, dv b) { return dadd(dadd(dmul(a.x, b.x), dmul(a.y, b.y)), dmul(a.z, b.z)); }
static dv dvcross(dv a, dv b)
{
    return DV(dsub(dmul(a.y, b.z), dmul(a.z, b.y)), dsub(dmul(a.z, b.x), dmul(a.x, b.z)),
              dsub(dmul(a.x, b.y), dmul(a.y, b.x)));
}
static dv dvunit(dv a) { return dvscale(a, ddiv(dc(1.0), dsqrt_(dvdot(a, a)))); }

static dv drodrigues(v3 k, dn th, dv v)
{
    dv K = dvc(k);
    dn c = dcos_(th), s = dsin_(th);
    dn one_c = dsub(dc(1.0), c);
    return dvadd(dvadd(dvscale(v, c), dvscale(dvcross(K, v), s)), dvscale(K, dmul(dvdot(K, v), one_c)));
}

/* Segment parameters as duals: tangents only for the tracked segment. */
static void seg_params(const orc_scene *s, int k, int tracked, dn p[6])
{
    for (int m = 0; m < 6; ++m) p[m] = (k == tracked) ? dvar(s->params[6 * k + m], m) : dc(s->params[6 * k + m]);
}

static dv dreflect(dv d, dv n) { return dvsub(d, dvscale(n, dmul(dc(2.0), dvdot(d, n)))); }

static dn dplane_t(dv o, dv d, dv c, dv n) { return ddiv(dvdot(dvsub(c, o), n), dvdot(d, n)); }

/* ------------------------------------------------------------------------ */
/* Propagation                                                               */
/* ------------------------------------------------------------------------ */

typedef struct { int64_t prim; int root; } pathrec;

static double mind(double a, double b) { return a < b ? a : b; }

static double pixel_margin(double u, double half_extent, double pitch)
{
    double f = u + half_extent;
    if (f < 0) return -f;
    double cell = f / pitch;
    double i = floor(cell);
    return mind(f - i * pitch, (i + 1) * pitch - f);
}

static double seg_dist(v3 P, v3 a, v3 b)
{
    v3 e = vsub(b, a);
    return vlen(vcross(vsub(P, a), e)) / vlen(e);
}

typedef struct {
    const orc_scene *s;
    const orc_source *src;
    uint64_t n, seed, first_id;
    const uint64_t *ids;       /* optional list of photon ids */
    int use_bvh, with_jac;
    const orc_outputs *out;
    uint64_t begin, end;
} job;

/* Forward-mode pass along the recorded path with tangents on the six
 * parameters of segment `tracked` only (every other segment held at its
 * current parameters): J = d(u,v)/d(params of tracked), [2][6]. */
static void jacobian_of(const orc_scene *s, const photon *ph, const pathrec *path, int npath, int tracked, double *J)
{
    int64_t nc = s->d.n_cap, nr = s->d.n_rect, tb = nc + nr + 2;
    dv o = dvc(ph->o), d = dvc(ph->d);
    for (int q = 0; q < npath; ++q) {
        int64_t p = path[q].prim;
        if (p < nc) {                                   /* spherical cap */
            int k = s->cap_seg[p];
            dn pr[6];
            seg_params(s, k, tracked, pr);
            dv ax = drodrigues(vload(s->seg_e2 + 3 * k), pr[1],
                               drodrigues(vload(s->seg_e1 + 3 * k), pr[0], dvc(vload(s->seg_u0 + 3 * k))));
            dv C = dvadd(dvadd(dvc(vload(s->seg_pivot + 3 * k)), DV(pr[3], pr[4], pr[5])), dvscale(ax, pr[2]));
            dv f = dvsub(o, C);
            dn b = dvdot(f, d);
            dn c = dsub(dvdot(f, f), dmul(pr[2], pr[2]));
            dn sq = dsqrt_(dsub(dmul(b, b), c));
            dn t = path[q].root == 0 ? dsub(dneg(b), sq) : dadd(dneg(b), sq);
            dv P = dvadd(o, dvscale(d, t));
            dv n = dvscale(dvsub(C, P), ddiv(dc(1.0), pr[2]));
            d = dreflect(d, n);
            o = P;
        } else if (p < nc + nr) {                       /* flat rectangle */
            int i = (int)(p - nc);
            dv c = dvc(vload(s->rect_c + 3 * i)), n = dvc(vload(s->rect_n + 3 * i));
            dn t = dplane_t(o, d, c, n);
            o = dvadd(o, dvscale(d, t));
            d = dreflect(d, n);
        } else if (p == nc + nr) {                      /* detector plane */
            dv c = dvc(vload(s->d.det_c)), n = dvc(vload(s->d.det_n));
            dn t = dplane_t(o, d, c, n);
            dv P = dvadd(o, dvscale(d, t));
            dn u = dvdot(dvsub(P, c), dvc(vload(s->d.det_u)));
            dn v = dvdot(dvsub(P, c), dvc(vload(s->d.det_v)));
            for (int m = 0; m < 6; ++m) { J[m] = u.g[m]; J[6 + m] = v.g[m]; }
            return;
        } else if (p >= tb) {                           /* triangle */
            int64_t j = p - tb;
            int k = s->tri_seg[j];
            dv w[3];
            if (k >= 0) {
                dn pr[6];
                seg_params(s, k, tracked, pr);
                v3 piv = vload(s->seg_pivot + 3 * k);
                dn sc = ddiv(pr[2], dc(s->seg_r0[k]));
                for (int m = 0; m < 3; ++m) {
                    dv rel = dvscale(dvc(vsub(vload(s->tri_v0 + 9 * j + 3 * m), piv)), sc);
                    dv r = drodrigues(vload(s->seg_e2 + 3 * k), pr[1], drodrigues(vload(s->seg_e1 + 3 * k), pr[0], rel));
                    w[m] = dvadd(dvadd(dvc(piv), DV(pr[3], pr[4], pr[5])), r);
                }
            } else {
                for (int m = 0; m < 3; ++m) w[m] = dvc(vload(s->tri + 9 * j + 3 * m));
            }
            dv n = dvunit(dvcross(dvsub(w[1], w[0]), dvsub(w[2], w[0])));
            dn t = dplane_t(o, d, w[0], n);
            o = dvadd(o, dvscale(d, t));
            d = dreflect(d, n);
        }
    }
    for (int m = 0; m < 12; ++m) J[m] = NAN;
}

/* Jacobians of the detector coordinates with respect to every parametrised
 * segment on the path: one forward-mode pass per distinct segment (the total
 * derivative is their sum by the chain rule).  segs[k] / Js[k] for the k-th
 * distinct segment met; the single-segment outputs seg_out / J keep the one
 * segment (-1 none; -2 several, -3 more than ORC_MAX_PATH_SEGS: J NaN). */
static void jacobian(const orc_scene *s, const photon *ph, const pathrec *path, int npath, int32_t *seg_out,
                     double *J, int32_t *segs, double *Js)
{
    int64_t nc = s->d.n_cap, nr = s->d.n_rect, tb = nc + nr + 2;
    int found[ORC_MAX_PATH_SEGS], nfound = 0, too_many = 0;
    for (int q = 0; q < npath; ++q) {
        int64_t p = path[q].prim;
        int k = -1;
        if (p < nc) k = s->cap_seg[p];
        else if (p >= tb) k = s->tri_seg[p - tb];
        if (k < 0) continue;
        int seen = 0;
        for (int m = 0; m < nfound; ++m) seen |= found[m] == k;
        if (seen) continue;
        if (nfound == ORC_MAX_PATH_SEGS) { too_many = 1; break; }
        found[nfound++] = k;
    }
    for (int m = 0; m < ORC_MAX_PATH_SEGS; ++m) segs[m] = -1;
    for (int m = 0; m < 12 * ORC_MAX_PATH_SEGS; ++m) Js[m] = NAN;
    for (int m = 0; m < 12; ++m) J[m] = NAN;
    if (too_many) { *seg_out = -3; return; }
    for (int m = 0; m < nfound; ++m) {
        segs[m] = found[m];
        jacobian_of(s, ph, path, npath, found[m], Js + 12 * m);
    }
    if (nfound == 0) {
        *seg_out = -1;
        jacobian_of(s, ph, path, npath, -1, J);   /* no tangent: zeros */
    } else if (nfound == 1) {
        *seg_out = found[0];
        memcpy(J, Js, 12 * sizeof(double));
    } else {
        *seg_out = -2;
    }
}

static void trace_photon(const job *jb, uint64_t i)
{
    const orc_scene *s = jb->s;
    const orc_outputs *out = jb->out;
    uint64_t g = jb->ids ? jb->ids[i] : jb->first_id + i;
    photon ph;
    make_photon(jb->src, jb->seed, g, i, &ph);
    v3 o = ph.o, d = ph.d;
    int64_t nc = s->d.n_cap, nr = s->d.n_rect, det_id = nc + nr, box_id = nc + nr + 1, tb = nc + nr + 2;
    int fate = ORC_MAX_BOUNCES, pixel = -1, nb = 0;
    double hxyz[3] = {NAN, NAN, NAN}, huv[2] = {NAN, NAN}, htime = NAN;
    double travelled = 0.0;         /* path length so far (mm) */
    double emargin = INFINITY, rmargin = ph.margin, pmargin = INFINITY;
    pathrec path[64];
    int npath = 0;
    uint32_t blk[4];
    int have_blk = -1;
    int eff = 1;                    /* efficiencies applied at the surfaces */
    int nloop = s->d.max_bounces;
    if (jb->src->prefilter) {
        double m;
        if (!prefilter_keep(s, jb->src, jb->seed, g, ph.lambda, &m)) {
            fate = ORC_PREFILTERED;
            nloop = 0;
        }
        rmargin = fmin(m, ph.margin);
        eff = 0;
    }

    for (int b = 0; b < nloop; ++b) {
        hitrec h;
        closest_hit(s, o, d, jb->use_bvh, &h);
        if (h.prim < 0) { fate = ORC_ESCAPED; break; }
        ++nb;
        if (npath < 64) { path[npath].prim = h.prim; path[npath].root = h.root; ++npath; }
        v3 P = vadd(o, vmul(d, h.t));
        travelled += h.t;
        if (h.prim == det_id) {
            v3 n = vload(s->d.det_n), c = vload(s->d.det_c);
            if (vdot(d, n) >= 0) { fate = ORC_ABSORBED; break; }
            double u = vdot(vsub(P, c), vload(s->d.det_u)), v = vdot(vsub(P, c), vload(s->d.det_v));
            double p = s->d.det_pitch;
            double hu = 0.5 * s->d.det_nx * p, hv = 0.5 * s->d.det_ny * p;
            emargin = mind(emargin, mind(s->d.det_half[0] - fabs(u), s->d.det_half[1] - fabs(v)));
            pmargin = mind(pixel_margin(u, hu, p), pixel_margin(v, hv, p));
            double fi = floor((u + hu) / p), fj = floor((v + hv) / p);
            if (fi < 0 || fi >= s->d.det_nx || fj < 0 || fj >= s->d.det_ny) { fate = ORC_ABSORBED; break; }
            pixel = (int)fj * s->d.det_nx + (int)fi;
            hxyz[0] = P.x; hxyz[1] = P.y; hxyz[2] = P.z;
            htime = ph.t0 + travelled * ph.ng / C_MM_PER_NS;
            huv[0] = u; huv[1] = v;
            if (eff) {
                double qe = table(s->d.n_qe, s->d.qe_x, s->d.qe_y, ph.lambda);
                rmargin = mind(rmargin, fabs(ph.u_qe - qe));
                fate = (ph.u_qe < qe) ? ORC_DETECTED : ORC_QE_REJECTED;
            } else {
                fate = ORC_DETECTED;
            }
            break;
        }
        if (h.prim == box_id) { fate = ORC_ABSORBED; break; }
        /* mirror or absorber surface */
        int mat;
        v3 n;
        if (h.prim < nc) {
            int i2 = (int)h.prim;
            mat = s->cap_mat[i2];
            n = vmul(vsub(vload(s->cap_C + 3 * i2), P), 1.0 / s->cap_R[i2]);
            if (s->mat_kind[mat] == ORC_MIRROR) {
                v3 O = vload(s->cap_origin + 3 * i2);
                double a = vdot(vsub(P, O), vload(s->cap_a + 3 * i2)), bb = vdot(vsub(P, O), vload(s->cap_b + 3 * i2));
                const double *bd = s->cap_bounds + 4 * i2;
                emargin = mind(emargin, mind(mind(a - bd[0], bd[1] - a), mind(bb - bd[2], bd[3] - bb)));
            }
        } else if (h.prim < nc + nr) {
            int i2 = (int)(h.prim - nc);
            mat = s->rect_mat[i2];
            n = vload(s->rect_n + 3 * i2);
            if (s->mat_kind[mat] == ORC_MIRROR) {
                v3 c = vload(s->rect_c + 3 * i2);
                double u = vdot(vsub(P, c), vload(s->rect_u + 3 * i2)), v = vdot(vsub(P, c), vload(s->rect_v + 3 * i2));
                emargin = mind(emargin, mind(s->rect_half[2 * i2] - fabs(u), s->rect_half[2 * i2 + 1] - fabs(v)));
            }
        } else {
            int64_t j = h.prim - tb;
            mat = s->tri_mat[j];
            n = vload(s->tri_nrm + 3 * j);
            if (s->mat_kind[mat] == ORC_MIRROR) {
                v3 a = vload(s->tri + 9 * j), bq = vload(s->tri + 9 * j + 3), c = vload(s->tri + 9 * j + 6);
                emargin = mind(emargin, mind(seg_dist(P, a, bq), mind(seg_dist(P, bq, c), seg_dist(P, c, a))));
            }
        }
        if (s->mat_kind[mat] != ORC_MIRROR || vdot(d, n) >= 0) { fate = ORC_ABSORBED; break; }
        /* reflectivity roulette: word (b mod 4) of block 1 + b/4 */
        if (eff) {
            if (have_blk != 1 + b / 4) { photon_block(jb->seed, g, (uint32_t)(1 + b / 4), blk); have_blk = 1 + b / 4; }
            double uR = u24(blk[b % 4]);
            double R = table(s->mat_nrefl[mat], s->mat_refl_x + ORC_MAX_TABLE * mat,
                             s->mat_refl_y + ORC_MAX_TABLE * mat, ph.lambda);
            rmargin = mind(rmargin, fabs(uR - R));
            if (uR >= R) { fate = ORC_ABSORBED_MIRROR; break; }
        }
        d = vsub(d, vmul(n, 2.0 * vdot(d, n)));
        o = P;
    }

    if (out->fate) out->fate[i] = (uint8_t)fate;
    if (out->pixel) out->pixel[i] = pixel;
    if (out->hit_xyz) for (int a = 0; a < 3; ++a) out->hit_xyz[3 * i + a] = hxyz[a];
    if (out->hit_uv) { out->hit_uv[2 * i] = huv[0]; out->hit_uv[2 * i + 1] = huv[1]; }
    if (out->hit_time) out->hit_time[i] = htime;
    if (out->edge_margin) out->edge_margin[i] = emargin;
    if (out->roulette_margin) out->roulette_margin[i] = rmargin;
    if (out->pixel_margin) out->pixel_margin[i] = pmargin;
    if (out->n_bounce) out->n_bounce[i] = nb;
    if (jb->with_jac && (out->jac || out->segment || out->segments || out->jacs)) {
        int32_t sg = -1, sgs[ORC_MAX_PATH_SEGS];
        double J[12], Js[12 * ORC_MAX_PATH_SEGS];
        if (fate == ORC_DETECTED || fate == ORC_QE_REJECTED) {
            jacobian(s, &ph, path, npath, &sg, J, sgs, Js);
        } else {
            for (int m = 0; m < 12; ++m) J[m] = NAN;
            for (int m = 0; m < ORC_MAX_PATH_SEGS; ++m) sgs[m] = -1;
            for (int m = 0; m < 12 * ORC_MAX_PATH_SEGS; ++m) Js[m] = NAN;
        }
        if (out->segment) out->segment[i] = sg;
        if (out->jac) for (int m = 0; m < 12; ++m) out->jac[12 * i + m] = J[m];
        if (out->segments) for (int m = 0; m < ORC_MAX_PATH_SEGS; ++m) out->segments[ORC_MAX_PATH_SEGS * i + m] = sgs[m];
        if (out->jacs)
            for (int m = 0; m < 12 * ORC_MAX_PATH_SEGS; ++m) out->jacs[12 * ORC_MAX_PATH_SEGS * i + m] = Js[m];
    }
}

static void *run_job(void *arg)
{
    const job *jb = (const job *)arg;
    for (uint64_t i = jb->begin; i < jb->end; ++i) trace_photon(jb, i);
    return NULL;
}

static int propagate_any(const orc_scene *s, const orc_source *src, const uint64_t *ids, uint64_t n, uint64_t seed,
                         uint64_t first_id, int use_bvh, int with_jacobian, int n_threads, const orc_outputs *out)
{
    if (!s || !src || !out) { set_err("null argument"); return -1; }
    if (ids && src->kind == ORC_SRC_EXPLICIT) { set_err("id lists need a generated source"); return -1; }
    if (src->prefilter) {
        if (src->pf_n < 0 || src->pf_n > 4) { set_err("prefilter: 0..4 materials"); return -1; }
        for (int k = 0; k < src->pf_n; ++k)
            if (src->pf_mats[k] < 0 || src->pf_mats[k] >= s->d.n_mat || s->mat_kind[src->pf_mats[k]] != ORC_MIRROR) {
                set_err("prefilter material is not a mirror");
                return -1;
            }
    }
    if (src->kind != ORC_SRC_EXPLICIT) {
        if (!(src->n_radiator > 0) || !(src->lambda_min > 0) || !(src->lambda_max > src->lambda_min)) {
            set_err("bad source spectrum");
            return -1;
        }
        if (src->n_disp < 0 || src->n_disp > ORC_MAX_TABLE) { set_err("dispersion: 0..32 nodes"); return -1; }
        for (int k = 0; k < src->n_disp; ++k) {
            if (!(src->disp_n[k] >= 1.0) || (k > 0 && !(src->disp_x[k] > src->disp_x[k - 1]))) {
                set_err("dispersion: increasing wavelengths and indices >= 1");
                return -1;
            }
        }
        /* the largest index over the band must be above threshold for every track */
        double nmax = src->n_disp > 0 ? max_index(src) : src->n_radiator;
        if (src->kind == ORC_SRC_TRACK && !(nmax * src->beta > 1.0)) { set_err("n beta <= 1"); return -1; }
        if (src->kind == ORC_SRC_BATCH) {
            for (int64_t k = 0; k < src->n_tracks; ++k)
                if (!(nmax * src->tracks[8 * k + 7] > 1.0)) { set_err("n beta <= 1"); return -1; }
            uint64_t total = src->offsets[src->n_tracks];
            if (!ids && first_id + n > total) { set_err("photon id beyond the batch"); return -1; }
            if (ids)
                for (uint64_t i = 0; i < n; ++i)
                    if (ids[i] >= total) { set_err("photon id beyond the batch"); return -1; }
        }
    }
    if (n_threads < 1) n_threads = 1;
    if ((uint64_t)n_threads > n) n_threads = n > 0 ? (int)n : 1;
    job *jobs = calloc((size_t)n_threads, sizeof(job));
    pthread_t *th = calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); set_err("out of memory"); return -1; }
    for (int k = 0; k < n_threads; ++k) {
        jobs[k].s = s;
        jobs[k].src = src;
        jobs[k].n = n;
        jobs[k].seed = seed;
        jobs[k].first_id = first_id;
        jobs[k].ids = ids;
        jobs[k].use_bvh = use_bvh;
        jobs[k].with_jac = with_jacobian;
        jobs[k].out = out;
        jobs[k].begin = n * (uint64_t)k / (uint64_t)n_threads;
        jobs[k].end = n * (uint64_t)(k + 1) / (uint64_t)n_threads;
    }
    if (n_threads == 1) {
        run_job(&jobs[0]);
    } else {
        for (int k = 0; k < n_threads; ++k) pthread_create(&th[k], NULL, run_job, &jobs[k]);
        for (int k = 0; k < n_threads; ++k) pthread_join(th[k], NULL);
    }
    free(jobs);
    free(th);
    return 0;
}

int orc_propagate(const orc_scene *s, const orc_source *src, uint64_t n, uint64_t seed, uint64_t first_id,
                  int use_bvh, int with_jacobian, int n_threads, const orc_outputs *out)
{
    return propagate_any(s, src, NULL, n, seed, first_id, use_bvh, with_jacobian, n_threads, out);
}

int orc_propagate_ids(const orc_scene *s, const orc_source *src, const uint64_t *ids, uint64_t n, uint64_t seed,
                      int use_bvh, int with_jacobian, int n_threads, const orc_outputs *out)
{
    return propagate_any(s, src, ids, n, seed, 0, use_bvh, with_jacobian, n_threads, out);
}

/* ------------------------------------------------------------------------ */
/* Cherenkov yield (Frank-Tamm)                                              */
/* ------------------------------------------------------------------------ */

static double yield_integrand(const orc_source *src, double beta, double lambda_nm)
{
    return ft_weight(index_at(src, lambda_nm), beta) / (lambda_nm * lambda_nm);
}

int orc_cherenkov_yield(const orc_source *src, double beta, double *photons_per_mm)
{
    if (!src || !photons_per_mm) { set_err("null argument"); return -1; }
    if (!(src->lambda_min > 0) || !(src->lambda_max > src->lambda_min) || !(beta > 0)) {
        set_err("bad spectrum or beta");
        return -1;
    }
    if (src->n_disp < 0 || src->n_disp > ORC_MAX_TABLE) { set_err("dispersion: 0..32 nodes"); return -1; }
    /* breakpoints: the band ends and every table node inside the band; the
     * threshold crossing inside a segment is handled by refining: composite
     * Simpson with 20000 panels per piece of the piecewise-linear n */
    double bp[ORC_MAX_TABLE + 2];
    int nb = 0;
    bp[nb++] = src->lambda_min;
    for (int k = 0; k < src->n_disp; ++k)
        if (src->disp_x[k] > src->lambda_min && src->disp_x[k] < src->lambda_max) bp[nb++] = src->disp_x[k];
    bp[nb++] = src->lambda_max;
    double integral = 0.0;   /* of w / lambda^2 over lambda in nm, units 1/nm */
    const int panels = 20000;
    for (int q = 0; q + 1 < nb; ++q) {
        double lo = bp[q], hi = bp[q + 1];
        /* threshold inside this piece: split there so Simpson sees no kink */
        double cut[3] = {lo, hi, hi};
        int nc = 2;
        double wlo = 1.0 - 1.0 / (beta * beta * index_at(src, lo) * index_at(src, lo));
        double whi = 1.0 - 1.0 / (beta * beta * index_at(src, hi) * index_at(src, hi));
        if ((wlo > 0) != (whi > 0)) {
            /* n is linear on the piece: solve n(lambda) = 1/beta */
            double nl = index_at(src, lo), nh = index_at(src, hi);
            double lam = lo + (1.0 / beta - nl) / (nh - nl) * (hi - lo);
            cut[1] = lam;
            cut[2] = hi;
            nc = 3;
        }
        for (int c = 0; c + 1 < nc; ++c) {
            double a = cut[c], b = cut[c + 1];
            double h = (b - a) / panels, sum = yield_integrand(src, beta, a) + yield_integrand(src, beta, b);
            for (int j = 1; j < panels; ++j) sum += (j % 2 ? 4.0 : 2.0) * yield_integrand(src, beta, a + j * h);
            integral += sum * h / 3.0;
        }
    }
    /* lambda in mm: integral of w / lambda_mm^2 d lambda_mm = 1e6 x the nm integral */
    *photons_per_mm = 2.0 * M_PI * FINE_STRUCTURE * 1e6 * integral;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Film read-out emulation (Section 4.4)                                     */
/* ------------------------------------------------------------------------ */

int orc_film_readout(const orc_film *film, const uint8_t *fate, const double *hit_uv, uint64_t n, double *image,
                     uint8_t *hits)
{
    if (!film || !image || (n && (!fate || !hit_uv))) { set_err("null argument"); return -1; }
    if (film->width < 1 || film->height < 1 || !(film->distance > 0) || !(film->fov > 0) || !(film->fov < M_PI) ||
        !(film->sigma > 0)) {
        set_err("bad film");
        return -1;
    }
    const int W = film->width, H = film->height;
    const double f = 0.5 * W / tan(0.5 * film->fov);
    const double r = 4.0 * film->sigma;
    for (uint64_t p = 0; p < n; ++p) {
        if (fate[p] != ORC_DETECTED) continue;
        double x = 0.5 * W + f * hit_uv[2 * p] / film->distance;
        double y = 0.5 * H + f * hit_uv[2 * p + 1] / film->distance;
        /* pixels with centres i + 1/2 in [x - r, x + r] */
        int i0 = (int)ceil(x - r - 0.5), i1 = (int)floor(x + r - 0.5);
        int j0 = (int)ceil(y - r - 0.5), j1 = (int)floor(y + r - 0.5);
        for (int j = j0 > 0 ? j0 : 0; j <= j1 && j < H; ++j)
            for (int i = i0 > 0 ? i0 : 0; i <= i1 && i < W; ++i) {
                double dx = i + 0.5 - x, dy = j + 0.5 - y;
                image[(int64_t)j * W + i] += 255.0 * exp(-(dx * dx + dy * dy) / (2.0 * film->sigma * film->sigma));
            }
    }
    if (hits)
        for (int64_t k = 0; k < (int64_t)W * H; ++k) hits[k] = fmin(image[k], 255.0) >= film->threshold;
    return 0;
}
