// Device functions of the photon path: random stream, generation, closest hit,
// interaction.  Shared by the forward, batch and adjoint kernels.
//
// Precision: FP32 throughout, except the Cherenkov cone constants of batch
// tracks (1/(n beta) and its sine, FP64 to avoid cancellation in 1 - cos^2)
// and the rare watertight-test fallback on exactly-zero edge functions.
#pragma once

#include "rich_dev.h"

namespace rich {

// ---------------------------------------------------------------- vectors

struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 ld3(const float *p) { return V3{p[0], p[1], p[2]}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 fma3(float s, V3 a, V3 b) {  // s*a + b
    return V3{fmaf(s, a.x, b.x), fmaf(s, a.y, b.y), fmaf(s, a.z, b.z)};
}
__device__ __forceinline__ V3 mat3(const float *m, V3 v) {  // row-major 3x3 times v
    return V3{fmaf(m[0], v.x, fmaf(m[1], v.y, m[2] * v.z)), fmaf(m[3], v.x, fmaf(m[4], v.y, m[5] * v.z)),
              fmaf(m[6], v.x, fmaf(m[7], v.y, m[8] * v.z))};
}
__device__ __forceinline__ float comp(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

// Scene data (caps, rects, detector, materials and their tables) is never
// written while a propagation kernel runs: the prepare kernel updates it in an
// earlier launch.  Reading it through the constant address space tells the
// compiler so, and reads at wave-uniform addresses (the loops over analytic
// primitives and table nodes) become one scalar load per wave instead of one
// vector load per lane.  Without it, any output store earlier in the kernel
// keeps the compiler from proving the data unchanged.
#define RICH_CONST __attribute__((address_space(4)))

// Work counters of the measurement build (compiled with -DRICH_WORK_COUNTERS;
// the product library has none of this).  Each counts one unit of work per
// active lane: a traced photon, a Philox block (of which the regrouping's
// second draw of block 0 for its sort key is also counted apart), a
// closest-hit query (ray set-up and the detector plane), a cap's bounding-box
// test and its sphere test, a rectangle, the analytic box, a BVH4 node whose
// four child boxes are tested, a leaf, a triangle test, an entry into a mesh
// instance's frame (and apart those that rotate and scale the ray), a
// reflection, a detector hit; in the adjoint, a counted photon's pass back
// through the detector plane and each reflection it sweeps back through (cap
// or facet).  Lanes of a wave are summed with one atomic per counter and wave;
// a second word in the counter's line counts the waves that did the unit, so
// lanes / (64 x waves) is the unit's SIMD efficiency.
enum WorkUnit {
    kWorkPhotons, kWorkPhilox, kWorkSortKeys, kWorkQueries, kWorkCapBoxes, kWorkCaps, kWorkRects, kWorkBoxes,
    kWorkNodes, kWorkLeaves, kWorkTris, kWorkInstances, kWorkMovingInstances, kWorkReflections, kWorkDetections,
    kWorkBackDetector, kWorkBackCaps, kWorkBackFacets, kWorkBackPlanes, kWorkUnits
};
#ifdef RICH_WORK_COUNTERS
static __device__ unsigned long long rich_work[16 * kWorkUnits];   // one 128-byte line per counter
__device__ __forceinline__ void work(int unit) {
    const unsigned long long m = __ballot(1);
    if (__lane_id() == __ffsll((long long)m) - 1) {
        atomicAdd(&rich_work[16 * unit], (unsigned long long)__popcll(m));
        atomicAdd(&rich_work[16 * unit + 1], 1ull);
    }
}
#else
__device__ __forceinline__ void work(int) {}
#endif
template <class T>
__device__ __forceinline__ const RICH_CONST T &cref(const T &x) {
    return *(const RICH_CONST T *)&x;
}
__device__ __forceinline__ V3 ld3(const RICH_CONST float *p) { return V3{p[0], p[1], p[2]}; }

// ---------------------------------------------------------------- Philox4x32-10

// Counter-based generator of Salmon et al. (SC'11): ten rounds of two 32x32->64
// multiplies whose halves are cross-mixed with the other words and the key;
// the key advances by the Weyl constants (golden ratio, sqrt 3) each round.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c.x;   // one 32x32->64 multiply gives both halves
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint4 photon_block(uint64_t seed, uint64_t g, uint32_t blk) {
    work(kWorkPhilox);
    return philox4x32_10(make_uint4((uint32_t)g, (uint32_t)(g >> 32), blk, kStreamTag), (uint32_t)seed,
                         (uint32_t)(seed >> 32));
}

// top 24 bits as a float in [0,1): exact
__device__ __forceinline__ float u24(uint32_t x) { return (float)(x >> 8) * 5.9604644775390625e-8f; }

// Hardware reciprocal (1 ulp).  Used on the geometric path where a few ulps
// are far below the tolerance; the IEEE division sequence costs ~10 instructions.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------- tables

// Piecewise-linear table with per-segment slopes, clamped outside its range.
// The loop bound and the node addresses are uniform, so the nodes arrive
// through scalar loads and each lane only selects.
template <class P>   // const float * or const RICH_CONST float *
__device__ __forceinline__ float lerp_table(int n, P x, P y, P sl, float l) {
    float v = l <= x[0] ? y[0] : y[n - 1];
    for (int j = 0; j + 1 < n; ++j) {
        float xa = x[j];
        if (l >= xa && l < x[j + 1]) v = fmaf(sl[j], l - xa, y[j]);
    }
    return v;
}

// ---------------------------------------------------------------- generation

struct Photon {
    V3 o, d;
    float lambda;
    float u_qe;
    float t0;       // emission time after the track start (ns)
    float ng_c;     // group index / c (ns per mm)
};

// n(lambda) - 1 and the table slope dn/dlambda at l (slope 0 outside the
// table), by the same uniform scan as lerp_table.
__device__ __forceinline__ float disp_lookup(const DevSource &src, float l, float &slope) {
    const int n = src.n_disp;
    float v = l <= src.disp_x[0] ? src.disp_m[0] : src.disp_m[n - 1];
    slope = 0.0f;
    for (int j = 0; j + 1 < n; ++j) {
        float xa = src.disp_x[j];
        if (l >= xa && l < src.disp_x[j + 1]) {
            v = fmaf(src.disp_s[j], l - xa, src.disp_m[j]);
            slope = src.disp_s[j];
        }
    }
    return v;
}

// Frank-Tamm weight 1 - 1/(beta n)^2 (zero below threshold), FP64: n - 1 is
// small, so the cone and the acceptance need more than FP32 carries in n.
__device__ __forceinline__ double ft_weight(double n, double beta) {
    double w = 1.0 - 1.0 / (beta * beta * n * n);
    return w > 0.0 ? w : 0.0;
}

__device__ __forceinline__ int find_track(const uint64_t *off, int n_tracks, uint64_t g) {
    int lo = 0, hi = n_tracks;  // last k with off[k] <= g
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// Track of photon g when the wave's photons mostly share one: a scalar
// binary search (constant address space, wave-uniform index) for the wave's
// first active photon; lanes outside that track's id range try the next two
// tracks (a wave of consecutive ids that crosses a boundary) and search on
// their own only beyond them.
__device__ __forceinline__ int find_track_wave(const uint64_t *off, int n_tracks, uint64_t g) {
    const RICH_CONST uint64_t *oc = (const RICH_CONST uint64_t *)off;
    const uint64_t g0 = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(g >> 32)) << 32) |
                        __builtin_amdgcn_readfirstlane((uint32_t)g);
    int lo = 0, hi = n_tracks;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (oc[mid] <= g0) lo = mid; else hi = mid;
    }
    if (g >= oc[lo] && g < oc[lo + 1]) return lo;
    if (g >= oc[lo + 1]) {
        for (int k = lo + 1; k < lo + 3 && k < n_tracks; ++k)
            if (g < off[k + 1]) return k;
    }
    return find_track(off, n_tracks, g);
}

// Orthonormal basis (b1, b2) around unit n, after Duff et al., JCGT 2017.
__device__ __forceinline__ void basis(V3 n, V3 &b1, V3 &b2) {
    float sgn = copysignf(1.0f, n.z);
    float a = -1.0f / (sgn + n.z);
    float b = n.x * n.y * a;
    b1 = V3{1.0f + sgn * n.x * n.x * a, sgn * b, -sgn * n.x};
    b2 = V3{b, sgn + n.y * n.y * a, -n.y};
}

// wave_track: the wave's photons come from consecutive ids (forward and batch
// kernels), so most lanes share the first lane's track; the adjoint's queued
// photons do not, and search per lane.  track >= 0: the caller knows the
// photon's track (batch processing order) and no search is made.
__device__ __forceinline__ Photon make_photon(const DevSource &src, uint64_t seed, uint64_t g, uint64_t i,
                                              bool wave_track = true, int track = -1) {
    uint4 w = photon_block(seed, g, 0);
    Photon ph;
    ph.u_qe = u24(w.w);
    if (src.kind == 2) {
        ph.o = ld3(src.ex_o + 3 * i);
        ph.d = ld3(src.ex_d + 3 * i);
        ph.lambda = src.ex_l[i];
        ph.t0 = 0.0f;
        float slope = 0.0f, m = src.n_disp > 0 ? disp_lookup(src, ph.lambda, slope) : 0.0f;
        ph.ng_c = (src.n_disp > 0 ? 1.0f + fmaf(-ph.lambda, slope, m) : src.ng_const) * kInvC;
        return ph;
    }
    V3 P0, T, E1, E2;
    float L, ct, st, beta;
    if (src.kind == 1) {
        int k = track >= 0 ? track
                           : (wave_track ? find_track_wave(src.offsets, src.n_tracks, g)
                                         : find_track(src.offsets, src.n_tracks, g));
        const float4 *tr = reinterpret_cast<const float4 *>(src.tracks) + 2 * k;
        float4 a = tr[0], b = tr[1];
        P0 = V3{a.x, a.y, a.z};
        T = V3{a.w, b.x, b.y};
        T = rsqrtf(dot(T, T)) * T;
        L = b.z;
        beta = b.w;
        double c = 1.0 / (src.n_radiator * (double)b.w);
        ct = (float)c;
        st = (float)sqrt((1.0 - c) * (1.0 + c));
        basis(T, E1, E2);
    } else {
        P0 = ld3(src.P0);
        T = ld3(src.T);
        E1 = ld3(src.E1);
        E2 = ld3(src.E2);
        L = src.length;
        ct = src.cos_t;
        st = src.sin_t;
        beta = src.beta;
    }
    ph.lambda = rcp(fmaf(-u24(w.y), src.inv_span, src.inv_lmin));
    ph.ng_c = src.ng_const * kInvC;
    if (src.n_disp > 0) {
        // Frank-Tamm spectrum with dispersion: accept the 1/lambda^2 draw with
        // probability w(lambda)/w_max, else draw again from the next block
        const double b2 = (double)beta;
        const double wmax = ft_weight(src.disp_nmax, b2);
        float slope = 0.0f, m = 0.0f;
        for (int k = 0; k < kDispMaxTries; ++k) {
            uint4 r = photon_block(seed, g, kDispBlock - (uint32_t)k);
            if (k > 0) ph.lambda = rcp(fmaf(-u24(r.y), src.inv_span, src.inv_lmin));
            m = disp_lookup(src, ph.lambda, slope);
            if ((double)u24(r.x) < ft_weight(1.0 + (double)m, b2) / wmax) break;
        }
        // the cone at the photon's own index
        double c = 1.0 / ((1.0 + (double)m) * b2);
        ct = (float)c;
        st = (float)sqrt((1.0 - c) * (1.0 + c));
        ph.ng_c = (1.0f + fmaf(-ph.lambda, slope, m)) * kInvC;
    }
    float sp, cp;
    sincospif(2.0f * u24(w.x), &sp, &cp);
    V3 d = fma3(ct, T, st * fma3(cp, E1, sp * E2));
    ph.d = rsqrtf(dot(d, d)) * d;
    const float s = u24(w.z) * L;
    ph.o = fma3(s, T, P0);
    ph.t0 = s / beta * kInvC;
    return ph;
}

// ---------------------------------------------------------------- ray state

struct Ray {
    V3 o, d;          // current frame (world or instance-local)
    V3 inv;           // 1/d with zeros nudged away
    V3 oi;            // o * inv
};

constexpr float kFarScale = 1.0000004f;

__device__ __forceinline__ float safe_inv(float x) {
    return rcp(fabsf(x) > 1e-30f ? x : copysignf(1e-30f, x));
}

__device__ __forceinline__ void ray_setup(Ray &r, V3 o, V3 d) {
    r.o = o;
    r.d = d;
    r.inv = V3{safe_inv(d.x), safe_inv(d.y), safe_inv(d.z)};
    r.oi = V3{o.x * r.inv.x, o.y * r.inv.y, o.z * r.inv.z};
}

// Watertight permutation and shear of a direction (Woop, Benthin, Wald).
struct Shear {
    int kx, ky, kz;
    float sx, sy, sz;
};
__device__ __forceinline__ Shear make_shear(V3 d) {
    Shear w;
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    w.kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    w.kx = w.kz == 2 ? 0 : w.kz + 1;
    w.ky = w.kx == 2 ? 0 : w.kx + 1;
    float dz = comp(d, w.kz);
    if (dz < 0.0f) { int t = w.kx; w.kx = w.ky; w.ky = t; }
    w.sz = rcp(dz);
    w.sx = comp(d, w.kx) * w.sz;
    w.sy = comp(d, w.ky) * w.sz;
    return w;
}

// Slab test of an AABB with the robust far-distance scaling of Ize (JCGT 2013).
// Returns INFINITY on a miss, else a visiting-order key: the entry distance,
// or, when the ray starts inside the box, the exit distance (an enclosure
// that contains the origin is then visited after the surfaces in front of it,
// whose hits cull most of it).
__device__ __forceinline__ float slab_entry(const Ray &r, float lx, float ly, float lz, float hx, float hy, float hz,
                                            float tmax) {
    float t0x = fmaf(lx, r.inv.x, -r.oi.x), t1x = fmaf(hx, r.inv.x, -r.oi.x);
    float t0y = fmaf(ly, r.inv.y, -r.oi.y), t1y = fmaf(hy, r.inv.y, -r.oi.y);
    float t0z = fmaf(lz, r.inv.z, -r.oi.z), t1z = fmaf(hz, r.inv.z, -r.oi.z);
    float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
    float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z)) * 1.0000004f;
    tf = fminf(tf, tmax);
    return tn <= tf ? (tn > 0.0f ? tn : tf) : INFINITY;
}

// Node-child version of slab_entry with the near and far planes already
// chosen by the direction signs (inverted empty boxes give tn > tf: a miss).
__device__ __forceinline__ float child_key(const Ray &r, float nx, float ny, float nz, float fx, float fy, float fz,
                                           float tmax) {
    float tn = fmaxf(fmaxf(fmaf(nx, r.inv.x, -r.oi.x), fmaf(ny, r.inv.y, -r.oi.y)),
                     fmaxf(fmaf(nz, r.inv.z, -r.oi.z), 0.0f));
    float tf = fminf(fminf(fmaf(fx, r.inv.x, -r.oi.x), fmaf(fy, r.inv.y, -r.oi.y)), fmaf(fz, r.inv.z, -r.oi.z));
    tf = fminf(tf * kFarScale, tmax);
    return tn <= tf ? (tn > 0.0f ? tn : tf) : INFINITY;
}

// ---------------------------------------------------------------- closest hit

struct Hit {
    float t;
    uint32_t prim;   // global primitive id (ties: lower wins)
    uint32_t tri;    // triangle slot (meshes)
    int32_t inst;    // instance of the triangle
    int32_t root;    // sphere root taken (caps)
};

__device__ __forceinline__ bool better(float t, uint32_t prim, const Hit &h) {
    return t < h.t || (t == h.t && prim < h.prim);
}

// Sphere cap with the cancellation-free discriminant of Haines et al.
// (Ray Tracing Gems, ch. 7): disc = R^2 - |f - (f.d) d|^2, roots q and c/q.
__device__ __forceinline__ bool hit_cap(const RICH_CONST CapDev &cp, V3 o, V3 d, float tmin, float &t_out, int &root) {
    V3 C = ld3(cp.C);
    V3 f = o - C;
    float b = dot(f, d);
    V3 fp = fma3(-b, d, f);
    float R = cp.R;
    float disc = fmaf(R, R, -dot(fp, fp));
    if (!(disc >= 0.0f)) return false;
    float sq = sqrtf(disc);
    float c = fmaf(-R, R, dot(f, f));
    float q = -(b + copysignf(sq, b));
    if (q == 0.0f) return false;
    float r0 = c * rcp(q), r1 = q;
    float ta = fminf(r0, r1), tb = fmaxf(r0, r1);
    V3 ax = ld3(cp.axis), O = ld3(cp.O), A = ld3(cp.A), B = ld3(cp.B);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        float t = k == 0 ? ta : tb;
        if (!(t > tmin)) continue;
        V3 P = fma3(t, d, o);
        if (dot(P - C, ax) >= 0.0f) continue;
        V3 PO = P - O;
        float a = dot(PO, A), bb = dot(PO, B);
        if (a >= cp.a_lo && a < cp.a_hi && bb >= cp.b_lo && bb < cp.b_hi) {
            t_out = t;
            root = k;
            return true;
        }
    }
    return false;
}

__device__ __forceinline__ bool hit_plane_rect(V3 c, V3 n, V3 U, V3 W, float hu, float hv, V3 o, V3 d, float tmin,
                                               float &t_out) {
    float dn = dot(d, n);
    if (dn == 0.0f) return false;
    V3 co = c - o;
    float t = dot(co, n) * rcp(dn);
    if (!(t > tmin)) return false;
    V3 Pc = fma3(t, d, o - c);
    float u = dot(Pc, U), v = dot(Pc, W);
    if (fabsf(u) <= hu && fabsf(v) <= hv) {
        t_out = t;
        return true;
    }
    return false;
}

// Box surface through the ray's inverse direction: entry or exit, whichever is first beyond tmin.
__device__ __forceinline__ bool hit_box(const float *lo, const float *hi, const Ray &r, float tmin, float &t_out) {
    float t0x = fmaf(lo[0], r.inv.x, -r.oi.x), t1x = fmaf(hi[0], r.inv.x, -r.oi.x);
    float t0y = fmaf(lo[1], r.inv.y, -r.oi.y), t1y = fmaf(hi[1], r.inv.y, -r.oi.y);
    float t0z = fmaf(lo[2], r.inv.z, -r.oi.z), t1z = fmaf(hi[2], r.inv.z, -r.oi.z);
    float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fminf(t0z, t1z));
    float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z));
    if (tn > tf) return false;
    if (tn > tmin) { t_out = tn; return true; }
    if (tf > tmin) { t_out = tf; return true; }
    return false;
}

// Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013), two-sided.
// Each edge function is two rounded products and one difference, never
// contracted into an FMA: only then does a triangle's edge function equal the
// exact negative of its neighbour's for their shared edge, so a ray through
// that edge cannot be rejected by both.
__device__ __forceinline__ bool hit_tri(const Ray &r, const Shear &sh, const float4 &a, const float4 &b,
                                        const float4 &c, float tmin, float &t_out) {
#pragma clang fp contract(off)
    V3 A = V3{a.x, a.y, a.z} - r.o, B = V3{b.x, b.y, b.z} - r.o, C = V3{c.x, c.y, c.z} - r.o;
    float Akz = comp(A, sh.kz), Bkz = comp(B, sh.kz), Ckz = comp(C, sh.kz);
    float Ax = fmaf(-sh.sx, Akz, comp(A, sh.kx)), Ay = fmaf(-sh.sy, Akz, comp(A, sh.ky));
    float Bx = fmaf(-sh.sx, Bkz, comp(B, sh.kx)), By = fmaf(-sh.sy, Bkz, comp(B, sh.ky));
    float Cx = fmaf(-sh.sx, Ckz, comp(C, sh.kx)), Cy = fmaf(-sh.sy, Ckz, comp(C, sh.ky));
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = U + V + W;
    if (det == 0.0f) return false;
    float T = fmaf(U, sh.sz * Akz, fmaf(V, sh.sz * Bkz, W * (sh.sz * Ckz)));
    float t = T * rcp(det);
    if (!(t > tmin)) return false;
    t_out = t;
    return true;
}

// Re-origin the ray at o (same direction): only the origin terms change.
__device__ __forceinline__ void set_origin(Ray &r, V3 o) {
    r.o = o;
    r.oi = V3{o.x * r.inv.x, o.y * r.inv.y, o.z * r.inv.z};
}

// This lane's traversal stack in a block's LDS (layout at kStackRow).
__device__ __forceinline__ uint32_t *lane_stack(uint32_t *lds) {
    return lds + (threadIdx.x >> 6) * (kStackDepth * kStackRow) + (threadIdx.x & 63);
}

// Closest triangle along (ow, dw) with t < h.t, through the two-level BVH4.
// stk is this lane's stack (lane_stack); sp is the word offset of its next
// free entry, depth x kStackRow.
__device__ __forceinline__ void traverse(const DevScene &S, const Ray &world, Hit &h, uint32_t *stk) {
    const V3 ow = world.o, dw = world.d;
    Ray r = world;
    int inst = -1;
    bool moved = false;   // current frame rotated/scaled (a parametrised segment)
    int sp = 0;
    constexpr int kEnd = kStackDepth * kStackRow;
    uint32_t ref = S.top_root;
    const float tmin = S.t_min;
    while (true) {
        if (!(ref & kLeafBit)) {
            work(kWorkNodes);
            // near/far planes per axis follow the direction signs; 32-bit byte
            // offsets from the uniform base keep the address arithmetic scalar
            const char *nb = reinterpret_cast<const char *>(S.nodes);
            const uint32_t off = ref << 7;
            const float4 nx = *reinterpret_cast<const float4 *>(nb + (off + (r.inv.x >= 0.0f ? 0u : 16u)));
            const float4 fx = *reinterpret_cast<const float4 *>(nb + (off + (r.inv.x >= 0.0f ? 16u : 0u)));
            const float4 ny = *reinterpret_cast<const float4 *>(nb + (off + (r.inv.y >= 0.0f ? 32u : 48u)));
            const float4 fy = *reinterpret_cast<const float4 *>(nb + (off + (r.inv.y >= 0.0f ? 48u : 32u)));
            const float4 nz = *reinterpret_cast<const float4 *>(nb + (off + (r.inv.z >= 0.0f ? 64u : 80u)));
            const float4 fz = *reinterpret_cast<const float4 *>(nb + (off + (r.inv.z >= 0.0f ? 80u : 64u)));
            const uint4 ch = *reinterpret_cast<const uint4 *>(nb + (off + 96u));
            const float tmax = h.t;
            // keys: distance bits with the child slot in the two lowest mantissa bits
            // (non-negative floats order like unsigned integers; a miss is +inf)
            uint32_t k0 = (__float_as_uint(child_key(r, nx.x, ny.x, nz.x, fx.x, fy.x, fz.x, tmax)) & ~3u) | 0u;
            uint32_t k1 = (__float_as_uint(child_key(r, nx.y, ny.y, nz.y, fx.y, fy.y, fz.y, tmax)) & ~3u) | 1u;
            uint32_t k2 = (__float_as_uint(child_key(r, nx.z, ny.z, nz.z, fx.z, fy.z, fz.z, tmax)) & ~3u) | 2u;
            uint32_t k3 = (__float_as_uint(child_key(r, nx.w, ny.w, nz.w, fx.w, fy.w, fz.w, tmax)) & ~3u) | 3u;
            // 4-element sorting network, branch-free
            uint32_t t;
            t = min(k0, k1); k1 = max(k0, k1); k0 = t;
            t = min(k2, k3); k3 = max(k2, k3); k2 = t;
            t = min(k0, k2); k2 = max(k0, k2); k0 = t;
            t = min(k1, k3); k3 = max(k1, k3); k1 = t;
            t = min(k1, k2); k2 = max(k1, k2); k1 = t;
            const uint32_t kMiss = 0x7F800000u;   // +inf
            if (k0 >= kMiss) {
                if (sp == 0) break;
                sp -= kStackRow;
                ref = stk[sp];
                continue;
            }
            // child of a key by its slot bits, with selects only (children of
            // empty slots never pass the slab test: their boxes are inverted)
            auto pick = [&](uint32_t k) -> uint32_t {
                const uint32_t lo = (k & 1u) ? ch.y : ch.x;
                const uint32_t hi = (k & 1u) ? ch.w : ch.z;
                return (k & 2u) ? hi : lo;
            };
            // the hit children after the nearest go on the stack, farthest
            // deepest; the keys are sorted, so k3 hit implies k2 and k1 hit
            uint32_t p2 = k2 < kMiss, p3 = k3 < kMiss;
            int need = (k1 < kMiss) + (int)p2 + (int)p3;
            if (sp + need * kStackRow > kEnd) {
                atomicOr(S.status, 2u);  // RICH_FLAG_STACK_OVERFLOW: the farthest are dropped
                need = (kEnd - sp) / kStackRow;
                p3 = need >= 3;
                p2 = need >= 2;
            }
            if (need > 0) {
                // the entries land in slots 0..need-1 above the top: a write to
                // a slot that a later write also takes is overwritten by it
                stk[sp] = pick(k3);
                stk[sp + (int)p3 * kStackRow] = pick(k2);
                stk[sp + (int)(p2 + p3) * kStackRow] = pick(k1);
                sp += need * kStackRow;
            }
            ref = pick(k0);
            continue;
        }
        if (ref == kExitMarker) {
            if (moved) ray_setup(r, ow, dw);
            else set_origin(r, ow);
            inst = -1;
            moved = false;
        } else if (ref & kInstBit) {
            int k = (int)(ref & ~(kLeafBit | kInstBit));
            if (sp == kEnd) {
                atomicOr(S.status, 2u);
            } else {
                stk[sp] = kExitMarker;
                sp += kStackRow;
                work(kWorkInstances);
                const Instance &in = S.inst[k];
                if (in.segment < 0) {
                    set_origin(r, ow - ld3(in.org));   // fixed instances only translate
                } else {
                    work(kWorkMovingInstances);
                    ray_setup(r, mat3(in.m, ow - ld3(in.org)), mat3(in.m, dw));
                    moved = true;
                }
                inst = k;
                ref = in.root;
                continue;
            }
        } else {
            uint32_t first = ref & 0x07FFFFFFu;
            uint32_t cnt = ((ref >> 27) & 7u) + 1u;
            work(kWorkLeaves);
            const Shear sh = make_shear(r.d);
            for (uint32_t q = first; q < first + cnt; ++q) {
                work(kWorkTris);
                const char *tb = reinterpret_cast<const char *>(S.tris) + (q << 6);
                float4 a = *reinterpret_cast<const float4 *>(tb);
                float4 b = *reinterpret_cast<const float4 *>(tb + 16);
                float4 c = *reinterpret_cast<const float4 *>(tb + 32);
                float t;
                if (hit_tri(r, sh, a, b, c, tmin, t)) {
                    uint32_t prim = S.prim_tri + __float_as_uint(a.w);
                    if (better(t, prim, h)) {
                        h.t = t;
                        h.prim = prim;
                        h.tri = q;
                        h.inst = inst;
                    }
                }
            }
        }
        if (sp == 0) break;
        sp -= kStackRow;
        ref = stk[sp];
    }
}

template <class D>
__device__ __forceinline__ void closest_hit(const DevScene &S, const D &det, V3 o, V3 d, Hit &h, uint32_t *stk) {
    h.t = INFINITY;
    h.prim = 0xFFFFFFFFu;
    h.tri = 0;
    h.inst = -1;
    h.root = 0;
    const float tmin = S.t_min;
    Ray r;
    ray_setup(r, o, d);
    float t;
    for (int i = 0; i < S.n_caps; ++i) {
        const RICH_CONST CapDev &cp = cref(S.caps[i]);
        work(kWorkCapBoxes);
        if (slab_entry(r, cp.lo[0], cp.lo[1], cp.lo[2], cp.hi[0], cp.hi[1], cp.hi[2], h.t) == INFINITY) continue;
        work(kWorkCaps);
        int root;
        if (hit_cap(cp, o, d, tmin, t, root) && better(t, (uint32_t)i, h)) {
            h.t = t;
            h.prim = (uint32_t)i;
            h.root = root;
        }
    }
    for (int i = 0; i < S.n_rects; ++i) {
        const RICH_CONST RectDev &rc = cref(S.rects[i]);
        work(kWorkRects);
        if (hit_plane_rect(ld3(rc.c), ld3(rc.n), ld3(rc.u), ld3(rc.v), rc.hu, rc.hv, o, d, tmin, t) &&
            better(t, (uint32_t)(S.n_caps + i), h)) {
            h.t = t;
            h.prim = (uint32_t)(S.n_caps + i);
        }
    }
    if (hit_plane_rect(ld3(det.c), ld3(det.n), ld3(det.u), ld3(det.v), det.hu, det.hv, o, d, tmin, t) &&
        better(t, S.prim_det, h)) {
        h.t = t;
        h.prim = S.prim_det;
    }
    if (S.has_box) work(kWorkBoxes);
    if (S.has_box && hit_box(S.box_lo, S.box_hi, r, tmin, t) && better(t, S.prim_box, h)) {
        h.t = t;
        h.prim = S.prim_box;
    }
    if (S.has_mesh) traverse(S, r, h, stk);
}

// Reflectivity of material `mat` at `lambda`.  The loop over materials is
// uniform so every table is read through scalar loads; lanes select their own.
__device__ __forceinline__ float reflectivity(const DevScene &S, int mat, float lambda) {
    float v = 0.0f;
    for (int m = 0; m < S.n_mats; ++m) {
        const RICH_CONST MatDev &M = cref(S.mats[m]);
        if (M.kind != 0) continue;
        float r = lerp_table(M.n, M.x, M.y, M.s, lambda);
        v = (mat == m) ? r : v;
    }
    return v;
}

// ---------------------------------------------------------------- interaction

constexpr int kDetected = 0, kQeRejected = 1, kAbsorbedMirror = 2, kAbsorbed = 3, kEscaped = 4, kMaxBounces = 5;

struct PathEnd {
    int fate;
    int pixel;
    V3 P;
    float u, v;
    float time;     // arrival time at the detector hit (ns)
};

// Receives every reflection and the detector hit; the forward kernels ignore them.
struct NoRecord {
    __device__ __forceinline__ void reflect(int b, const Hit &h, V3 o, V3 d, V3 P, V3 n) {}
    __device__ __forceinline__ void detect(int b, V3 o, V3 d, float t) {}
};

__device__ __forceinline__ V3 surface_normal(const DevScene &S, const Hit &h, V3 P, int &mat) {
    if (h.prim < (uint32_t)S.n_caps) {
        const CapDev &cp = S.caps[h.prim];
        mat = cp.material;
        return rcp(cp.R) * (ld3(cp.C) - P);
    }
    if (h.prim < S.prim_det) {
        const RectDev &rc = S.rects[h.prim - S.n_caps];
        mat = rc.material;
        return ld3(rc.n);
    }
    const Tri &tr = S.tris[h.tri];
    mat = (int)tr.material;
    V3 n = ld3(tr.n);
    if (h.inst >= 0 && S.inst[h.inst].segment >= 0) n = mat3(S.inst[h.inst].rot, n);
    return n;
}

constexpr int kPrefiltered = 6;

// Pre-propagation efficiency filter: keep the photon with probability
// QE(lambda) * prod_k refl_k(lambda), as one accept-reject per photon.
template <class D>
__device__ __forceinline__ bool prefilter_keep(const DevScene &S, const D &det, const DevSource &src,
                                               const Photon &ph, uint64_t seed, uint64_t g) {
    float p = lerp_table(det.n_qe, det.qe_x, det.qe_y, det.qe_s, ph.lambda);
    for (int k = 0; k < src.pf_n; ++k) p *= reflectivity(S, src.pf_mats[k], ph.lambda);
    return u24(photon_block(seed, g, kPrefilterBlock).x) < p;
}

// Trace one photon.  With `efficiencies` false (photons kept by the
// pre-filter) mirrors always reflect and the detector always detects.
template <class D, class Rec>
__device__ __forceinline__ void propagate(const DevScene &S, const D &det, const Photon &ph, uint64_t seed,
                                          uint64_t g, uint32_t *stk, PathEnd &end, Rec &rec,
                                          bool efficiencies = true) {
    V3 o = ph.o, d = ph.d;
    end.fate = kMaxBounces;
    end.pixel = -1;
    // a track below the Cherenkov threshold has no cone (NaN direction): no light
    if (!(fabsf(d.x) <= 1.0f && fabsf(d.y) <= 1.0f && fabsf(d.z) <= 1.0f)) {
        end.fate = kEscaped;
        return;
    }
    uint4 blk = make_uint4(0, 0, 0, 0);
    int have = -1;
    float clock = ph.t0;        // time at the start of the current segment (ns)
    work(kWorkPhotons);
    for (int b = 0; b < S.max_bounces; ++b) {
        Hit h;
        work(kWorkQueries);
        closest_hit(S, det, o, d, h, stk);
        if (h.prim == 0xFFFFFFFFu) {
            end.fate = kEscaped;
            break;
        }
        if (h.prim == S.prim_det) {
            if (dot(d, ld3(det.n)) >= 0.0f) {
                end.fate = kAbsorbed;
                break;
            }
            V3 Pc = fma3(h.t, d, o - ld3(det.c));
            float u = dot(Pc, ld3(det.u)), v = dot(Pc, ld3(det.v));
            float fi = floorf((u + det.act_hu) * det.inv_pitch), fj = floorf((v + det.act_hv) * det.inv_pitch);
            if (!(fi >= 0.0f && fi < (float)det.nx && fj >= 0.0f && fj < (float)det.ny)) {  // NaN-safe
                end.fate = kAbsorbed;
                break;
            }
            end.pixel = (int)fj * det.nx + (int)fi;
            end.P = fma3(h.t, d, o);
            end.u = u;
            end.v = v;
            end.time = fmaf(h.t, ph.ng_c, clock);
            work(kWorkDetections);
            rec.detect(b, o, d, h.t);
            if (efficiencies) {
                float qe = lerp_table(det.n_qe, det.qe_x, det.qe_y, det.qe_s, ph.lambda);
                end.fate = ph.u_qe < qe ? kDetected : kQeRejected;
            } else {
                end.fate = kDetected;
            }
            break;
        }
        if (h.prim == S.prim_box) {
            end.fate = kAbsorbed;
            break;
        }
        V3 P = fma3(h.t, d, o);
        int mat;
        V3 n = surface_normal(S, h, P, mat);
        if (S.mats[mat].kind != 0 || dot(d, n) >= 0.0f) {
            end.fate = kAbsorbed;
            break;
        }
        if (efficiencies) {
            int bid = 1 + (b >> 2);
            if (have != bid) {
                blk = photon_block(seed, g, (uint32_t)bid);
                have = bid;
            }
            int w = b & 3;
            uint32_t word = w == 0 ? blk.x : (w == 1 ? blk.y : (w == 2 ? blk.z : blk.w));
            float refl = reflectivity(S, mat, ph.lambda);
            if (u24(word) >= refl) {
                end.fate = kAbsorbedMirror;
                break;
            }
        }
        work(kWorkReflections);
        rec.reflect(b, h, o, d, P, n);
        clock = fmaf(h.t, ph.ng_c, clock);
        V3 dr = fma3(-2.0f * dot(d, n), n, d);
        d = rsqrtf(dot(dr, dr)) * dr;
        o = P;
    }
}

}  // namespace rich
