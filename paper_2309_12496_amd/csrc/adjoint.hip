// Reverse-mode derivative of detector hit coordinates with respect to the
// mirror-segment parameters (tilt_x, tilt_y, R, dx, dy, dz).
//
// Each lane recomputes its photon's path with the forward device functions,
// keeping the reflections in registers, then sweeps back from the detector:
//   detector plane  P' = o + t d, t = ((c - o).n)/(d.n):
//                   g_o = g_P' - n (d.g_P')/(d.n),  g_d = t g_o
//   reflection      d' = d - 2 (d.n) n:
//                   g_d += g_d' - 2 n (n.g_d'),   g_n = -2 [(g_d'.n) d + (d.n) g_d']
//   sphere cap      |P - C| = R, n = (C - P)/R, w = P - C, s = (g_P.d)/(w.d):
//                   g_C = g_n/R + s w, g_R = -(g_n.n)/R + s R, g_o = g_P - g_n/R - s w
//   moving facet    plane through q with normal n, s = (g_P.d)/(n.d):
//                   g_q = s n, g_n += s (q - P), g_o = g_P - s n
// and maps g_C, g_R or g_q, g_n onto the six parameters of the segment.
// Visibility changes at edges are ignored (interior derivative).
//
// Work distribution.  Masks usually keep a few percent of the photons, in
// clumps (the tracks that light the detector).  Two small kernels first count
// the masked ids of every chunk of 4096 ids and scan the counts, so that the
// masked photons have ranks 0..M-1 in id order.  A persistent grid (every
// block resident at once) then takes consecutive ranks: whole rounds of groups
// of 256, one per wave and round, then the rest in groups of 256, 128 or 64
// dealt round robin, the size that loads the busiest wave least; every pass
// but the last is full.  A group of 128 or 256 is sorted by cone azimuth (a
// counting sort in lane order) and traced in passes of 64, so that each pass
// holds neighbouring rays, as the forward launch sorts its photons.
//
// Sums are deterministic: groups map statically to waves and the regrouping
// order is fixed; per segment the wave reduces with a butterfly and lane 0
// adds into wave-private LDS accumulators; blocks then sum their waves in
// order, and a final kernel sums the blocks in order.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"
#include "trace.h"

namespace rich {

// Block partial sums of rich_propagate_adjoint_noalloc.  In host code the
// name stands for a host-side shadow: kernels get the device address that
// adjoint_scratch looks up, never this name.
__device__ __align__(256) float scratch[kAdjScratchFloats];

namespace {

constexpr int kAdjBlock = 256;
constexpr uint32_t kMaskChunk = 4096;  // ids per chunk of the mask count
constexpr int kGroup = 256;            // ranks of a regrouped group: four passes
constexpr uint64_t kSegment = 1ull << 32;   // ids per launch: group lists hold 32-bit ids
constexpr int kMaxRefl = 4;
// Kind of surface a reflection meets, in the top two bits of its record's code.
constexpr uint32_t kKindCap = 0u, kKindRect = 1u, kKindStaticTri = 2u, kKindFacet = 3u;
constexpr uint32_t kIndexMask = 0x3FFFFFFFu;

// What the adjoint keeps of each reflection while the photon is traced: the
// hit distance, the surface (kind, and cap, rectangle or triangle index) and
// the instance of a triangle.  Three registers per reflection instead of the
// thirteen of point, direction and normal, which the reverse sweep rebuilds
// by replaying the reflections from the photon's start with the forward
// pass's arithmetic; the traversal, which needs the most registers, runs
// with fewer live.
struct PathRecorder {
    float t0 = 0.0f, t1 = 0.0f, t2 = 0.0f, t3 = 0.0f;
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    int32_t i0 = -1, i1 = -1, i2 = -1, i3 = -1;
    int n = 0;
    bool overflow = false;
    bool hit_det = false;
    float det_t = 0.0f;
    uint32_t n_caps = 0, prim_det = 0;
    const Instance *inst = nullptr;

    __device__ __forceinline__ void reflect(int b, const Hit &h, V3 o, V3 d, V3 P, V3 nrm) {
        uint32_t code;
        if (h.prim < n_caps) {
            code = (kKindCap << 30) | h.prim;
        } else if (h.prim < prim_det) {
            code = (kKindRect << 30) | (h.prim - n_caps);
        } else if (h.inst < 0 || inst[h.inst].segment < 0) {
            code = (kKindStaticTri << 30) | h.tri;
        } else {
            code = (kKindFacet << 30) | h.tri;
        }
        switch (n) {
            case 0: t0 = h.t; c0 = code; i0 = h.inst; break;
            case 1: t1 = h.t; c1 = code; i1 = h.inst; break;
            case 2: t2 = h.t; c2 = code; i2 = h.inst; break;
            case 3: t3 = h.t; c3 = code; i3 = h.inst; break;
            default: overflow = true; break;
        }
        ++n;
    }
    __device__ __forceinline__ void detect(int b, V3 o, V3 d, float t) {
        hit_det = true;
        det_t = t;
    }
    __device__ __forceinline__ float t(int k) const { return k == 0 ? t0 : (k == 1 ? t1 : (k == 2 ? t2 : t3)); }
    __device__ __forceinline__ uint32_t code(int k) const {
        return k == 0 ? c0 : (k == 1 ? c1 : (k == 2 ? c2 : c3));
    }
    __device__ __forceinline__ int32_t instance(int k) const {
        return k == 0 ? i0 : (k == 1 ? i1 : (k == 2 ? i2 : i3));
    }
};

// Unit normal of a recorded reflection at P, as the forward pass forms it.
__device__ __forceinline__ V3 recorded_normal(const DevScene &S, uint32_t code, int32_t inst, V3 P) {
    const uint32_t kind = code >> 30, idx = code & kIndexMask;
    if (kind == kKindCap) {
        const CapDev &cp = S.caps[idx];
        return rcp(cp.R) * (ld3(cp.C) - P);
    }
    if (kind == kKindRect) return ld3(S.rects[idx].n);
    V3 n = ld3(S.tris[idx].n);
    if (kind == kKindFacet) n = mat3(S.inst[inst].rot, n);
    return n;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Add each lane's 6 values into acc[seg*6 + j], segment by segment, in a fixed order.
__device__ __forceinline__ void wave_accumulate(float *acc, int seg, const float g[6]) {
    const int lane = __lane_id();
    while (true) {
        unsigned long long m = __ballot(seg >= 0);
        if (m == 0ull) break;
        int leader = __ffsll((long long)m) - 1;
        int s = __shfl(seg, leader);
        bool mine = seg == s;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            float v = wave_sum(mine ? g[j] : 0.0f);
            if (lane == 0) acc[6 * s + j] += v;
        }
        if (mine) seg = -1;
    }
}

__device__ __forceinline__ V3 plane_back(V3 gP, V3 d, V3 n) {
    float s = dot(gP, d) / dot(n, d);
    return fma3(-s, n, gP);
}

// Bit 7 of each byte set where the byte of w is nonzero.
__device__ __forceinline__ uint32_t nonzero_high_bits(uint32_t w) {
    return (((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) & 0x80808080u;
}

__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t w) { return __popc(nonzero_high_bits(w)); }

// Bit t set where byte t of the lane's 64 mask bytes (16 words) is nonzero.
__device__ __forceinline__ uint64_t nonzero_bitmap(const uint32_t w[16]) {
    uint64_t m = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint32_t h = nonzero_high_bits(w[q]);   // bits 7, 15, 23, 31
        const uint32_t nib = ((h >> 7) & 1u) | ((h >> 14) & 2u) | ((h >> 21) & 4u) | ((h >> 28) & 8u);
        m |= (uint64_t)nib << (4 * q);
    }
    return m;
}

// This lane's 64 mask bytes [b, b + 64) as 16 words (bytes at or beyond n
// read as zero): four 16-byte loads when they lie inside [0, n) and the mask
// is 16-byte aligned, else bytes.
__device__ __forceinline__ void load_mask64(const uint8_t *mask, uint64_t b, uint64_t n, uint32_t w[16]) {
    if (b + 64 <= n && ((reinterpret_cast<uintptr_t>(mask) & 15u) == 0)) {
        const uint4 *p = reinterpret_cast<const uint4 *>(mask + b);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 v = p[q];
            w[4 * q] = v.x;
            w[4 * q + 1] = v.y;
            w[4 * q + 2] = v.z;
            w[4 * q + 3] = v.w;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) w[q] = 0u;
    for (int t = 0; t < 64 && b + t < n; ++t)
        if (mask[b + t]) w[t >> 2] |= 0xFFu << (8 * (t & 3));
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Exclusive prefix sum over the wave's lanes.
__device__ __forceinline__ uint32_t wave_exclusive_u32(uint32_t v) {
    const int lane = __lane_id();
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x - v;
}

}  // namespace

// Masked ids of each chunk of kMaskChunk ids: one wave per chunk.
__global__ __launch_bounds__(256) void mask_count_kernel(const uint8_t *mask, uint64_t n, uint64_t n_chunks,
                                                         uint32_t *counts) {
    const uint64_t k = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (k >= n_chunks) return;
    uint32_t w[16];
    load_mask64(mask, k * kMaskChunk + 64ull * (uint64_t)__lane_id(), n, w);
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) c += nonzero_bytes(w[q]);
    c = wave_sum_u32(c);
    if (__lane_id() == 0) counts[k] = c;
}

// Exclusive scan of the chunk counts into offsets[0..n_chunks] (offsets[n_chunks]
// = masked total), one block: each thread sums a contiguous slice, the block
// scans the slice sums, each thread writes its slice.
__global__ __launch_bounds__(1024) void mask_scan_kernel(const uint32_t *counts, uint64_t n_chunks,
                                                         unsigned long long *offsets) {
    __shared__ unsigned long long part[1024];
    const uint64_t t = threadIdx.x;
    const uint64_t per = (n_chunks + 1023) / 1024;
    const uint64_t lo = t * per < n_chunks ? t * per : n_chunks;
    const uint64_t hi = lo + per < n_chunks ? lo + per : n_chunks;
    unsigned long long sum = 0;
#pragma unroll 8
    for (uint64_t j = lo; j < hi; ++j) sum += counts[j];   // unrolled: the loads overlap
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        unsigned long long y = t >= (uint64_t)off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    unsigned long long run = part[t] - sum;
#pragma unroll 8
    for (uint64_t j = lo; j < hi; ++j) {
        offsets[j] = run;
        run += counts[j];
    }
    if (t == 1023) offsets[n_chunks] = part[1023];
}

namespace {

// Largest chunk k < n_chunks with offsets[k] <= r (offsets[0] = 0 <= r):
// a 64-way search, one probe per lane and round.
__device__ __forceinline__ uint64_t find_chunk(const unsigned long long *offsets, uint64_t n_chunks, uint64_t r) {
    uint64_t lo = 0, hi = n_chunks;
    const uint64_t lane = (uint64_t)__lane_id();
    while (hi - lo > 1) {
        const uint64_t step = (hi - lo + 63) / 64;
        const uint64_t idx = lo + lane * step;
        const unsigned long long m = __ballot(idx < hi && offsets[idx] <= r);
        const uint64_t last = 63 - __clzll((long long)m);
        lo += last * step;
        hi = lo + step < hi ? lo + step : hi;
    }
    return lo;
}

// One pass of up to 64 photons (lanes with act set; i = id within the launch):
// retrace, sweep back, add into this wave's accumulators.
__device__ __forceinline__ void adjoint_pass(const DevScene &S, const DevSource &src, const AdjointArgs &a,
                                             const RICH_CONST DetDev &det, float cut2, uint32_t *stk, float *acc,
                                             bool act, uint64_t i, uint64_t first, uint64_t seed) {
    const int lane = __lane_id();
    PathRecorder rec;
    rec.n_caps = (uint32_t)S.n_caps;
    rec.prim_det = S.prim_det;
    rec.inst = S.inst;
    PathEnd end;
    end.fate = -1;
    float gu = 0.0f, gv = 0.0f, loss = 0.0f, cnt = 0.0f;
    V3 o0 = v3(0.0f, 0.0f, 0.0f), d0 = v3(0.0f, 0.0f, 1.0f);   // the photon's start, for the replay
    if (act) {
        uint64_t g = first + i;
        Photon ph = make_photon(src, seed, g, i, false);
        o0 = ph.o;
        d0 = ph.d;
        if (!src.prefilter) {
            propagate(S, det, ph, seed, g, stk, end, rec);
        } else if (prefilter_keep(S, det, src, ph, seed, g)) {
            propagate(S, det, ph, seed, g, stk, end, rec, false);
        } else {
            end.fate = kPrefiltered;
        }
        act = rec.hit_det && (end.fate == kDetected || end.fate == kQeRejected);
        if (act && rec.overflow) {
            atomicOr(S.status, 4u);  // RICH_FLAG_PATH_OVERFLOW
            act = false;
        }
    }
    if (act) {
        if (a.targets) {
            float du = end.u - a.targets[2 * i], dv = end.v - a.targets[2 * i + 1];
            float r2 = du * du + dv * dv;
            act = r2 <= cut2;
            gu = 2.0f * du;
            gv = 2.0f * dv;
            loss = act ? r2 : 0.0f;
        } else {
            gu = a.grad_uv[2 * i];
            gv = a.grad_uv[2 * i + 1];
        }
        cnt = act ? 1.0f : 0.0f;
    }
    // replay the reflections: point, incoming direction and normal of each
    V3 RP[kMaxRefl], RD[kMaxRefl], RN[kMaxRefl];
    {
        V3 o = o0, d = d0;
#pragma unroll
        for (int k = 0; k < kMaxRefl; ++k) {
            RP[k] = o;
            RD[k] = d;
            RN[k] = d;
            if (act && k < rec.n) {
                const V3 P = fma3(rec.t(k), d, o);
                const V3 nr = recorded_normal(S, rec.code(k), rec.instance(k), P);
                RP[k] = P;
                RN[k] = nr;
                const V3 dr = fma3(-2.0f * dot(d, nr), nr, d);
                d = rsqrtf(dot(dr, dr)) * dr;
                o = P;
            }
        }
        d0 = d;   // the direction the photon reaches the detector with
    }
    // detector plane
    V3 gP = v3(0.0f, 0.0f, 0.0f), gD = v3(0.0f, 0.0f, 0.0f);
    if (act) {
        work(kWorkBackDetector);
        V3 gPd = fma3(gu, ld3(det.u), gv * ld3(det.v));
        gP = plane_back(gPd, d0, ld3(det.n));
        gD = rec.det_t * gP;
    }
    // reflections, last to first (uniform loop so the wave reductions stay converged)
#pragma unroll
    for (int k = kMaxRefl - 1; k >= 0; --k) {
        int seg = -1;
        float gp[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (act && k < rec.n) {
            const V3 xP = RP[k], xd = RD[k], xn = RN[k];
            const float xt = rec.t(k);
            const uint32_t kind = rec.code(k) >> 30, idx = rec.code(k) & kIndexMask;
            float gdn = dot(gD, xn);
            float dn = dot(xd, xn);
            V3 h = -2.0f * fma3(gdn, xd, dn * gD);       // adjoint of the normal
            V3 gDin = fma3(-2.0f * gdn, xn, gD);
            V3 gO;
            if (kind == kKindCap) {
                work(kWorkBackCaps);
                const CapDev &cp = S.caps[idx];
                float invR = 1.0f / cp.R;
                V3 w = xP - ld3(cp.C);
                V3 gPt = fma3(-invR, h, gP);
                float s = dot(gPt, xd) / dot(w, xd);
                gO = fma3(-s, w, gPt);
                V3 gC = fma3(s, w, invR * h);
                float gR = fmaf(s, cp.R, -dot(h, xn) * invR);
                seg = cp.segment;
                gp[0] = dot(gC, ld3(cp.dCdtx));
                gp[1] = dot(gC, ld3(cp.dCdty));
                gp[2] = gR + dot(gC, ld3(cp.axis));
                gp[3] = gC.x;
                gp[4] = gC.y;
                gp[5] = gC.z;
            } else if (kind == kKindFacet) {
                work(kWorkBackFacets);
                const Instance &in = S.inst[rec.instance(k)];
                const Tri &tr = S.tris[idx];
                V3 vl = ld3(tr.v0), nl = ld3(tr.n);
                V3 rv = mat3(in.rot, vl);
                V3 q = fma3(in.scale, rv, ld3(in.org));
                float s = dot(gP, xd) / dot(xn, xd);
                gO = fma3(-s, xn, gP);
                V3 gq = s * xn;
                V3 gn = fma3(s, q - xP, h);
                seg = in.segment;
                gp[0] = in.scale * dot(gq, mat3(in.drx, vl)) + dot(gn, mat3(in.drx, nl));
                gp[1] = in.scale * dot(gq, mat3(in.dry, vl)) + dot(gn, mat3(in.dry, nl));
                gp[2] = dot(gq, rv) * in.inv_r0;
                gp[3] = gq.x;
                gp[4] = gq.y;
                gp[5] = gq.z;
            } else {
                work(kWorkBackPlanes);
                gO = plane_back(gP, xd, xn);
            }
            gP = gO;
            gD = fma3(xt, gO, gDin);
        }
        wave_accumulate(acc, seg, gp);
    }
    float wl = wave_sum(loss), wc = wave_sum(cnt);
    if (lane == 0) {
        acc[a.n_par] += wl;
        acc[a.n_par + 1] += wc;
    }
}

}  // namespace

// Held to 3 waves per SIMD (160 VGPRs, no spills); at 4 the traversal spills.
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(3))) void adjoint_kernel(
    DevScene S, DevSource src, AdjointArgs a, uint64_t n,
                                                            uint64_t first, uint64_t seed, uint64_t n_chunks,
                                                            uint32_t row0) {
    extern __shared__ uint32_t lds[];
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const int width = a.n_par + 2;
    uint32_t *stk = lane_stack(lds);
    float *acc_all = reinterpret_cast<float *>(lds + (size_t)blockDim.x * kStackDepth);
    float *acc = acc_all + wave * width;
    for (int j = lane; j < width; j += 64) acc[j] = 0.0f;
    // While no photon is traced the wave's own stack columns hold its group:
    // rows 0-3 the ids in rank order, rows 4-7 the regrouped ids, row 8 the
    // running offsets of the 64 azimuth bins.
    uint32_t *const wave_rows = lds + wave * (kStackDepth * kStackRow);
    auto cell = [&](int j) -> uint32_t & { return wave_rows[j]; };

    const RICH_CONST DetDev &det = cref(*S.det);
    // Squared residual cut; a negative or NaN cut admits no photon.
    float cut2 = __builtin_inff();
    if (a.residual_cut) {
        float c = *a.residual_cut;
        cut2 = c >= 0.0f ? c * c : -1.0f;
    }
    const uint64_t M = a.mask ? (uint64_t)a.chunk_offsets[n_chunks] : n;
    const uint64_t W = (uint64_t)gridDim.x * waves;
    const uint64_t wid = (uint64_t)blockIdx.x * waves + wave;
    // Every wave takes the same number of whole rounds of regrouped groups of
    // 256 ranks (group round * W + wid).  The ranks left after the last whole
    // round go out in groups of 256, 128 or 64, group q to wave q mod W: the
    // size with the fewest passes on the busiest wave, the larger on a tie
    // (larger groups are regrouped into more coherent passes).
    const uint64_t big_rounds = M / ((uint64_t)kGroup * W);
    const uint64_t tail = big_rounds * (uint64_t)kGroup * W;
    uint64_t tail_gs = 64, tail_groups = (M - tail + 63) / 64;
    uint64_t best = (tail_groups + W - 1) / W;   // passes on the busiest wave
    for (uint64_t gsz = 128; gsz <= (uint64_t)kGroup; gsz *= 2) {
        const uint64_t groups = (M - tail + gsz - 1) / gsz;
        const uint64_t passes = (groups + W - 1) / W * (gsz / 64);
        if (passes <= best) {
            best = passes;
            tail_gs = gsz;
            tail_groups = groups;
        }
    }
    const uint64_t n_tasks = big_rounds + (tail_groups + W - 1 - wid) / W;
    for (uint64_t task = 0; task < n_tasks; ++task) {
        const bool in_rounds = task < big_rounds;
        const uint64_t gs = in_rounds ? (uint64_t)kGroup : tail_gs;
        const uint64_t r0 = in_rounds ? (task * W + wid) * (uint64_t)kGroup
                                      : tail + ((task - big_rounds) * W + wid) * tail_gs;
        const int cnt = (int)(M - r0 < gs ? M - r0 : gs);
        const bool big = gs > 64;   // regrouped
        // ids of ranks r0 .. r0 + cnt - 1 into rows 0-3
        if (!a.mask) {
            for (int j = lane; j < cnt; j += 64) cell(j) = (uint32_t)(r0 + (uint64_t)j);
        } else {
            uint64_t k = find_chunk(a.chunk_offsets, n_chunks, r0);
            uint64_t filled = 0;
            while (filled < (uint64_t)cnt) {
                const uint64_t first_rank = a.chunk_offsets[k], end_rank = a.chunk_offsets[k + 1];
                if (end_rank > r0 + filled) {
                    const uint64_t b = k * kMaskChunk + 64ull * (uint64_t)lane;
                    uint32_t w[16];
                    load_mask64(a.mask, b, n, w);
                    uint64_t bits = nonzero_bitmap(w);
                    const uint32_t c = (uint32_t)__popcll(bits);
                    uint64_t rank = first_rank + wave_exclusive_u32(c);
                    if (c > 0 && rank < r0 + (uint64_t)cnt && rank + c > r0) {
                        while (bits) {
                            const int t = __ffsll((long long)bits) - 1;
                            bits &= bits - 1;
                            if (rank >= r0 && rank < r0 + (uint64_t)cnt) cell((int)(rank - r0)) = (uint32_t)(b + t);
                            ++rank;
                        }
                    }
                }
                filled = end_rank - r0 < (uint64_t)cnt ? end_rank - r0 : (uint64_t)cnt;
                ++k;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        int src_row = 0;
        if (big) {
            // counting sort by the azimuth's top 6 bits (Philox block 0, word 0),
            // equal bins in (round, lane) order
            uint32_t id[4], bin[4];
            cell(512 + lane) = 0u;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = 64 * q + lane;
                id[q] = 0u;
                bin[q] = 64u;
                if (j < cnt) {
                    id[q] = cell(j);
                    work(kWorkSortKeys);
                    bin[q] = photon_block(seed, first + id[q], 0).x >> 26;
                    atomicAdd(&cell(512 + (int)bin[q]), 1u);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            const uint32_t nb = cell(512 + lane);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            cell(512 + lane) = wave_exclusive_u32(nb);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            const unsigned long long below_mask = (1ull << lane) - 1ull;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool valid = 64 * q + lane < cnt;
                unsigned long long same = __ballot(valid);
#pragma unroll
                for (int bit = 0; bit < 6; ++bit) {
                    const unsigned long long m = __ballot((bin[q] >> bit) & 1u);
                    same &= ((bin[q] >> bit) & 1u) ? m : ~m;
                }
                const uint32_t below = (uint32_t)__popcll(same & below_mask);
                if (valid) cell(256 + (int)(cell(512 + (int)bin[q]) + below)) = id[q];
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if (valid && below == 0) cell(512 + (int)bin[q]) += (uint32_t)__popcll(same);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
            src_row = 4;
        }
        // the passes' ids into registers: the stack rows are needed for tracing
        uint32_t id0 = 0, id1 = 0, id2 = 0, id3 = 0;
        if (lane < cnt) id0 = cell(64 * src_row + lane);
        if (64 + lane < cnt) id1 = cell(64 * (src_row + 1) + lane);
        if (128 + lane < cnt) id2 = cell(64 * (src_row + 2) + lane);
        if (192 + lane < cnt) id3 = cell(64 * (src_row + 3) + lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int n_pass = (cnt + 63) / 64;
#pragma unroll 1
        for (int p = 0; p < n_pass; ++p) {
            const uint32_t i = p == 0 ? id0 : (p == 1 ? id1 : (p == 2 ? id2 : id3));
            adjoint_pass(S, src, a, det, cut2, stk, acc, 64 * p + lane < cnt, (uint64_t)i, first, seed);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    __syncthreads();
    for (int j = threadIdx.x; j < width; j += blockDim.x) {
        float s = 0.0f;
        for (int w = 0; w < waves; ++w) s += acc_all[w * width + j];
        a.partials[((size_t)row0 + blockIdx.x) * width + j] = s;
    }
}

// Fixed-order sum of column j of the block partials: thread t adds blocks
// t, t+256, ... in order, then an LDS tree of fixed shape combines the threads.
__device__ __forceinline__ float column_sum(const float *partials, int n_blocks, int width, int j, float *red) {
    float s = 0.0f;
    for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) s += partials[(size_t)b * width + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    float v = red[0];
    __syncthreads();
    return v;
}

// One block per output: gradient entries 0..n_par-1 and the loss (n_par).
// Every block recomputes the photon count the same way; fused-loss mode
// divides by it.
__global__ __launch_bounds__(256) void adjoint_reduce_kernel(const float *partials, int n_blocks, int n_par,
                                                             int fused, float *grad, float *loss) {
    __shared__ float red[256];
    const int width = n_par + 2;
    const int j = blockIdx.x;
    float v = column_sum(partials, n_blocks, width, j, red);
    float cnt = column_sum(partials, n_blocks, width, n_par + 1, red);
    float scale = fused ? (cnt > 0.0f ? 1.0f / cnt : 0.0f) : 1.0f;
    if (threadIdx.x == 0) {
        if (j < n_par) grad[j] = v * scale;
        else if (loss) *loss = v * scale;
    }
}

static size_t adjoint_lds_bytes(int n_par) {
    return (size_t)kAdjBlock * kStackDepth * sizeof(uint32_t) + (size_t)(kAdjBlock / 64) * (n_par + 2) * sizeof(float);
}

AdjointPlan adjoint_plan(uint64_t n, int n_par, int n_cu, bool masked) {
    AdjointPlan p{};
    const uint64_t seg = n < kSegment ? n : kSegment;
    p.n_segments = n > kSegment ? (int)((n + kSegment - 1) / kSegment) : 1;
    // a persistent grid: as many blocks as the compute units hold at once
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, adjoint_kernel, kAdjBlock, adjoint_lds_bytes(n_par)) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const uint64_t want = (seg + 1023) / 1024;   // a pass of 64 for each wave when every id counts
    const uint64_t cap = (uint64_t)(n_cu > 0 ? n_cu : 256) * (uint64_t)per_cu;
    p.n_blocks = (int)(want < 1 ? 1 : (want < cap ? want : cap));
    p.n_chunks = masked ? (seg + kMaskChunk - 1) / kMaskChunk : 0;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t bytes = up((size_t)p.n_segments * p.n_blocks * (size_t)(n_par + 2) * sizeof(float));
    p.counts_offset = bytes;
    if (masked) bytes = up(bytes + p.n_chunks * sizeof(uint32_t));
    p.offsets_offset = bytes;
    if (masked) bytes += (p.n_chunks + 1) * sizeof(unsigned long long);
    p.bytes = bytes;
    return p;
}

hipError_t launch_adjoint(const DevScene &S, const DevSource &src, const AdjointArgs &args, uint64_t n, uint64_t first,
                          uint64_t seed, const AdjointPlan &plan, void *work, hipStream_t st) {
    char *w = static_cast<char *>(work);
    const size_t lds = adjoint_lds_bytes(args.n_par);
    for (int s = 0; s < plan.n_segments; ++s) {
        const uint64_t base = (uint64_t)s * kSegment;
        const uint64_t ns = n - base < kSegment ? n - base : kSegment;
        AdjointArgs a = args;
        a.partials = reinterpret_cast<float *>(w);
        if (a.grad_uv) a.grad_uv += 2 * base;
        if (a.targets) a.targets += 2 * base;
        DevSource ds = src;
        if (ds.kind == 2) {
            ds.ex_o += 3 * base;
            ds.ex_d += 3 * base;
            ds.ex_l += base;
        }
        uint64_t n_chunks = 0;
        if (a.mask) {
            a.mask += base;
            a.chunk_counts = reinterpret_cast<uint32_t *>(w + plan.counts_offset);
            a.chunk_offsets = reinterpret_cast<const unsigned long long *>(w + plan.offsets_offset);
            n_chunks = (ns + kMaskChunk - 1) / kMaskChunk;
            if (n_chunks > 0) {
                hipLaunchKernelGGL(mask_count_kernel, dim3((unsigned)((n_chunks + 3) / 4)), dim3(256), 0, st, a.mask, ns,
                                   n_chunks, a.chunk_counts);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(mask_scan_kernel, dim3(1), dim3(1024), 0, st, (const uint32_t *)a.chunk_counts, n_chunks,
                               const_cast<unsigned long long *>(a.chunk_offsets));
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(adjoint_kernel, dim3(plan.n_blocks), dim3(kAdjBlock), lds, st, S, ds, a, ns, first + base,
                           seed, n_chunks, (uint32_t)(s * plan.n_blocks));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(adjoint_reduce_kernel, dim3(args.n_par + 1), dim3(256), 0, st,
                       (const float *)reinterpret_cast<float *>(w), plan.n_segments * plan.n_blocks, args.n_par,
                       args.targets ? 1 : 0, args.grad, args.loss);
    return hipGetLastError();
}

hipError_t adjoint_scratch(int device, float **ptr) {
    static std::mutex mu;
    static float *addr[kAdjScratchDevices] = {};
    if (device < 0 || device >= kAdjScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = static_cast<float *>(p);
    }
    *ptr = addr[device];
    return hipSuccess;
}


}  // namespace rich

#ifdef RICH_WORK_COUNTERS
// Measurement build only: the adjoint kernel's work counters (this file's
// copy), as rich_work_counters gives the forward and batch kernels'.
extern "C" int rich_work_counters_adjoint(unsigned long long *out, int reset) {
    unsigned long long raw[16 * rich::kWorkUnits];
    if (hipDeviceSynchronize() != hipSuccess) return -3;
    if (hipMemcpyFromSymbol(raw, HIP_SYMBOL(rich::rich_work), sizeof raw) != hipSuccess) return -3;
    for (int u = 0; u < rich::kWorkUnits; ++u) {
        out[u] = raw[16 * u];
        out[rich::kWorkUnits + u] = raw[16 * u + 1];
    }
    if (reset) {
        unsigned long long zero[16 * rich::kWorkUnits] = {};
        if (hipMemcpyToSymbol(HIP_SYMBOL(rich::rich_work), zero, sizeof zero) != hipSuccess) return -3;
    }
    return 0;
}
#endif
