// librich kernels for gfx950: parameter refresh, forward propagation (one
// photon per lane), the persistent batch kernel, and small helpers.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "trace.h"

namespace rich {

// ---------------------------------------------------------------- parameters (FP64)

namespace {

struct D3 {
    double x, y, z;
};
__device__ inline D3 dload(const double *p) { return D3{p[0], p[1], p[2]}; }
__device__ inline D3 dadd(D3 a, D3 b) { return D3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline D3 dsub(D3 a, D3 b) { return D3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline D3 dmul(D3 a, double s) { return D3{a.x * s, a.y * s, a.z * s}; }
__device__ inline double ddot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline D3 dcross(D3 a, D3 b) {
    return D3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// rotation of v about unit axis k by angle th (Rodrigues)
__device__ inline D3 drot(D3 k, double th, D3 v) {
    double c = cos(th), s = sin(th);
    return dadd(dadd(dmul(v, c), dmul(dcross(k, v), s)), dmul(k, ddot(k, v) * (1.0 - c)));
}
__device__ inline void store3(float *p, D3 v) {
    p[0] = (float)v.x;
    p[1] = (float)v.y;
    p[2] = (float)v.z;
}

}  // namespace

// One thread per cap and per instance; thread 0 then refits the top-level boxes.
__global__ void prepare_kernel(PrepareArgs a) {
    int tid = threadIdx.x;
    for (int i = tid; i < a.n_caps; i += blockDim.x) {
        const CapStatic &cs = a.caps_static[i];
        const SegDev &sg = a.segs[cs.segment];
        const float *p = a.params + 6 * cs.segment;
        double tx = p[0], ty = p[1], R = p[2];
        D3 e1 = dload(sg.e1), e2 = dload(sg.e2), u0 = dload(sg.u0);
        D3 r1 = drot(e1, tx, u0);
        D3 ax = drot(e2, ty, r1);
        D3 C = dadd(dadd(dload(sg.pivot), D3{p[3], p[4], p[5]}), dmul(ax, R));
        CapDev &cd = a.caps[i];
        store3(cd.C, C);
        cd.R = (float)R;
        store3(cd.axis, ax);
        cd.segment = cs.segment;
        store3(cd.O, dload(cs.O));
        cd.material = cs.material;
        store3(cd.A, dload(cs.A));
        store3(cd.B, dload(cs.B));
        cd.a_lo = (float)cs.bounds[0];
        cd.a_hi = (float)cs.bounds[1];
        cd.b_lo = (float)cs.bounds[2];
        cd.b_hi = (float)cs.bounds[3];
        store3(cd.dCdtx, dmul(drot(e2, ty, dcross(e1, r1)), R));
        store3(cd.dCdty, dmul(dcross(e2, ax), R));
        // box of the cap: the cell prism over the sphere heights reached inside the cell
        D3 O = dload(cs.O), A = dload(cs.A), B = dload(cs.B);
        D3 W = dcross(A, B);
        D3 CO = dsub(C, O);
        double ca = ddot(CO, A), cb = ddot(CO, B), cw = ddot(CO, W);
        double sgn = ddot(ax, W) > 0 ? -1.0 : 1.0;   // pivot side of the centre along W
        double qa = fmin(fmax(ca, cs.bounds[0]), cs.bounds[1]) - ca;
        double qb = fmin(fmax(cb, cs.bounds[2]), cs.bounds[3]) - cb;
        double rmin2 = qa * qa + qb * qb;
        double fa = fmax(fabs(cs.bounds[0] - ca), fabs(cs.bounds[1] - ca));
        double fb = fmax(fabs(cs.bounds[2] - cb), fabs(cs.bounds[3] - cb));
        double rmax2 = fa * fa + fb * fb;
        double h0 = cw + sgn * sqrt(fmax(0.0, R * R - rmax2));
        double h1 = cw + sgn * sqrt(fmax(0.0, R * R - rmin2));
        double hlo = fmin(h0, h1), hhi = fmax(h0, h1);
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int c = 0; c < 8; ++c) {
            double aa = cs.bounds[(c & 1) ? 1 : 0], bb = cs.bounds[(c & 2) ? 3 : 2], hh = (c & 4) ? hhi : hlo;
            D3 P = dadd(dadd(dadd(O, dmul(A, aa)), dmul(B, bb)), dmul(W, hh));
            double q[3] = {P.x, P.y, P.z};
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], q[k]);
                hi[k] = fmax(hi[k], q[k]);
            }
        }
        for (int k = 0; k < 3; ++k) {
            double pad = 1e-2 + 1e-6 * fmax(fabs(lo[k]), fabs(hi[k]));
            cd.lo[k] = (float)(lo[k] - pad);
            cd.hi[k] = (float)(hi[k] + pad);
        }
    }
    for (int j = tid; j < a.n_inst; j += blockDim.x) {
        Instance &in = a.inst[j];
        if (in.segment < 0) continue;
        const SegDev &sg = a.segs[in.segment];
        const float *p = a.params + 6 * in.segment;
        double tx = p[0], ty = p[1], R = p[2];
        double s = R / sg.r0;
        D3 e1 = dload(sg.e1), e2 = dload(sg.e2);
        D3 cols[3], dcx[3], dcy[3];
        for (int c = 0; c < 3; ++c) {
            D3 ej = D3{c == 0 ? 1.0 : 0.0, c == 1 ? 1.0 : 0.0, c == 2 ? 1.0 : 0.0};
            D3 r1 = drot(e1, tx, ej);
            cols[c] = drot(e2, ty, r1);
            dcx[c] = drot(e2, ty, dcross(e1, r1));
            dcy[c] = dcross(e2, cols[c]);
        }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double rc = r == 0 ? cols[c].x : (r == 1 ? cols[c].y : cols[c].z);
                in.rot[3 * r + c] = (float)rc;
                in.m[3 * c + r] = (float)(rc / s);   // (1/s) Rot^T
                in.drx[3 * r + c] = (float)(r == 0 ? dcx[c].x : (r == 1 ? dcx[c].y : dcx[c].z));
                in.dry[3 * r + c] = (float)(r == 0 ? dcy[c].x : (r == 1 ? dcy[c].y : dcy[c].z));
            }
        D3 org = dadd(dload(sg.pivot), D3{p[3], p[4], p[5]});
        store3(in.org, org);
        in.scale = (float)s;
        in.inv_r0 = (float)(1.0 / sg.r0);
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int c = 0; c < 8; ++c) {
            D3 l = D3{(c & 1) ? in.loc_hi[0] : in.loc_lo[0], (c & 2) ? in.loc_hi[1] : in.loc_lo[1],
                      (c & 4) ? in.loc_hi[2] : in.loc_lo[2]};
            D3 w = dadd(org, dmul(dadd(dadd(dmul(cols[0], l.x), dmul(cols[1], l.y)), dmul(cols[2], l.z)), s));
            double q[3] = {w.x, w.y, w.z};
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], q[k]);
                hi[k] = fmax(hi[k], q[k]);
            }
        }
        for (int k = 0; k < 3; ++k) {
            double pad = 1e-2 + 1e-6 * fmax(fabs(lo[k]), fabs(hi[k]));
            in.lo[k] = (float)(lo[k] - pad);
            in.hi[k] = (float)(hi[k] + pad);
        }
    }
    __syncthreads();
    __threadfence_block();
    if (tid == 0) {
        // children follow their parent in depth-first order: refit from the back
        for (int i = a.n_top - 1; i >= 0; --i) {
            Node4 &nd = a.nodes[i];
            for (int k = 0; k < 4; ++k) {
                uint32_t c = nd.child[k];
                if (c == kEmpty) continue;
                float lo[3], hi[3];
                if (c & kLeafBit) {
                    const Instance &in = a.inst[c & ~(kLeafBit | kInstBit)];
                    for (int q = 0; q < 3; ++q) {
                        lo[q] = in.lo[q];
                        hi[q] = in.hi[q];
                    }
                } else {
                    const Node4 &ch = a.nodes[c];
                    for (int q = 0; q < 3; ++q) {
                        lo[q] = INFINITY;
                        hi[q] = -INFINITY;
                    }
                    for (int m = 0; m < 4; ++m) {
                        if (ch.child[m] == kEmpty) continue;
                        lo[0] = fminf(lo[0], ch.lox[m]);
                        lo[1] = fminf(lo[1], ch.loy[m]);
                        lo[2] = fminf(lo[2], ch.loz[m]);
                        hi[0] = fmaxf(hi[0], ch.hix[m]);
                        hi[1] = fmaxf(hi[1], ch.hiy[m]);
                        hi[2] = fmaxf(hi[2], ch.hiz[m]);
                    }
                }
                nd.lox[k] = lo[0];
                nd.loy[k] = lo[1];
                nd.loz[k] = lo[2];
                nd.hix[k] = hi[0];
                nd.hiy[k] = hi[1];
                nd.hiz[k] = hi[2];
            }
        }
    }
}

hipError_t launch_prepare(const PrepareArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(prepare_kernel, dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Graph-safe zeroing of small counters (no memset node in captured graphs).
__global__ void fill_u64_kernel(unsigned long long *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_fill_u64(unsigned long long *p, int n, hipStream_t st) {
    hipLaunchKernelGGL(fill_u64_kernel, dim3((n + 63) / 64), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------- per-photon body

// Trace photon g (output slot i), write its results and return its fate (-1
// for inactive lanes).  Every lane of the wave must call this together: the
// hit list uses wave-wide ballots.
// Per-photon output store.  kStream: a non-temporal store, which L2 keeps
// for a short time only, so that a large batch's gigabytes of outputs do
// not push the scene out of L2 (the batch kernel; the forward kernel writes
// each line in several passes and keeps them in L2 to merge).
template <bool kStream, class T>
__device__ __forceinline__ void put(T *p, T v) {
    if constexpr (kStream) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// kConstDet: read the detector through the constant address space (scalar
// loads).  The forward kernel gains from it; the batch kernel, held to 128
// VGPRs, spills the extra scalar state and reads the detector per lane.  The
// batch kernel (kConstDet false) streams its outputs past L2.
// rejected: the pre-filter's decision for this photon is already known to be
// a rejection (the forward sort took it), so it is neither generated nor
// tested again.
template <bool kConstDet>
__device__ __forceinline__ int photon_job(const DevScene &S, const DevSource &src, const DevOutputs &out, bool active,
                                          uint64_t i, uint64_t g, uint64_t seed, uint32_t *stk,
                                          int track = -1, bool rejected = false) {
    PathEnd end;
    end.fate = -1;
    end.pixel = -1;
    if (active) {
        if (rejected) {
            end.fate = kPrefiltered;
        } else {
            Photon ph = make_photon(src, seed, g, i, true, track);
            NoRecord rec;
            auto run = [&](const auto &det) {
                if (!src.prefilter) {
                    propagate(S, det, ph, seed, g, stk, end, rec);
                } else if (prefilter_keep(S, det, src, ph, seed, g)) {
                    propagate(S, det, ph, seed, g, stk, end, rec, false);
                } else {
                    end.fate = kPrefiltered;
                }
            };
            if constexpr (kConstDet) run(cref(*S.det));
            else run(*S.det);
        }
        bool on_det = end.fate == kDetected || end.fate == kQeRejected;
        constexpr bool kStream = !kConstDet;
        const float nan = __builtin_nanf("");
        if (out.fate) put<kStream>(out.fate + i, (uint8_t)end.fate);
        if (out.pixel) put<kStream>(out.pixel + i, on_det ? end.pixel : -1);
        if (out.hit_xyz) {
            float *p = out.hit_xyz + 3 * i;
            put<kStream>(p, on_det ? end.P.x : nan);
            put<kStream>(p + 1, on_det ? end.P.y : nan);
            put<kStream>(p + 2, on_det ? end.P.z : nan);
        }
        if (out.hit_uv) {
            float *p = out.hit_uv + 2 * i;
            put<kStream>(p, on_det ? end.u : nan);
            put<kStream>(p + 1, on_det ? end.v : nan);
        }
        if (out.hit_time) put<kStream>(out.hit_time + i, on_det ? end.time : nan);
        if (out.histogram && end.fate == kDetected) atomicAdd(out.histogram + end.pixel, 1u);
    }
    if (out.hit_list) {
        const int lane = __lane_id();
        unsigned long long m = __ballot(end.fate == kDetected);
        if (m) {
            int leader = __ffsll((long long)m) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(out.hit_count, (unsigned long long)__popcll(m));
            uint32_t lo = __shfl((uint32_t)base, leader), hi = __shfl((uint32_t)(base >> 32), leader);
            base = ((unsigned long long)hi << 32) | lo;
            if (end.fate == kDetected) {
                unsigned long long slot = base + __popcll(m & ((1ull << lane) - 1ull));
                if (slot < out.hit_capacity) {
                    char *rec = reinterpret_cast<char *>(out.hit_list) + 24 * slot;
                    *reinterpret_cast<uint64_t *>(rec) = g;
                    *reinterpret_cast<int32_t *>(rec + 8) = end.pixel;
                    float *xyz = reinterpret_cast<float *>(rec + 12);
                    xyz[0] = end.P.x;
                    xyz[1] = end.P.y;
                    xyz[2] = end.P.z;
                } else {
                    atomicOr(S.status, 1u);  // RICH_FLAG_HITLIST_OVERFLOW
                }
            }
        }
    }
    return end.fate;
}

// Per-wave fate tally: ballots give wave-uniform counts, so no atomics here.
__device__ __forceinline__ void tally_wave(uint32_t cnt[kFates], int fate) {
#pragma unroll
    for (int f = 0; f < kFates; ++f)
        cnt[f] += (uint32_t)__builtin_amdgcn_readfirstlane((int)__popcll(__ballot(fate == f)));
}

// Fold the per-wave tallies of a block into the caller's fate counters.  The
// block sums its waves in LDS; thread 0 adds the block total into one of
// kTallySlots cache-line slots (so concurrent blocks contend on 16 lines, not
// one); the last block to finish moves the slot totals into out.fate_counts
// and leaves the slots at zero for the next launch.  Called by every thread.
__device__ __forceinline__ void flush_tally(const DevScene &S, const DevOutputs &out, const uint32_t cnt[kFates],
                                            uint32_t *lds_cnt) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
    if (lane == 0)
        for (int f = 0; f < kFates; ++f) lds_cnt[kFates * wave + f] = cnt[f];
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long *slot = S.tally + (size_t)(blockIdx.x % kTallySlots) * kTallyStride;
        for (int f = 0; f < kFates; ++f) {
            unsigned long long sum = 0;
            for (int w = 0; w < waves; ++w) sum += lds_cnt[kFates * w + f];
            if (sum) atomicAdd(slot + f, sum);
        }
        __threadfence();
        unsigned long long *fin = S.tally + (size_t)kTallySlots * kTallyStride;
        unsigned long long done = atomicAdd(fin, 1ull);
        if (done == (unsigned long long)gridDim.x - 1ull) {
            __threadfence();
            for (int f = 0; f < kFates; ++f) {
                unsigned long long tot = 0;
                for (int k = 0; k < kTallySlots; ++k) tot += atomicExch(S.tally + (size_t)k * kTallyStride + f, 0ull);
                if (tot) atomicAdd(out.fate_counts + f, tot);
            }
            atomicExch(fin, 0ull);
        }
    }
}

// ---------------------------------------------------------------- forward: sorted order or grid-stride

constexpr int kForwardBlock = 256;

// Regrouping bin of photon g among `bins` bins: its cone azimuth's uniform
// (word 0 of its first Philox block) in bins 0..bins-2, and the last bin
// for photons the pre-filter rejects (so kept photons fill waves densely).
__device__ __forceinline__ uint32_t regroup_bin(const DevScene &S, const DevSource &src, uint64_t seed, uint64_t g,
                                                uint64_t i, uint32_t bins) {
    const uint32_t top = bins - 1u;
    work(kWorkSortKeys);
    const uint4 w = photon_block(seed, g, 0);
    if (src.prefilter && src.n_disp == 0 && src.kind != 2) {
        // the wavelength alone decides (with dispersion or explicit photons
        // the rejected ones are not set apart)
        Photon ph;
        ph.lambda = rcp(fmaf(-u24(w.y), src.inv_span, src.inv_lmin));
        if (!prefilter_keep(S, *S.det, src, ph, seed, g)) return top;
    }
    if (src.kind == 2) return 0u;
    const uint32_t b = (uint32_t)(((uint64_t)w.x * bins) >> 32);
    return b < top ? b : top - 1u;
}

// Photons of a forward launch are traced in an order sorted by cone azimuth
// within windows of kWindow ids: sort_photons_kernel counting-sorts each
// window by the azimuth's uniform (word 0 of the photon's first Philox block;
// the photons the pre-filter rejects last) into kBins bins, and the trace
// kernel's waves then take 64 neighbours in that order, whose rays meet the
// same parts of the scene.  Every photon keeps its id and random numbers and
// writes its outputs at its id; only the lane that traces it changes.  Wider
// windows give each wave closer directions but cost the sort more: traced
// launches sort windows of 32,768 ids, pre-filtered ones (whose trace is
// short) windows of 8192.
template <int kWindow, int kBins, int kThreads>
struct SortShape {
    static constexpr int window = kWindow, bins = kBins, threads = kThreads;
    static_assert(kWindow % kThreads == 0 && kBins % kThreads == 0 && kWindow <= 65536 &&
                      kSortedChunk % kWindow == 0 && kSortedChunk <= (uint64_t(1) << 31) && kThreads % 64 == 0 &&
                      kThreads >= kBatchCounters,   // one block zeroes every claim counter
                  "sort shape");
};
using WideSort = SortShape<32768, 2048, 1024>;
using NarrowSort = SortShape<8192, 1024, 512>;

template <class Shape>
__global__ __launch_bounds__(Shape::threads) void sort_photons_kernel(DevScene S, DevSource src, uint64_t n,
                                                                      uint64_t first, uint64_t seed, uint32_t *sorted,
                                                                      unsigned long long *counter) {
    constexpr int kSortWindow = Shape::window, kSortBins = Shape::bins, kSortThreads = Shape::threads;
    __shared__ uint32_t bins[kSortBins];
    // the trace kernel's claim counters start at zero (it runs next on the stream)
    if (blockIdx.x == 0 && threadIdx.x < kBatchCounters) counter[threadIdx.x] = 0;
    __shared__ uint16_t slot[kSortWindow];
    __shared__ uint32_t wave_sum[kSortThreads / 64];
    constexpr int per = kSortWindow / kSortThreads;
    const uint64_t w0 = (uint64_t)blockIdx.x * kSortWindow;
    const uint32_t m = (uint32_t)(n - w0 < (uint64_t)kSortWindow ? n - w0 : (uint64_t)kSortWindow);
    for (int q = threadIdx.x; q < kSortBins; q += kSortThreads) bins[q] = 0;
    __syncthreads();
    // bin and rank within the bin (16 bits each) of this thread's photons
    uint32_t key[per];
#pragma unroll
    for (int j = 0; j < per; ++j) {
        const uint32_t l = (uint32_t)(j * kSortThreads) + threadIdx.x;
        key[j] = 0;
        if (l < m) {
            const uint32_t b = regroup_bin(S, src, seed, first + w0 + l, w0 + l, kSortBins);
            key[j] = b | (atomicAdd(bins + b, 1u) << 16);
        }
    }
    __syncthreads();
    // exclusive scan of the bin counts: per thread, then per wave, then across waves
    constexpr int bpt = kSortBins / kSortThreads;
    uint32_t c[bpt], sum = 0;
#pragma unroll
    for (int q = 0; q < bpt; ++q) {
        c[q] = bins[bpt * threadIdx.x + q];
        sum += c[q];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = sum;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
    }
    if (lane == 63) wave_sum[wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int w = 0; w < wave; ++w) run += wave_sum[w];
#pragma unroll
    for (int q = 0; q < bpt; ++q) {
        bins[bpt * threadIdx.x + q] = run;
        run += c[q];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < per; ++j) {
        const uint32_t l = (uint32_t)(j * kSortThreads) + threadIdx.x;
        if (l < m) slot[bins[key[j] & 0xFFFFu] + (key[j] >> 16)] = (uint16_t)l;
    }
    // photons the pre-filter rejects fill the window's last bin (when the
    // wavelength alone decides): their sorted entries carry the top bit, and
    // the trace writes their fate without generating them again
    const uint32_t rejected_from = src.prefilter && src.n_disp == 0 && src.kind != 2 ? bins[kSortBins - 1] : m;
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < m; q += kSortThreads)
        sorted[w0 + q] = (uint32_t)(w0 + slot[q]) | (q >= rejected_from ? 0x80000000u : 0u);
}

// kRejectBit: sorted entries with the top bit set are photons the sort
// already saw the pre-filter reject (pre-filtered launches only).
template <bool kRejectBit>
__global__ __launch_bounds__(kForwardBlock) void forward_kernel(DevScene S, DevSource src, DevOutputs out, uint64_t n,
                                                                uint64_t first, uint64_t seed, const uint32_t *sorted,
                                                                unsigned long long *counter) {
    extern __shared__ uint32_t lds_stack[];
    uint32_t cnt[kFates] = {0, 0, 0, 0, 0, 0, 0};
    if (!sorted) {
        const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
        for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
            uint64_t i = base + threadIdx.x;
            int fate = photon_job<true>(S, src, out, i < n, i, first + i, seed, lane_stack(lds_stack));
            if (out.fate_counts) tally_wave(cnt, fate);
        }
    } else {
        // The sorted positions are split into one contiguous range per XCD
        // (workgroups are dealt to the eight XCDs round robin), so that an
        // XCD's photons in flight are neighbours in the sorted order and
        // their outputs lie in few windows.  Each wave claims the next 64
        // positions of its XCD's range from that range's counter (its own
        // cache line), so the waves of a CU trace neighbouring directions at
        // once and a wave that drew cheap photons takes more.
        const uint32_t parts = gridDim.x >= 8 ? 8u : 1u;
        const uint32_t x = blockIdx.x % parts;
        const uint64_t span = (n + (uint64_t)parts * 64 - 1) / ((uint64_t)parts * 64) * 64;
        const uint64_t lo = (uint64_t)x * span, hi = lo + span < n ? lo + span : n;
        unsigned long long *ctr = counter + kCounterStride * x;
        const int lane = threadIdx.x & 63;
        while (true) {
            unsigned long long c = 0;
            if (lane == 0) c = atomicAdd(ctr, 64ull);
            const uint32_t c_lo = __shfl((uint32_t)c, 0), c_hi = __shfl((uint32_t)(c >> 32), 0);
            const uint64_t k = lo + (((uint64_t)c_hi << 32) | c_lo) + (uint64_t)lane;
            if (k - lane >= hi) break;
            const bool active = k < hi;
            if constexpr (kRejectBit) {
                const uint32_t e = active ? sorted[k] : 0u;
                const uint64_t i = e & 0x7FFFFFFFu;
                int fate = photon_job<true>(S, src, out, active, i, first + i, seed, lane_stack(lds_stack), -1,
                                            (e >> 31) != 0u);
                if (out.fate_counts) tally_wave(cnt, fate);
            } else {
                const uint64_t i = active ? sorted[k] : 0;
                int fate = photon_job<true>(S, src, out, active, i, first + i, seed, lane_stack(lds_stack));
                if (out.fate_counts) tally_wave(cnt, fate);
            }
        }
    }
    if (out.fate_counts) flush_tally(S, out, cnt, lds_stack + (size_t)blockDim.x * kStackDepth);
}

// Large analytic launches: waves claim 64 ids at a time from their XCD's
// counter in one contiguous range of ids per XCD (as the sorted trace claims
// sorted positions), so the XCD's waves finish together.
__global__ __launch_bounds__(kForwardBlock) void forward_ids_kernel(DevScene S, DevSource src, DevOutputs out,
                                                                    uint64_t n, uint64_t first, uint64_t seed,
                                                                    unsigned long long *counter) {
    extern __shared__ uint32_t lds_stack[];
    uint32_t cnt[kFates] = {0, 0, 0, 0, 0, 0, 0};
    const uint32_t parts = gridDim.x >= 8 ? 8u : 1u;
    const uint32_t x = blockIdx.x % parts;
    const uint64_t span = (n + (uint64_t)parts * 64 - 1) / ((uint64_t)parts * 64) * 64;
    const uint64_t lo = (uint64_t)x * span, hi = lo + span < n ? lo + span : n;
    unsigned long long *ctr = counter + kCounterStride * x;
    const int lane = threadIdx.x & 63;
    while (true) {
        unsigned long long c = 0;
        if (lane == 0) c = atomicAdd(ctr, 64ull);
        const uint32_t c_lo = __shfl((uint32_t)c, 0), c_hi = __shfl((uint32_t)(c >> 32), 0);
        const uint64_t i = lo + (((uint64_t)c_hi << 32) | c_lo) + (uint64_t)lane;
        if (i - lane >= hi) break;
        int fate = photon_job<true>(S, src, out, i < hi, i, first + i, seed, lane_stack(lds_stack));
        if (out.fate_counts) tally_wave(cnt, fate);
    }
    if (out.fate_counts) flush_tally(S, out, cnt, lds_stack + (size_t)blockDim.x * kStackDepth);
}

bool forward_sorted(const DevScene &S, const DevSource &src) {
    return (S.has_mesh && src.kind != 2) || src.prefilter;
}

// How a forward launch hands photons to lanes: a grid-stride loop over the
// ids (small analytic launches: no extra launch before it), or waves claiming
// 64 positions at a time, of the sorted order (meshed scenes, pre-filter) or
// of the ids themselves (large analytic launches).
enum ForwardMode { kGridStride = 0, kSortedClaims = 1, kIdClaims = 2 };

// Analytic launches of at least this many photons claim their ids (after a
// fill launch that zeroes the counters); smaller ones are launch bound.
constexpr uint64_t kIdClaimsMin = uint64_t(1) << 22;

hipError_t launch_forward(const DevScene &S, const DevSource &src, const DevOutputs &out, uint64_t n, uint64_t first,
                          uint64_t seed, int n_cu, uint32_t *sorted, unsigned long long *counter, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const bool sort = forward_sorted(S, src);
    if (!counter || (sort && !sorted)) return hipErrorInvalidValue;
    const size_t lds = (size_t)kForwardBlock * kStackDepth * sizeof(uint32_t) +
                       kFates * (kForwardBlock / 64) * sizeof(uint32_t);
    // One block per resident slot (registers and LDS decide how many fit on
    // a CU), each looping over its photons; a grid of more blocks runs in
    // waves of blocks, and a partial last wave leaves most CUs idle.  The
    // grid-stride form takes two blocks per slot, which measured faster
    // there.  A claiming grid is a multiple of the eight XCDs, each XCD's
    // blocks claiming from its own counter.
    auto slots = [lds](const void *kernel) {
        int b = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, kForwardBlock, lds) == hipSuccess && b > 0 ? b
                                                                                                                  : 4;
    };
    static const int per_cu[3] = {slots((const void *)forward_kernel<false>), slots((const void *)forward_kernel<false>),
                                  slots((const void *)forward_ids_kernel)};
    // sorted launches go in chunks of at most kSortedChunk photons (the order
    // buffer's size); the outputs of a chunk start at its first photon
    const uint64_t step = sort ? kSortedChunk : n;
    for (uint64_t off = 0; off < n; off += step) {
        const uint64_t m = n - off < step ? n - off : step;
        const int mode = sort ? kSortedClaims : (m >= kIdClaimsMin ? kIdClaims : kGridStride);
        DevOutputs o = out;   // every per-photon output is optional
        if (o.fate) o.fate += off;
        if (o.pixel) o.pixel += off;
        if (o.hit_xyz) o.hit_xyz += 3 * off;
        if (o.hit_uv) o.hit_uv += 2 * off;
        if (o.hit_time) o.hit_time += off;
        const uint64_t cap = (uint64_t)(n_cu > 0 ? n_cu : 256) * (uint64_t)per_cu[mode] * (mode == kGridStride ? 2u : 1u);
        uint64_t blocks = (m + kForwardBlock - 1) / kForwardBlock;
        if (blocks > cap) blocks = cap;
        if (mode != kGridStride && blocks >= 8) blocks -= blocks % 8;
        hipError_t e = hipSuccess;
        if (mode == kSortedClaims) {
            // the sort also zeroes the claim counters
            if (src.prefilter)
                hipLaunchKernelGGL(sort_photons_kernel<NarrowSort>,
                                   dim3((unsigned)((m + NarrowSort::window - 1) / NarrowSort::window)),
                                   dim3(NarrowSort::threads), 0, st, S, src, m, first + off, seed, sorted, counter);
            else
                hipLaunchKernelGGL(sort_photons_kernel<WideSort>,
                                   dim3((unsigned)((m + WideSort::window - 1) / WideSort::window)),
                                   dim3(WideSort::threads), 0, st, S, src, m, first + off, seed, sorted, counter);
            e = hipGetLastError();
        } else if (mode == kIdClaims) {
            e = launch_fill_u64(counter, kBatchCounters, st);
        }
        if (e != hipSuccess) return e;
        const dim3 grid((unsigned)blocks), block(kForwardBlock);
        if (mode == kIdClaims)
            hipLaunchKernelGGL(forward_ids_kernel, grid, block, lds, st, S, src, o, m, first + off, seed, counter);
        else if (mode == kSortedClaims && src.prefilter && src.n_disp == 0 && src.kind != 2)
            hipLaunchKernelGGL(forward_kernel<true>, grid, block, lds, st, S, src, o, m, first + off, seed,
                               (const uint32_t *)sorted, counter);
        else
            hipLaunchKernelGGL(forward_kernel<false>, grid, block, lds, st, S, src, o, m, first + off, seed,
                               (const uint32_t *)(mode == kSortedClaims ? sorted : nullptr), counter);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------- batch: processing order

constexpr int kOrderCellBits = 7;                        // cells per axis: 128
constexpr int kOrderCells = 1 << (2 * kOrderCellBits);   // 16384

// Cell of a direction: the octahedral map of the unit sphere onto [-1, 1]^2
// (the lower hemisphere folded outwards), a 128 x 128 grid, cells numbered in
// Morton order so that neighbouring numbers are neighbouring directions.
__device__ __forceinline__ uint32_t direction_cell(float x, float y, float z) {
    const float s = fabsf(x) + fabsf(y) + fabsf(z);
    float u = s > 0.0f ? x / s : 0.0f, v = s > 0.0f ? y / s : 0.0f;
    if (z < 0.0f) {
        const float fu = (1.0f - fabsf(v)) * copysignf(1.0f, u), fv = (1.0f - fabsf(u)) * copysignf(1.0f, v);
        u = fu;
        v = fv;
    }
    const int n = 1 << kOrderCellBits;
    const uint32_t iu = (uint32_t)min(max((int)((u + 1.0f) * 0.5f * n), 0), n - 1);
    const uint32_t iv = (uint32_t)min(max((int)((v + 1.0f) * 0.5f * n), 0), n - 1);
    uint32_t m = 0;
    for (int b = 0; b < kOrderCellBits; ++b) m |= (((iu >> b) & 1u) << (2 * b)) | (((iv >> b) & 1u) << (2 * b + 1));
    return m;
}

__global__ void order_cells_kernel(const float *tracks, int n_tracks, uint32_t *hist, uint32_t *cell_of) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tracks) return;
    const float4 *tr = reinterpret_cast<const float4 *>(tracks) + 2 * t;
    const float4 a = tr[0], b = tr[1];
    const uint32_t c = direction_cell(a.w, b.x, b.y);
    cell_of[t] = c;
    atomicAdd(hist + c, 1u);
}

// In place: counts per cell -> first position of each cell (one block).
__global__ __launch_bounds__(1024) void order_scan_cells_kernel(uint32_t *hist) {
    __shared__ uint32_t part[1024];
    constexpr int per = kOrderCells / 1024;
    const int t = threadIdx.x;
    uint32_t v[per], sum = 0;
#pragma unroll
    for (int j = 0; j < per; ++j) {
        v[j] = hist[t * per + j];
        sum += v[j];
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t y = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
#pragma unroll
    for (int j = 0; j < per; ++j) {
        hist[t * per + j] = run;
        run += v[j];
    }
}

// Track t takes the next position of its cell (order within a cell is that of
// the atomics: it does not change any photon's result), and position pos goes
// to partition pos mod parts: order[] lists partition 0's tracks, then 1's, ...
// Each position's photon count goes beside it, into order_off (scanned next).
__global__ void order_scatter_kernel(const uint32_t *cell_of, const uint64_t *offsets, uint32_t *cursor,
                                     int n_tracks, int parts, int32_t *order, uint64_t *order_count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tracks) return;
    const uint32_t pos = atomicAdd(cursor + cell_of[t], 1u);
    const uint32_t c = pos % (uint32_t)parts, per = (uint32_t)n_tracks / (uint32_t)parts;
    const uint32_t rem = (uint32_t)n_tracks % (uint32_t)parts;
    const uint32_t q = c * per + min(c, rem) + pos / (uint32_t)parts;
    order[q] = t;
    order_count[q] = offsets[t + 1] - offsets[t];
}

// In place: photon counts by position -> photons of the tracks before each
// position, order_off[n_tracks] = the total (one block).
__global__ __launch_bounds__(1024) void order_offsets_kernel(int n_tracks, uint64_t *order_off) {
    __shared__ unsigned long long part[1024];
    const int t = threadIdx.x;
    const int per = (n_tracks + 1023) / 1024;
    const int lo = min(t * per, n_tracks), hi = min(lo + per, n_tracks);
    unsigned long long sum = 0;
#pragma unroll 8
    for (int q = lo; q < hi; ++q) sum += order_off[q];   // unrolled: the loads overlap
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        unsigned long long y = t >= off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    unsigned long long run = part[t] - sum;
#pragma unroll 8
    for (int q = lo; q < hi; ++q) {
        const unsigned long long c = order_off[q];
        order_off[q] = run;
        run += c;
    }
    if (t == 1023) order_off[n_tracks] = part[1023];
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t order_buffer_bytes(int n_tracks) {
    return align256((size_t)kOrderCells * 4) + align256((size_t)n_tracks * 4) + align256((size_t)n_tracks * 4) +
           ((size_t)n_tracks + 1) * 8;
}

void set_order(DevSource &src, void *buffer) {
    const int T = src.n_tracks;
    char *b = static_cast<char *>(buffer);
    src.order = reinterpret_cast<const int32_t *>(b + align256((size_t)kOrderCells * 4) + align256((size_t)T * 4));
    src.order_off =
        reinterpret_cast<const uint64_t *>(b + align256((size_t)kOrderCells * 4) + 2 * align256((size_t)T * 4));
}

hipError_t launch_order(const DevSource &src, int n_parts, void *buffer, hipStream_t st) {
    const int T = src.n_tracks;
    char *b = static_cast<char *>(buffer);
    uint32_t *hist = reinterpret_cast<uint32_t *>(b);
    uint32_t *cell_of = reinterpret_cast<uint32_t *>(b + align256((size_t)kOrderCells * 4));
    int32_t *order = const_cast<int32_t *>(src.order);
    uint64_t *order_off = const_cast<uint64_t *>(src.order_off);
    hipError_t e = launch_fill_u64(reinterpret_cast<unsigned long long *>(hist), kOrderCells / 2, st);
    if (e != hipSuccess) return e;
    const int blocks = (T + 255) / 256;
    hipLaunchKernelGGL(order_cells_kernel, dim3(blocks), dim3(256), 0, st, src.tracks, T, hist, cell_of);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(order_scan_cells_kernel, dim3(1), dim3(1024), 0, st, hist);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(order_scatter_kernel, dim3(blocks), dim3(256), 0, st, (const uint32_t *)cell_of, src.offsets,
                       hist, T, n_parts, order, order_off);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(order_offsets_kernel, dim3(1), dim3(1024), 0, st, T, order_off);
    return hipGetLastError();
}

// Photon id of processing position v of a batch: v itself in id order, else
// the photon v - order_off[k] of the k-th track in processing order, whose
// index goes to `track` (-1 when unknown: make_photon then searches).  When n
// is not the tracks' photon total the order is not used (ids beyond it are
// drawn from the last track, as in id order).
__device__ __forceinline__ uint64_t batch_photon_id(const DevSource &src, uint64_t v, uint64_t n, int &track) {
    track = -1;
    if (!src.order) return v;
    const RICH_CONST uint64_t *oo = (const RICH_CONST uint64_t *)src.order_off;
    if (oo[src.n_tracks] != n || v >= n) return v;
    const int k = find_track_wave(src.order_off, src.n_tracks, v);
    const int t = src.order[k];
    const uint64_t g = src.offsets[t] + (v - oo[k]);
    if (g >= n) return v;   // offsets that do not rise (bad input) never send a write out of range
    track = t;
    return g;
}

// ---------------------------------------------------------------- batch: persistent, dynamic chunks

// Each wave repeatedly claims `chunk` consecutive photon ids from a global
// counter and traces them 64 at a time until the ids run out.  Every wave
// leaves the loop when a claim starts at or beyond n.
constexpr int kWaveGroup = 256;   // photons a batch wave regroups by cone azimuth

// Held to 128 VGPRs (4 waves per SIMD; 12 bytes of spills per lane): left
// alone the compiler takes a few more registers and a wave less.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void batch_kernel(
    DevScene S, DevSource src, DevOutputs out, uint64_t n, uint64_t seed, unsigned long long *counter, int chunk,
    int whole_batch, uint64_t part, int n_parts) {
    extern __shared__ uint32_t lds_stack[];
    const int lane = __lane_id();
    uint32_t *stk = lane_stack(lds_stack);
    const int wave = threadIdx.x >> 6;
    uint32_t *wperm = lds_stack + (size_t)blockDim.x * kStackDepth + kFates * (blockDim.x / 64) +
                      (size_t)wave * (kWaveGroup + 64);
    uint32_t *wbins = wperm + kWaveGroup;
    uint32_t cnt[kFates] = {0, 0, 0, 0, 0, 0, 0};
    if (whole_batch && blockIdx.x == 0 && threadIdx.x == 0 && src.offsets[src.n_tracks] != n)
        atomicOr(S.status, 8u);  // RICH_FLAG_BATCH_SIZE: n is not the photon total of the tracks
    // The processing positions 0..n-1 (photon ids, or with a processing order
    // its positions) are cut into n_parts contiguous partitions of `part`
    // positions (a multiple of the chunk); block b claims chunks of partition
    // b mod n_parts from that partition's own counter.  Blocks are dispatched
    // to the 8 XCDs round robin, so with 8 partitions each XCD works through
    // its own run of tracks and its L2 holds their geometry only.
    const int xp = (int)(blockIdx.x % (unsigned)n_parts);
    unsigned long long *ctr = counter + kCounterStride * xp;
    const uint64_t p_lo = (uint64_t)xp * part;
    const uint64_t p_hi = min(p_lo + part, n);
    while (true) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(ctr, (unsigned long long)chunk);
        uint32_t lo = __shfl((uint32_t)base, 0), hi = __shfl((uint32_t)(base >> 32), 0);
        base = p_lo + (((unsigned long long)hi << 32) | lo);
        if (base >= p_hi) break;
        // With meshes (or the pre-filter), each kWaveGroup-photon slice of the
        // chunk is regrouped by cone azimuth (64 bins of the azimuth's
        // uniform; pre-filter rejects last) in this wave's own LDS region, so
        // that each 64-photon pass traces neighbouring directions.  Only
        // chunks made of whole slices are regrouped: a partial slice would
        // reach into the next claim.  A wave's LDS operations complete in
        // order; the fences keep the compiler from moving them across phases.
        const bool regroup = (S.has_mesh || src.prefilter) && chunk % kWaveGroup == 0;
        const int group = regroup ? kWaveGroup : 64;
        for (int k = 0; k < chunk; k += group) {
            if (regroup) {
                constexpr int per = kWaveGroup / 64;
                wbins[lane] = 0;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                uint32_t bin[per], rank[per];
                for (int j = 0; j < per; ++j) {
                    const uint64_t v = base + (uint64_t)(k + j * 64 + lane);
                    int tk = -1;
                    const uint64_t g = v < n ? batch_photon_id(src, v, n, tk) : v;
                    bin[j] = v < n ? regroup_bin(S, src, seed, g, g, 64u) : 63u;
                    rank[j] = atomicAdd(wbins + bin[j], 1u);
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                const uint32_t c = wbins[lane];
                uint32_t incl = c;
                for (int d = 1; d < 64; d <<= 1) {
                    uint32_t v = __shfl_up(incl, d);
                    if (lane >= d) incl += v;
                }
                wbins[lane] = incl - c;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                for (int j = 0; j < per; ++j)
                    wperm[min(wbins[bin[j]] + rank[j], (uint32_t)kWaveGroup - 1u)] = (uint32_t)(j * 64 + lane);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
            for (int j = 0; j < group; j += 64) {
                const uint32_t off = regroup ? wperm[j + lane] : (uint32_t)(j + lane);
                const uint64_t v = base + (uint64_t)k + off;
                int tk = -1;
                const uint64_t g = v < n ? batch_photon_id(src, v, n, tk) : v;
                int fate = photon_job<false>(S, src, out, v < n, g, g, seed, stk, tk);
                if (out.fate_counts) tally_wave(cnt, fate);
            }
            if (regroup) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
    }
    if (out.fate_counts) flush_tally(S, out, cnt, lds_stack + (size_t)blockDim.x * kStackDepth);
}

// Dynamic LDS of the batch kernel: per-lane stacks, per-wave fate tallies,
// per-wave regrouping buffers.
size_t batch_lds_bytes(int block) {
    return (size_t)block * kStackDepth * sizeof(uint32_t) + kFates * (block / 64) * sizeof(uint32_t) +
           (size_t)(block / 64) * (kWaveGroup + 64) * sizeof(uint32_t);
}

int batch_parts(int grid) { return (grid >= kBatchParts && grid % kBatchParts == 0) ? kBatchParts : 1; }

hipError_t launch_batch(const DevScene &S, const DevSource &src, const DevOutputs &out, uint64_t n, uint64_t seed,
                        unsigned long long *counter, int block, int chunk, int grid, bool whole_batch, hipStream_t st) {
    size_t lds = batch_lds_bytes(block);
    const int n_parts = batch_parts(grid);
    const uint64_t per = (n + n_parts - 1) / n_parts;
    const uint64_t part = (per + chunk - 1) / chunk * chunk;
    hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(block), lds, st, S, src, out, n, seed, counter, chunk,
                       whole_batch ? 1 : 0, part, n_parts);
    return hipGetLastError();
}

}  // namespace rich

#ifdef RICH_WORK_COUNTERS
// Measurement build only: copy the forward and batch kernels' work counters
// to the host (WorkUnit order: kWorkUnits lane counts, then kWorkUnits wave
// counts), then zero them when reset is set.  Synchronises the current device.
extern "C" int rich_work_counters(unsigned long long *out, int reset) {
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
