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
// Sums are deterministic: photons map statically to waves; per segment the
// wave reduces with a butterfly and lane 0 adds into wave-private LDS
// accumulators; blocks then sum their waves in order, and a final kernel sums
// the blocks in order.
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
constexpr int kAdjQueue = 128;   // per-wave queue of masked photons: < 64 left over + 64 new

// Accumulator row length rounded up to keep the queue that follows 8-byte aligned.
__host__ __device__ inline int padded_width(int n_par) { return (n_par + 2 + 1) & ~1; }
constexpr int kMaxRefl = 4;
constexpr uint32_t kKindCap = 0u, kKindPlane = 1u, kKindFacet = 2u;

struct Refl {
    V3 P, d, n;
    float t;
    uint32_t kind;   // kKind*
    uint32_t idx;    // cap index, or triangle slot of a moving facet
    int32_t inst;
};

struct PathRecorder {
    Refl r0, r1, r2, r3;
    int n = 0;
    bool overflow = false;
    bool hit_det = false;
    V3 det_d;
    float det_t = 0.0f;
    uint32_t n_caps = 0, prim_det = 0;
    const Instance *inst = nullptr;

    __device__ __forceinline__ void reflect(int b, const Hit &h, V3 o, V3 d, V3 P, V3 nrm) {
        Refl x;
        x.P = P;
        x.d = d;
        x.n = nrm;
        x.t = h.t;
        x.inst = h.inst;
        if (h.prim < n_caps) {
            x.kind = kKindCap;
            x.idx = h.prim;
        } else if (h.prim < prim_det || h.inst < 0 || inst[h.inst].segment < 0) {
            x.kind = kKindPlane;
            x.idx = 0;
        } else {
            x.kind = kKindFacet;
            x.idx = h.tri;
        }
        switch (n) {
            case 0: r0 = x; break;
            case 1: r1 = x; break;
            case 2: r2 = x; break;
            case 3: r3 = x; break;
            default: overflow = true; break;
        }
        ++n;
    }
    __device__ __forceinline__ void detect(int b, V3 o, V3 d, float t) {
        hit_det = true;
        det_d = d;
        det_t = t;
    }
    __device__ __forceinline__ Refl get(int k) const {
        switch (k) {
            case 0: return r0;
            case 1: return r1;
            case 2: return r2;
            default: return r3;
        }
    }
};

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

}  // namespace

__global__ __launch_bounds__(kAdjBlock) void adjoint_kernel(DevScene S, DevSource src, AdjointArgs a, uint64_t n,
                                                            uint64_t first, uint64_t seed) {
    extern __shared__ uint32_t lds[];
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const int width = a.n_par + 2;
    uint32_t *stk = lds + threadIdx.x;
    float *acc_all = reinterpret_cast<float *>(lds + (size_t)blockDim.x * kStackDepth);
    float *acc = acc_all + wave * width;
    for (int j = lane; j < width; j += 64) acc[j] = 0.0f;
    // per-wave queue of masked photon indices (see below)
    uint64_t *queue = reinterpret_cast<uint64_t *>(acc_all + (size_t)waves * padded_width(a.n_par)) +
                      (size_t)wave * kAdjQueue;

    const RICH_CONST DetDev &det = cref(*S.det);
    // Squared residual cut; a negative or NaN cut admits no photon.
    float cut2 = __builtin_inff();
    if (a.residual_cut) {
        float c = *a.residual_cut;
        cut2 = c >= 0.0f ? c * c : -1.0f;
    }
    // Masks usually keep a few percent of the photons.  Each wave scans its
    // fixed share of the ids (64 at a time, strided over the grid), queues
    // the masked ones in order, and traces them 64 at a time, so lanes are
    // not left idle through a traversal.  The scan order, hence which
    // photons share a pass and the order of every sum, is fixed.
    const uint64_t nw = (uint64_t)gridDim.x * waves;
    uint64_t base = ((uint64_t)blockIdx.x * waves + wave) * 64;
    int queued = 0;   // wave-uniform, < 64 between passes
    while (true) {
        const bool more = base < n;
        if (more) {
            const uint64_t j = base + (uint64_t)lane;
            const bool want = j < n && (a.mask == nullptr || a.mask[j] != 0);
            const unsigned long long m = __ballot(want);
            if (want) queue[queued + __popcll(m & ((1ull << lane) - 1ull))] = j;
            queued += __popcll(m);
            base += nw * 64;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            if (queued < 64) continue;
        }
        if (queued == 0) break;
        const int take = queued < 64 ? queued : 64;
        queued -= take;
        bool act = lane < take;
        const uint64_t i = act ? queue[queued + lane] : 0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        PathRecorder rec;
        rec.n_caps = (uint32_t)S.n_caps;
        rec.prim_det = S.prim_det;
        rec.inst = S.inst;
        PathEnd end;
        end.fate = -1;
        float gu = 0.0f, gv = 0.0f, loss = 0.0f, cnt = 0.0f;
        if (act) {
            uint64_t g = first + i;
            Photon ph = make_photon(src, seed, g, i, false);
            if (!src.prefilter) {
                propagate(S, det, ph, seed, g, stk, blockDim.x, end, rec);
            } else if (prefilter_keep(S, det, src, ph, seed, g)) {
                propagate(S, det, ph, seed, g, stk, blockDim.x, end, rec, false);
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
        // detector plane
        V3 gP = v3(0.0f, 0.0f, 0.0f), gD = v3(0.0f, 0.0f, 0.0f);
        if (act) {
            work(kWorkBackDetector);
            V3 gPd = fma3(gu, ld3(det.u), gv * ld3(det.v));
            gP = plane_back(gPd, rec.det_d, ld3(det.n));
            gD = rec.det_t * gP;
        }
        // reflections, last to first (uniform loop so the wave reductions stay converged)
        for (int k = kMaxRefl - 1; k >= 0; --k) {
            int seg = -1;
            float gp[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            if (act && k < rec.n) {
                Refl x = rec.get(k);
                float gdn = dot(gD, x.n);
                float dn = dot(x.d, x.n);
                V3 h = -2.0f * fma3(gdn, x.d, dn * gD);       // adjoint of the normal
                V3 gDin = fma3(-2.0f * gdn, x.n, gD);
                V3 gO;
                if (x.kind == kKindCap) {
                    work(kWorkBackCaps);
                    const CapDev &cp = S.caps[x.idx];
                    float invR = 1.0f / cp.R;
                    V3 w = x.P - ld3(cp.C);
                    V3 gPt = fma3(-invR, h, gP);
                    float s = dot(gPt, x.d) / dot(w, x.d);
                    gO = fma3(-s, w, gPt);
                    V3 gC = fma3(s, w, invR * h);
                    float gR = fmaf(s, cp.R, -dot(h, x.n) * invR);
                    seg = cp.segment;
                    gp[0] = dot(gC, ld3(cp.dCdtx));
                    gp[1] = dot(gC, ld3(cp.dCdty));
                    gp[2] = gR + dot(gC, ld3(cp.axis));
                    gp[3] = gC.x;
                    gp[4] = gC.y;
                    gp[5] = gC.z;
                } else if (x.kind == kKindFacet) {
                    work(kWorkBackFacets);
                    const Instance &in = S.inst[x.inst];
                    const Tri &tr = S.tris[x.idx];
                    V3 vl = ld3(tr.v0), nl = ld3(tr.n);
                    V3 rv = mat3(in.rot, vl);
                    V3 q = fma3(in.scale, rv, ld3(in.org));
                    float s = dot(gP, x.d) / dot(x.n, x.d);
                    gO = fma3(-s, x.n, gP);
                    V3 gq = s * x.n;
                    V3 gn = fma3(s, q - x.P, h);
                    seg = in.segment;
                    gp[0] = in.scale * dot(gq, mat3(in.drx, vl)) + dot(gn, mat3(in.drx, nl));
                    gp[1] = in.scale * dot(gq, mat3(in.dry, vl)) + dot(gn, mat3(in.dry, nl));
                    gp[2] = dot(gq, rv) * in.inv_r0;
                    gp[3] = gq.x;
                    gp[4] = gq.y;
                    gp[5] = gq.z;
                } else {
                    work(kWorkBackPlanes);
                    gO = plane_back(gP, x.d, x.n);
                }
                gP = gO;
                gD = fma3(x.t, gO, gDin);
            }
            wave_accumulate(acc, seg, gp);
        }
        float wl = wave_sum(loss), wc = wave_sum(cnt);
        if (lane == 0) {
            acc[a.n_par] += wl;
            acc[a.n_par + 1] += wc;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < width; j += blockDim.x) {
        float s = 0.0f;
        for (int w = 0; w < waves; ++w) s += acc_all[w * width + j];
        a.partials[(size_t)blockIdx.x * width + j] = s;
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

int adjoint_block_size() { return kAdjBlock; }

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

hipError_t launch_adjoint(const DevScene &S, const DevSource &src, const AdjointArgs &a, uint64_t n, uint64_t first,
                          uint64_t seed, int n_blocks, hipStream_t st) {
    size_t lds = (size_t)kAdjBlock * kStackDepth * sizeof(uint32_t) +
                 (size_t)(kAdjBlock / 64) * padded_width(a.n_par) * sizeof(float) +
                 (size_t)(kAdjBlock / 64) * kAdjQueue * sizeof(uint64_t);
    hipLaunchKernelGGL(adjoint_kernel, dim3(n_blocks), dim3(kAdjBlock), lds, st, S, src, a, n, first, seed);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(adjoint_reduce_kernel, dim3(a.n_par + 1), dim3(256), 0, st, (const float *)a.partials, n_blocks,
                       a.n_par, a.targets ? 1 : 0, a.grad, a.loss);
    return hipGetLastError();
}

}  // namespace rich

#ifdef RICH_WORK_COUNTERS
// Measurement build only: the adjoint kernel's work counters (this file's
// copy), as rich_work_counters gives the forward and batch kernels'.
extern "C" int rich_work_counters_adjoint(unsigned long long *out, int reset) {
    unsigned long long raw[16 * rich::kWorkUnits];
    if (hipDeviceSynchronize() != hipSuccess) return -3;
    if (hipMemcpyFromSymbol(raw, HIP_SYMBOL(rich::rich_work), sizeof raw) != hipSuccess) return -3;
    for (int u = 0; u < rich::kWorkUnits; ++u) out[u] = raw[16 * u];
    if (reset) {
        unsigned long long zero[16 * rich::kWorkUnits] = {};
        if (hipMemcpyToSymbol(HIP_SYMBOL(rich::rich_work), zero, sizeof zero) != hipSuccess) return -3;
    }
    return 0;
}
#endif
