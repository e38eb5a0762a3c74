// Host-side launchers of the librich kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "rich_dev.h"

namespace rich {

struct PrepareArgs {
    const SegDev *segs;
    const CapStatic *caps_static;
    const float *params;        // [n_seg][6]
    CapDev *caps;
    int32_t n_caps;
    Instance *inst;
    int32_t n_inst;
    Node4 *nodes;               // top-level nodes occupy [0, n_top)
    int32_t n_top;
};

hipError_t launch_prepare(const PrepareArgs &a, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, int n, hipStream_t st);
// Work counters of the batch and sorted forward kernels: one per id
// partition, a 128-byte line apart.
constexpr int kBatchParts = 8;
constexpr int kCounterStride = 16;
constexpr int kBatchCounters = kBatchParts * kCounterStride;
// Forward launches on meshed scenes (and every pre-filtered launch) trace
// their photons in an order sorted by cone azimuth: the caller passes an order
// buffer of min(n, kSortedChunk) uint32 words (non-null when forward_sorted
// holds), and launches of more photons go in chunks of kSortedChunk.  Every
// launch takes kBatchCounters counter words for its waves' claims (the
// launch zeroes them itself).
constexpr uint64_t kSortedChunk = uint64_t(1) << 24;
bool forward_sorted(const DevScene &S, const DevSource &src);
hipError_t launch_forward(const DevScene &S, const DevSource &src, const DevOutputs &out, uint64_t n,
                          uint64_t first, uint64_t seed, int n_cu, uint32_t *sorted, unsigned long long *counter,
                          hipStream_t st);
// whole_batch: n is meant to be every photon of the tracks (flag raised if not);
// counter: kBatchCounters zeroed words
hipError_t launch_batch(const DevScene &S, const DevSource &src, const DevOutputs &out, uint64_t n, uint64_t seed,
                        unsigned long long *counter, int block, int chunk, int grid, bool whole_batch, hipStream_t st);
size_t batch_lds_bytes(int block);
// Processing order of a batch's tracks: by direction (cells of an octahedral
// map in Morton order), dealt round robin to the n_parts id partitions of the
// batch kernel, so that every partition (one per XCD) works through the whole
// acceptance but its tracks in flight point the same way.  Work buffer of
// order_buffer_bytes(n_tracks) bytes: set_order points src.order and
// src.order_off into it, launch_order fills them on the stream.
size_t order_buffer_bytes(int n_tracks);
void set_order(DevSource &src, void *buffer);
hipError_t launch_order(const DevSource &src, int n_parts, void *buffer, hipStream_t st);
int batch_parts(int grid);

struct AdjointArgs {
    const float *grad_uv;       // [N][2] or null
    const float *targets;       // [N][2] or null
    const uint8_t *mask;        // [N] or null (all)
    const float *residual_cut;  // [1] or null (fused-loss mode only)
    float *partials;            // [rows][n_par + 2], set by launch_adjoint
    float *grad;                // [n_seg][6]
    float *loss;                // [1] or null
    int32_t n_par;
    uint32_t *chunk_counts;                    // mask given: masked ids per chunk, set by launch_adjoint
    const unsigned long long *chunk_offsets;   // their exclusive scan, [n_chunks + 1]
};
// Device work buffer of one adjoint call: block partial sums (one row of
// n_par + 2 floats per block and launch segment of up to 2^32 ids), then, with
// a mask, the per-chunk counts and their scan.
struct AdjointPlan {
    int n_blocks;          // blocks of the persistent grid
    int n_segments;        // launches of up to 2^32 ids
    uint64_t n_chunks;     // mask chunks of the largest segment (0 without a mask)
    size_t counts_offset, offsets_offset, bytes;
};
AdjointPlan adjoint_plan(uint64_t n, int n_par, int n_cu, bool masked);
hipError_t launch_adjoint(const DevScene &S, const DevSource &src, const AdjointArgs &a, uint64_t n, uint64_t first,
                          uint64_t seed, const AdjointPlan &plan, void *work, hipStream_t st);
// Work buffer of the no-allocation adjoint entry point: a file-scope device
// array of kAdjScratchFloats floats (8 MiB) on every device the library runs
// on.  adjoint_scratch returns its device address on `device`, which must be
// current; the address is looked up once per device and cached.
constexpr size_t kAdjScratchFloats = size_t(1) << 21;
constexpr int kAdjScratchDevices = 64;
hipError_t adjoint_scratch(int device, float **ptr);

// Film read-out emulation: film coordinates x = cx + scale u, y = cy + scale v.
struct FilmArgs {
    int32_t width, height;
    float cx, cy, scale;
    float radius;       // 4 sigma (film pixels)
    float inv_2s2;      // 1 / (2 sigma^2)
    float threshold;
};
hipError_t launch_film(const FilmArgs &a, const uint8_t *fate, const float *uv, uint64_t n, float *image,
                       uint8_t *hits, hipStream_t st);

// One step of the alignment fit's optimiser (Adam with a cosine step size).
struct FitArgs {
    int32_t n_par;          // 6 x segments
    int32_t n_steps;        // schedule length
    double lr, lr_final, beta1, beta2, eps;
    float scale[6];         // column normalisation
    int32_t free[6];        // fitted columns
    float outlier_cut, cut_floor;
    const float *p0, *grad, *loss;
    float *state;           // z [n_par], m [n_par], v [n_par], steps taken
    float *params;          // the scene's parameter array
    float *params_out;      // optional copy
    float *losses;          // optional loss record [n_steps]
    float *cut;             // optional residual cut
};
hipError_t launch_fit_step(const FitArgs &a, hipStream_t st);

}  // namespace rich
