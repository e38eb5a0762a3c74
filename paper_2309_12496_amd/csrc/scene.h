// Host representation of a librich scene (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rich.h"
#include "rich_dev.h"

namespace rich {
constexpr int kStreamSlots = 64;   // streams that may launch on one scene
}  // namespace rich

// Device workspace of the launches made on one stream.  Launches on one
// scene from different streams may overlap: each stream has its own.
struct StreamWork {
    bool used = false;
    hipStream_t stream = nullptr;               // the launch stream that took this slot
    unsigned long long *counter = nullptr;      // batch work counters (in the scene's d_counters)
    unsigned long long *tally = nullptr;        // fate-count slots (in the scene's d_tallies), zero between launches
    float *partials = nullptr;                  // adjoint partial sums and mask counts, grown
    size_t partials_floats = 0;
    void *order = nullptr;                      // batch processing order (cells, tracks, offsets), grown
    size_t order_bytes = 0;
    uint32_t *sorted = nullptr;                 // forward photon order (one chunk's ids), grown
    uint64_t sorted_count = 0;
    // captured batch graph and the arguments it was captured with
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::string graph_key;
};

struct rich_scene {
    int device = 0;
    int n_cu = 0;

    // device memory (owned)
    rich::Node4 *d_nodes = nullptr;
    rich::Tri *d_tris = nullptr;
    rich::Instance *d_inst = nullptr;
    rich::CapDev *d_caps = nullptr;
    rich::CapStatic *d_caps_static = nullptr;
    rich::SegDev *d_segs = nullptr;
    rich::RectDev *d_rects = nullptr;
    rich::MatDev *d_mats = nullptr;
    rich::DetDev *d_det = nullptr;
    float *d_params = nullptr;
    unsigned int *d_status = nullptr;
    unsigned long long *d_counters = nullptr;  // batch work counters, kBatchCounters per stream slot
    unsigned long long *d_tallies = nullptr;   // fate-count slots, kTallyWords per stream slot

    rich::DevScene dev{};
    std::vector<int32_t> mat_kind;             // host copy of the material kinds
    int32_t n_segments = 0;
    int32_t n_top = 0;
    int32_t nx = 0, ny = 0;
    rich_scene_stats stats{};

    StreamWork slots[rich::kStreamSlots];
    std::mutex mu;                             // host calls on the scene, one at a time

    // launch shapes chosen by the autotuner, keyed by workload class
    std::map<std::string, rich_tuning> tuned;
};

namespace rich {
rich_status build_scene(const rich_scene_desc *d, int device, rich_scene **out);
void free_scene(rich_scene *s);
rich_status set_error(rich_status code, const char *fmt, ...);
}  // namespace rich
