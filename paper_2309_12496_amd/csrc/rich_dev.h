// Device-side data layout of librich (shared by the host scene builder and the kernels).
//
// HBM layout of a scene:
//   nodes  : Node4[]  128 B each, all BVH4s (top level first, then one BVH per
//            instance), depth-first so that a parent and its children are near.
//   tris   : Tri[]    64 B each, grouped by leaf, vertices in the local frame of
//            their instance, unit normals computed in FP64 on the host.
//   inst   : Instance[] world<->local transforms of mesh instances.
//   caps, rects, mats, detector tables: a few KB, read through the scalar cache.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rich {

constexpr uint32_t kStreamTag = 0x52494348u;   // fourth Philox counter word ("RICH")
constexpr int kStackDepth = 32;                // per-lane traversal stack entries (LDS)
// A wave's stacks are kStackDepth rows of 64 words in LDS: lane l's entry d
// is word 64 d + l of its wave's block.  The lanes of a row sit in distinct
// banks at any mix of depths, and consecutive entries are a fixed 256 B apart.
constexpr int kStackRow = 64;
constexpr int kMaxTable = 32;
constexpr int kFates = 7;                      // photon fates, RICH_N_FATES
constexpr int kTallySlots = 16;                // fate-count slots, one 128-byte line each
constexpr int kTallyStride = 16;               // 64-bit words per slot
constexpr int kTallyWords = kTallySlots * kTallyStride + kTallyStride;  // slots + finisher counter line

// BVH4 child reference encoding.
constexpr uint32_t kEmpty = 0xFFFFFFFFu;       // no child
constexpr uint32_t kLeafBit = 0x80000000u;     // leaf or instance
constexpr uint32_t kInstBit = 0x40000000u;     // with kLeafBit: instance reference
constexpr uint32_t kExitMarker = 0xFFFFFFFEu;  // stack entry: return to the world frame
constexpr uint32_t kLeafMaxTris = 8;
// Scene size limits: traversal addresses triangles (64 B) and nodes (128 B)
// with 32-bit byte offsets from the array bases.
constexpr int64_t kMaxTriangles = int64_t(1) << 26;   // exclusive
constexpr int64_t kMaxNodes = int64_t(1) << 25;       // exclusive
// leaf: kLeafBit | (count-1) << 27 | first   (first < 2^27, count 1..8)
// instance: kLeafBit | kInstBit | index
__host__ __device__ inline uint32_t make_leaf(uint32_t first, uint32_t count) {
    return kLeafBit | ((count - 1u) << 27) | first;
}
__host__ __device__ inline uint32_t make_inst(uint32_t idx) { return kLeafBit | kInstBit | idx; }

struct alignas(128) Node4 {
    float lox[4], hix[4], loy[4], hiy[4], loz[4], hiz[4];
    uint32_t child[4];
    uint32_t pad[4];
};
static_assert(sizeof(Node4) == 128, "Node4 must be 128 bytes");

// Triangle record: v0.xyz + global triangle index, v1.xyz + material, v2.xyz, normal.xyz.
struct alignas(16) Tri {
    float v0[3];
    uint32_t index;
    float v1[3];
    uint32_t material;
    float v2[3];
    uint32_t pad0;
    float n[3];
    uint32_t pad1;
};
static_assert(sizeof(Tri) == 64, "Tri must be 64 bytes");

// Mesh instance: local = m * (world - org); world normal = rot * local normal.
struct alignas(16) Instance {
    float m[9];
    float org[3];
    float rot[9];
    float scale;
    uint32_t root;       // root node of this instance's BVH
    int32_t segment;     // -1: fixed
    float lo[3], hi[3];  // world AABB at the current parameters
    float loc_lo[3], loc_hi[3];  // local AABB
    float drx[9];        // d rot / d tilt_x (for the adjoint)
    float dry[9];        // d rot / d tilt_y
    float inv_r0;        // 1 / nominal radius of the segment (0 for fixed meshes)
    float pad;
};

// Analytic spherical cap at the current parameters.
struct alignas(16) CapDev {
    float C[3];
    float R;
    float axis[3];       // unit pivot -> centre
    int32_t segment;
    float O[3];
    int32_t material;
    float A[3];
    float a_lo;
    float B[3];
    float a_hi;
    float lo[3];         // world AABB of the cap
    float b_lo;
    float hi[3];
    float b_hi;
    float dCdtx[3];      // derivatives of C for the adjoint
    float pad0;
    float dCdty[3];
    float pad1;
};

struct alignas(16) RectDev {
    float c[3];
    int32_t material;
    float n[3];
    float hu;
    float u[3];
    float hv;
    float v[3];
    float pad;
};

// Piecewise-linear table: nodes x, values y, slope s[j] = (y[j+1]-y[j])/(x[j+1]-x[j]) (FP64 on the host).
struct MatDev {
    int32_t kind;
    int32_t n;
    float x[kMaxTable];
    float y[kMaxTable];
    float s[kMaxTable];
};

struct DetDev {
    float c[3], n[3], u[3], v[3];
    float hu, hv;            // geometric half sizes
    float pitch;
    float act_hu, act_hv;    // half sizes of the pixel grid
    int32_t nx, ny;
    int32_t n_qe;
    float inv_pitch;
    float qe_x[kMaxTable];
    float qe_y[kMaxTable];
    float qe_s[kMaxTable];
};

// FP64 master data used by the parameter update kernel.
struct SegDev {
    double pivot[3], u0[3], e1[3], e2[3];
    double r0;
};

struct CapStatic {
    int32_t segment, material;
    double O[3], A[3], B[3];
    double bounds[4];
};

// Everything a propagation kernel reads, passed by value.
struct DevScene {
    const CapDev *caps;
    const RectDev *rects;
    const MatDev *mats;
    const Node4 *nodes;
    const Tri *tris;
    const Instance *inst;
    const DetDev *det;
    unsigned int *status;
    unsigned long long *tally;   // fate-count slots (kTallyWords), zero between launches
    int32_t n_caps, n_rects, n_mats, n_inst;
    int32_t has_mesh, has_box;
    uint32_t top_root;
    int32_t max_bounces;
    float t_min;
    uint32_t prim_det, prim_box, prim_tri;   // global primitive numbering
    float box_lo[3], box_hi[3];
    int32_t n_seg;
};

// Photon source as seen by the kernels.
struct DevSource {
    int32_t kind;        // 0 track, 1 batch, 2 explicit
    // track: emission origin, direction frame, cone, spectrum (precomputed on the host in FP64)
    float P0[3], T[3], E1[3], E2[3];
    float length, cos_t, sin_t;
    float inv_lmin, inv_span;   // 1/lambda_min and 1/lambda_min - 1/lambda_max
    // batch
    const float *tracks;        // rich_track[] as 8 floats
    const uint64_t *offsets;
    int32_t n_tracks;
    // batch processing order (null: id order): the tracks in the order their
    // photons are processed, and the exclusive scan of their counts in that
    // order ([n_tracks + 1]); photon ids, hence results, do not change
    const int32_t *order;
    const uint64_t *order_off;
    double n_radiator;
    // explicit
    const float *ex_o, *ex_d, *ex_l;
    // pre-propagation efficiency filter (0 materials and prefilter = 0: off)
    int32_t prefilter;
    int32_t pf_n;
    int32_t pf_mats[4];
    // radiator dispersion (n_disp = 0: constant index): nodes, n - 1 and the
    // segment slopes dn/dlambda; the largest index over the band (FP64 host)
    int32_t n_disp;
    float disp_x[kMaxTable], disp_m[kMaxTable], disp_s[kMaxTable];
    double disp_nmax;
    float ng_const;     // group index without a table
    float beta;         // track: particle velocity / c
};

constexpr uint32_t kDispBlock = 0x7FFFFFFEu;   // wavelength retries use blocks kDispBlock - k
constexpr int kDispMaxTries = 64;
constexpr float kInvC = 1.0f / 299.792458f;    // ns per mm in vacuum

constexpr uint32_t kPrefilterBlock = 0x7FFFFFFFu;   // Philox block of the pre-filter draw

struct DevOutputs {
    uint8_t *fate;
    int32_t *pixel;
    float *hit_xyz;
    float *hit_uv;
    uint32_t *histogram;
    unsigned long long *fate_counts;
    void *hit_list;             // rich_hit[]
    unsigned long long *hit_count;
    uint64_t hit_capacity;
    float *hit_time;
};

}  // namespace rich
