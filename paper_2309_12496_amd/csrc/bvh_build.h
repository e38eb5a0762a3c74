// Host-side BVH4 construction (binned SAH, FP64) for librich.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

#include "rich_dev.h"

namespace rich {

struct BuildTri {
    double v[3][3];      // vertices in the local frame of the instance
    double n[3];         // unit normal of the active side, computed in FP64
    uint32_t index;      // global triangle index (primitive order of the scene)
    uint32_t material;
    int32_t group = -1;  // subtree of an instance that holds several meshes (-1: none)
};

struct BuildBox {
    double lo[3], hi[3];
};

// Build a BVH4 over `tris`, appending nodes to `nodes` and leaf-ordered
// triangles to `out`.  Returns the root node index; `depth` gets the number of
// BVH4 levels and `bounds` the AABB of all triangles.  Triangles that all
// carry a group (two or more groups) get one subtree per group.  Returns
// kEmpty if a leaf came out empty or larger than kLeafMaxTris (a builder
// fault: the tree must not be used).
uint32_t build_mesh_bvh4(std::vector<BuildTri> &tris, std::vector<Node4> &nodes, std::vector<Tri> &out, int *depth,
                         BuildBox *bounds);

// Plane of a triangle as integers: unit normal to 1e-6, plane offset to 1e-3 mm.
struct PlaneKey {
    long long nx, ny, nz, off;
    bool operator<(const PlaneKey &o) const;
};
PlaneKey plane_key(const BuildTri &t);

// Plane of each triangle: triangles with equal plane keys share a group.
// Groups are numbered in order of first appearance.  Returns the number of
// groups, or -1 once a mesh has more than `max_groups` planes.
int plane_groups(const std::vector<BuildTri> &tris, int max_groups, std::vector<int> &grp);

// Build the top-level BVH4 over instance boxes; leaves reference instances.
// The nodes are appended to `nodes` starting at the current size.
uint32_t build_top_bvh4(const std::vector<BuildBox> &boxes, std::vector<Node4> &nodes, int *depth);

// Runs fn(k) for k in [0, n) on up to max_threads host threads, the calling
// one included.  The first exception a call throws is rethrown here once
// every thread has been joined (the remaining calls are skipped); if no
// thread can be started, the calling thread runs them all.
template <class F>
void parallel_for(size_t n, size_t max_threads, F &&fn) {
    std::atomic<size_t> next{0};
    std::exception_ptr err;
    std::mutex mu;
    auto work = [&]() {
        for (size_t k; (k = next.fetch_add(1)) < n;) {
            try {
                fn(k);
            } catch (...) {
                std::lock_guard<std::mutex> lock(mu);
                if (!err) err = std::current_exception();
                next.store(n);
            }
        }
    };
    std::vector<std::thread> pool;
    try {
        for (size_t i = 1; i < std::min(n, max_threads); ++i) pool.emplace_back(work);
    } catch (...) {
    }
    work();
    for (auto &th : pool) th.join();
    if (err) std::rethrow_exception(err);
}

// Outward-rounded FP32 bounds with a small pad against FP32 slab-test rounding.
float lower_f32(double x);
float upper_f32(double x);

}  // namespace rich
