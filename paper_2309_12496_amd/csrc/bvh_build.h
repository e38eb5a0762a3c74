// Host-side BVH4 construction (binned SAH, FP64) for librich.
#pragma once

#include <cstdint>
#include <vector>

#include "rich_dev.h"

namespace rich {

struct BuildTri {
    double v[3][3];      // vertices in the local frame of the instance
    double n[3];         // unit normal of the active side, computed in FP64
    uint32_t index;      // global triangle index (primitive order of the scene)
    uint32_t material;
};

struct BuildBox {
    double lo[3], hi[3];
};

// Build a BVH4 over `tris`, appending nodes to `nodes` and leaf-ordered
// triangles to `out`.  Returns the root node index; `depth` gets the number of
// BVH4 levels and `bounds` the AABB of all triangles.
uint32_t build_mesh_bvh4(std::vector<BuildTri> &tris, std::vector<Node4> &nodes, std::vector<Tri> &out, int *depth,
                         BuildBox *bounds);

// Build the top-level BVH4 over instance boxes; leaves reference instances.
// The nodes are appended to `nodes` starting at the current size.
uint32_t build_top_bvh4(const std::vector<BuildBox> &boxes, std::vector<Node4> &nodes, int *depth);

// Outward-rounded FP32 bounds with a small pad against FP32 slab-test rounding.
float lower_f32(double x);
float upper_f32(double x);

}  // namespace rich
