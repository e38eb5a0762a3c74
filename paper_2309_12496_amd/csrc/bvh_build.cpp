// Binned-SAH BVH builder: a binary tree built in FP64 over triangle centroids,
// collapsed into 4-wide nodes whose children are the (up to) four largest
// descendants, stored depth-first with FP32 boxes rounded outward.
#include "bvh_build.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <limits>
#include <map>
#include <thread>
#include <tuple>

namespace rich {

namespace {

constexpr int kBins = 32;
constexpr uint32_t kLeafSize = 4;      // largest leaf
constexpr uint32_t kAlwaysLeaf = 1;    // nodes of this many triangles or fewer are leaves
// Surface-area cost of testing a node against that of one triangle: a range
// of up to kLeafSize triangles becomes a leaf when testing them all costs no
// more than the node plus the children the split would make.
constexpr double kNodeCost = 1.0;
// A group of an instance with several meshes gets its own subtree when its
// box has at least this fraction of the instance box's surface area.
constexpr double kLargeGroupArea = 0.1;
// Ranges of at least kParallelMin triangles in the top kParallelDepth levels
// of a subtree build their right half on a thread of its own.
constexpr int kParallelDepth = 3;
constexpr uint32_t kParallelMin = 16384;

struct BNode {
    BuildBox box;
    int left = -1, right = -1;
    uint32_t first = 0, count = 0;
};

BuildBox empty_box() {
    BuildBox b;
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = std::numeric_limits<double>::infinity();
        b.hi[a] = -std::numeric_limits<double>::infinity();
    }
    return b;
}

void grow(BuildBox &b, const double *p) {
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = std::min(b.lo[a], p[a]);
        b.hi[a] = std::max(b.hi[a], p[a]);
    }
}

void grow(BuildBox &b, const BuildBox &o) {
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = std::min(b.lo[a], o.lo[a]);
        b.hi[a] = std::max(b.hi[a], o.hi[a]);
    }
}

double area(const BuildBox &b) {
    double dx = b.hi[0] - b.lo[0], dy = b.hi[1] - b.lo[1], dz = b.hi[2] - b.lo[2];
    if (dx < 0 || dy < 0 || dz < 0) return 0.0;
    return 2.0 * (dx * dy + dy * dz + dz * dx);
}

struct Builder {
    std::vector<BuildTri> &tris;
    std::vector<BuildBox> tbox;
    std::vector<double> cen;  // [n][3]
    std::vector<uint32_t> idx;
    std::vector<BNode> bn;

    explicit Builder(std::vector<BuildTri> &t) : tris(t) {
        size_t n = t.size();
        tbox.resize(n);
        cen.resize(3 * n);
        idx.resize(n);
        for (size_t i = 0; i < n; ++i) {
            BuildBox b = empty_box();
            for (int m = 0; m < 3; ++m) grow(b, t[i].v[m]);
            tbox[i] = b;
            for (int a = 0; a < 3; ++a) cen[3 * i + a] = 0.5 * (b.lo[a] + b.hi[a]);
            idx[i] = (uint32_t)i;
        }
    }

    // Given groups: an instance that holds several meshes gets one subtree per
    // large group (a plane whose box has at least kLargeGroupArea of the
    // instance box's surface area, such as an enclosure's wall), and one SAH
    // subtree over all the other triangles, so that the SAH never mixes a thin
    // enclosure wall into a mirror's boxes.  Nodes whose box holds the ray's
    // origin cannot be culled; with the walls as the only separate subtrees
    // the fewest such nodes stand above them.  Returns the root, or -1 unless
    // every triangle has a group and two or more subtrees result.
    int build_grouped() {
        std::map<int, int> dense;
        std::vector<int> grp(tris.size());
        for (size_t i = 0; i < tris.size(); ++i) {
            if (tris[i].group < 0) return -1;
            grp[i] = dense.emplace(tris[i].group, (int)dense.size()).first->second;
        }
        const int ng = (int)dense.size();
        std::vector<BuildBox> gbox(ng, empty_box());
        BuildBox all = empty_box();
        for (size_t i = 0; i < tris.size(); ++i) {
            grow(gbox[grp[i]], tbox[i]);
            grow(all, tbox[i]);
        }
        std::vector<int> sub(ng, -1);   // subtree of each group; the rest share the last one
        int n_sub = 0;
        for (int g = 0; g < ng; ++g)
            if (area(gbox[g]) >= kLargeGroupArea * area(all)) sub[g] = n_sub++;
        const bool rest = n_sub < ng;
        for (int g = 0; g < ng; ++g)
            if (sub[g] < 0) sub[g] = n_sub;
        if (n_sub + (rest ? 1 : 0) < 2) return -1;
        for (auto &v : grp) v = sub[v];
        return chain_groups(grp, n_sub + (rest ? 1 : 0));
    }

    // Planar grouping: a mesh made of a few planes (an enclosure's walls) gets
    // one subtree per plane, the planes chained under the root so that the
    // BVH4 root holds thin per-wall boxes rather than half-box boxes that
    // contain every ray starting inside.  Returns the root, or -1 if the mesh
    // is not a union of 2..64 planes.
    int build_planar() {
        std::vector<int> grp;
        int ng = plane_groups(tris, 64, grp);
        if (ng < 2) return -1;
        return chain_groups(grp, ng);
    }

    // Subtrees of the groups, largest first, chained under the root.
    int chain_groups(const std::vector<int> &grp, int ng) {
        std::vector<uint32_t> gcount(ng, 0);
        for (int g : grp) ++gcount[g];
        std::vector<int> order(ng);
        for (int g = 0; g < ng; ++g) order[g] = g;
        std::sort(order.begin(), order.end(), [&](int a, int b) { return gcount[a] > gcount[b] || (gcount[a] == gcount[b] && a < b); });
        std::vector<int> rank(ng);
        for (int r = 0; r < ng; ++r) rank[order[r]] = r;
        std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return rank[grp[a]] < rank[grp[b]]; });
        std::vector<uint32_t> start(ng + 1, 0);
        for (int r = 0; r < ng; ++r) start[r + 1] = start[r] + gcount[order[r]];
        // the groups' subtrees are independent: built on host threads into
        // their own node lists, then appended in group order with their
        // indices rebased (the same tree as building them in turn)
        std::vector<std::vector<BNode>> local(ng);
        std::vector<int> root(ng);
        parallel_for((size_t)ng, std::min(16u, std::max(1u, std::thread::hardware_concurrency())), [&](size_t r) {
            root[r] = build_into(local[r], start[r], start[r + 1] - start[r]);
        });
        for (int r = 0; r < ng; ++r) {
            const int base = (int)bn.size();
            for (BNode b : local[r]) {
                if (b.left >= 0) {
                    b.left += base;
                    b.right += base;
                }
                bn.push_back(b);
            }
            root[r] += base;
        }
        return chain(0, ng, start, root);
    }

    int chain(int r, int ng, const std::vector<uint32_t> &start, const std::vector<int> &root) {
        if (r == ng - 1) return root[r];
        int me = (int)bn.size();
        bn.emplace_back();
        int l = root[r];
        int rt = chain(r + 1, ng, start, root);
        BuildBox box = bn[l].box;
        grow(box, bn[rt].box);
        bn[me].box = box;
        bn[me].first = start[r];
        bn[me].count = start[ng] - start[r];
        bn[me].left = l;
        bn[me].right = rt;
        return me;
    }

    int build(uint32_t first, uint32_t count) { return build_into(bn, first, count); }

    // Binary SAH subtree over idx[first, first + count), appended to `out`
    // (child indices are positions in `out`).  The right halves of the top
    // kParallelDepth splits of large ranges are built on host threads of
    // their own and appended after the left ones: the same tree, so the same
    // emitted arrays, as building them in turn.
    int build_into(std::vector<BNode> &out, uint32_t first, uint32_t count, int depth = 0) {
        int me = (int)out.size();
        out.emplace_back();
        BuildBox box = empty_box(), cb = empty_box();
        for (uint32_t q = first; q < first + count; ++q) {
            grow(box, tbox[idx[q]]);
            grow(cb, &cen[3 * idx[q]]);
        }
        out[me].box = box;
        out[me].first = first;
        out[me].count = count;
        if (count <= kAlwaysLeaf) return me;

        // binned SAH over the centroid bounds
        double best_cost = std::numeric_limits<double>::infinity();
        int best_axis = -1, best_split = -1;
        for (int a = 0; a < 3; ++a) {
            double ext = cb.hi[a] - cb.lo[a];
            if (!(ext > 0)) continue;
            double scale = kBins / ext;
            BuildBox bb[kBins];
            uint32_t bc[kBins] = {};
            for (int k = 0; k < kBins; ++k) bb[k] = empty_box();
            for (uint32_t q = first; q < first + count; ++q) {
                int k = std::min(kBins - 1, (int)((cen[3 * idx[q] + a] - cb.lo[a]) * scale));
                ++bc[k];
                grow(bb[k], tbox[idx[q]]);
            }
            double right_area[kBins];
            uint32_t right_cnt[kBins];
            BuildBox acc = empty_box();
            uint32_t cnt = 0;
            for (int k = kBins - 1; k > 0; --k) {
                grow(acc, bb[k]);
                cnt += bc[k];
                right_area[k] = area(acc);
                right_cnt[k] = cnt;
            }
            acc = empty_box();
            cnt = 0;
            for (int k = 0; k < kBins - 1; ++k) {
                grow(acc, bb[k]);
                cnt += bc[k];
                if (cnt == 0 || right_cnt[k + 1] == 0) continue;
                double cost = area(acc) * cnt + right_area[k + 1] * right_cnt[k + 1];
                if (cost < best_cost) {
                    best_cost = cost;
                    best_axis = a;
                    best_split = k + 1;
                }
            }
        }
        if (count <= kLeafSize && (best_axis < 0 || area(box) * count <= kNodeCost * area(box) + best_cost)) return me;
        uint32_t mid;
        if (best_axis >= 0) {
            double ext = cb.hi[best_axis] - cb.lo[best_axis];
            double scale = kBins / ext;
            auto it = std::partition(idx.begin() + first, idx.begin() + first + count, [&](uint32_t i) {
                int k = std::min(kBins - 1, (int)((cen[3 * i + best_axis] - cb.lo[best_axis]) * scale));
                return k < best_split;
            });
            mid = (uint32_t)(it - idx.begin());
        } else {
            mid = first + count / 2;  // all centroids coincide: split the index range
        }
        if (mid == first || mid == first + count) mid = first + count / 2;
        int l, r;
        if (depth < kParallelDepth && count >= kParallelMin) {
            std::vector<BNode> right;
            int r_local = -1;
            parallel_for(2, 2, [&](size_t half) {
                if (half == 0) l = build_into(out, first, mid - first, depth + 1);
                else r_local = build_into(right, mid, first + count - mid, depth + 1);
            });
            const int base = (int)out.size();
            for (BNode b : right) {
                if (b.left >= 0) {
                    b.left += base;
                    b.right += base;
                }
                out.push_back(b);
            }
            r = r_local + base;
        } else {
            l = build_into(out, first, mid - first, depth + 1);
            r = build_into(out, mid, first + count - mid, depth + 1);
        }
        out[me].left = l;
        out[me].right = r;
        return me;
    }
};

void set_child_box(Node4 &nd, int k, const BuildBox &b) {
    nd.lox[k] = lower_f32(b.lo[0]);
    nd.loy[k] = lower_f32(b.lo[1]);
    nd.loz[k] = lower_f32(b.lo[2]);
    nd.hix[k] = upper_f32(b.hi[0]);
    nd.hiy[k] = upper_f32(b.hi[1]);
    nd.hiz[k] = upper_f32(b.hi[2]);
}

void clear_node(Node4 &nd) {
    for (int k = 0; k < 4; ++k) {
        nd.lox[k] = nd.loy[k] = nd.loz[k] = std::numeric_limits<float>::infinity();
        nd.hix[k] = nd.hiy[k] = nd.hiz[k] = -std::numeric_limits<float>::infinity();
        nd.child[k] = kEmpty;
        nd.pad[k] = 0;
    }
}

// Pick up to four descendants of a binary node: repeatedly open the largest internal one.
std::vector<int> gather4(const std::vector<BNode> &bn, int root) {
    std::vector<int> kids;
    if (bn[root].left < 0) {
        kids.push_back(root);
        return kids;
    }
    kids = {bn[root].left, bn[root].right};
    while (kids.size() < 4) {
        int pick = -1;
        double best = -1;
        for (size_t k = 0; k < kids.size(); ++k) {
            const BNode &c = bn[kids[k]];
            if (c.left >= 0 && area(c.box) > best) {
                best = area(c.box);
                pick = (int)k;
            }
        }
        if (pick < 0) break;
        int c = kids[pick];
        kids.erase(kids.begin() + pick);
        kids.push_back(bn[c].left);
        kids.push_back(bn[c].right);
    }
    return kids;
}

struct Emitter {
    const std::vector<BNode> &bn;
    const std::vector<uint32_t> &idx;
    const std::vector<BuildTri> &tris;
    std::vector<Node4> &nodes;
    std::vector<Tri> &out;
    int max_depth = 0;

    bool bad_leaf = false;   // a leaf the reference encoding cannot hold

    uint32_t leaf_ref(const BNode &b) {
        if (b.count == 0 || b.count > kLeafMaxTris) bad_leaf = true;
        uint32_t first = (uint32_t)out.size();
        for (uint32_t q = b.first; q < b.first + b.count; ++q) {
            const BuildTri &t = tris[idx[q]];
            Tri r;
            for (int a = 0; a < 3; ++a) {
                r.v0[a] = (float)t.v[0][a];
                r.v1[a] = (float)t.v[1][a];
                r.v2[a] = (float)t.v[2][a];
                r.n[a] = (float)t.n[a];
            }
            r.index = t.index;
            r.material = t.material;
            r.pad0 = r.pad1 = 0;
            out.push_back(r);
        }
        return make_leaf(first, b.count);
    }

    uint32_t emit(int root, int depth) {
        max_depth = std::max(max_depth, depth);
        uint32_t me = (uint32_t)nodes.size();
        nodes.emplace_back();
        clear_node(nodes[me]);
        std::vector<int> kids = gather4(bn, root);
        for (size_t k = 0; k < kids.size(); ++k) {
            const BNode &c = bn[kids[k]];
            uint32_t ref = (c.left < 0) ? leaf_ref(c) : emit(kids[k], depth + 1);
            Node4 &nd = nodes[me];
            set_child_box(nd, (int)k, c.box);
            nd.child[k] = ref;
        }
        return me;
    }
};

}  // namespace

bool PlaneKey::operator<(const PlaneKey &o) const {
    return std::tie(nx, ny, nz, off) < std::tie(o.nx, o.ny, o.nz, o.off);
}

PlaneKey plane_key(const BuildTri &t) {
    double off = t.n[0] * t.v[0][0] + t.n[1] * t.v[0][1] + t.n[2] * t.v[0][2];
    return {std::llround(t.n[0] * 1e6), std::llround(t.n[1] * 1e6), std::llround(t.n[2] * 1e6), std::llround(off * 1e3)};
}

int plane_groups(const std::vector<BuildTri> &tris, int max_groups, std::vector<int> &grp) {
    std::map<PlaneKey, int> key_to_group;
    grp.resize(tris.size());
    for (size_t i = 0; i < tris.size(); ++i) {
        auto it = key_to_group.find(plane_key(tris[i]));
        if (it == key_to_group.end()) {
            if ((int)key_to_group.size() >= max_groups) return -1;
            it = key_to_group.emplace(plane_key(tris[i]), (int)key_to_group.size()).first;
        }
        grp[i] = it->second;
    }
    return (int)key_to_group.size();
}

float lower_f32(double x) {
    double pad = 1e-3 + 1e-6 * std::fabs(x);
    float f = (float)(x - pad);
    while ((double)f > x - pad) f = std::nextafter(f, -std::numeric_limits<float>::infinity());
    return f;
}

float upper_f32(double x) {
    double pad = 1e-3 + 1e-6 * std::fabs(x);
    float f = (float)(x + pad);
    while ((double)f < x + pad) f = std::nextafter(f, std::numeric_limits<float>::infinity());
    return f;
}

uint32_t build_mesh_bvh4(std::vector<BuildTri> &tris, std::vector<Node4> &nodes, std::vector<Tri> &out, int *depth,
                         BuildBox *bounds) {
    Builder b(tris);
    b.bn.reserve(2 * tris.size() / kLeafSize + 2);
    int top = b.build_grouped();
    if (top < 0) top = b.build_planar();
    if (top < 0) top = b.build(0, (uint32_t)tris.size());
    if (bounds) *bounds = b.bn[top].box;
    Emitter e{b.bn, b.idx, tris, nodes, out};
    uint32_t root = e.emit(top, 1);
    if (depth) *depth = e.max_depth;
    return e.bad_leaf ? kEmpty : root;
}

uint32_t build_top_bvh4(const std::vector<BuildBox> &boxes, std::vector<Node4> &nodes, int *depth) {
    // binary median splits over instance boxes (largest extent first), one instance per leaf
    std::vector<BuildTri> pseudo(boxes.size());
    for (size_t i = 0; i < boxes.size(); ++i) {
        for (int a = 0; a < 3; ++a) {
            pseudo[i].v[0][a] = boxes[i].lo[a];
            pseudo[i].v[1][a] = boxes[i].hi[a];
            pseudo[i].v[2][a] = boxes[i].lo[a];
            pseudo[i].n[a] = 0;
        }
        pseudo[i].index = (uint32_t)i;
        pseudo[i].material = 0;
    }
    // one instance per leaf: build with leaf size 1 by splitting until single
    struct TopBuilder {
        std::vector<BuildTri> &t;
        std::vector<uint32_t> idx;
        std::vector<BNode> bn;
        int build(uint32_t first, uint32_t count, const std::vector<BuildBox> &bx) {
            int me = (int)bn.size();
            bn.emplace_back();
            BuildBox box = empty_box();
            for (uint32_t q = first; q < first + count; ++q) grow(box, bx[idx[q]]);
            bn[me].box = box;
            bn[me].first = first;
            bn[me].count = count;
            if (count == 1) return me;
            int axis = 0;
            double ext[3];
            for (int a = 0; a < 3; ++a) ext[a] = box.hi[a] - box.lo[a];
            if (ext[1] > ext[axis]) axis = 1;
            if (ext[2] > ext[axis]) axis = 2;
            std::sort(idx.begin() + first, idx.begin() + first + count, [&](uint32_t a, uint32_t b) {
                double ca = bx[a].lo[axis] + bx[a].hi[axis], cb = bx[b].lo[axis] + bx[b].hi[axis];
                return ca < cb || (ca == cb && a < b);
            });
            uint32_t mid = first + count / 2;
            int l = build(first, mid - first, bx);
            int r = build(mid, first + count - mid, bx);
            bn[me].left = l;
            bn[me].right = r;
            return me;
        }
    } tb{pseudo, {}, {}};
    // An instance whose box has at least kLargeGroupArea of the scene box's
    // area (the fixed meshes of an enclosure, which hold every ray origin)
    // hangs from the root itself: a node above it would hold the origin too
    // and be visited by every query.  Up to three such instances, the rest
    // in a median-split tree beside them.
    BuildBox all = empty_box();
    for (const auto &b : boxes) grow(all, b);
    std::vector<uint32_t> large, rest;
    for (size_t i = 0; i < boxes.size(); ++i)
        (area(boxes[i]) >= kLargeGroupArea * area(all) ? large : rest).push_back((uint32_t)i);
    int top;
    if (!large.empty() && large.size() <= 3 && !rest.empty()) {
        tb.idx = large;
        tb.idx.insert(tb.idx.end(), rest.begin(), rest.end());
        const uint32_t nl = (uint32_t)large.size();
        top = tb.build(nl, (uint32_t)rest.size(), boxes);
        for (int k = (int)nl - 1; k >= 0; --k) {
            const int leaf = tb.build((uint32_t)k, 1, boxes);
            const int me = (int)tb.bn.size();
            tb.bn.emplace_back();
            BuildBox box = tb.bn[leaf].box;
            grow(box, tb.bn[top].box);
            tb.bn[me].box = box;
            tb.bn[me].first = (uint32_t)k;
            tb.bn[me].count = (uint32_t)boxes.size() - (uint32_t)k;
            tb.bn[me].left = leaf;
            tb.bn[me].right = top;
            top = me;
        }
    } else {
        tb.idx.resize(boxes.size());
        for (size_t i = 0; i < boxes.size(); ++i) tb.idx[i] = (uint32_t)i;
        top = tb.build(0, (uint32_t)boxes.size(), boxes);
    }

    int maxd = 0;
    std::vector<Node4> &nd = nodes;
    struct TopEmit {
        const std::vector<BNode> &bn;
        const std::vector<uint32_t> &idx;
        std::vector<Node4> &nodes;
        int &maxd;
        uint32_t emit(int root, int depth) {
            maxd = std::max(maxd, depth);
            uint32_t me = (uint32_t)nodes.size();
            nodes.emplace_back();
            clear_node(nodes[me]);
            std::vector<int> kids;
            if (bn[root].left < 0) kids.push_back(root);
            else kids = gather4(bn, root);
            for (size_t k = 0; k < kids.size(); ++k) {
                const BNode &c = bn[kids[k]];
                uint32_t ref = (c.left < 0) ? make_inst(idx[c.first]) : emit(kids[k], depth + 1);
                set_child_box(nodes[me], (int)k, c.box);
                nodes[me].child[k] = ref;
            }
            return me;
        }
    } te{tb.bn, tb.idx, nd, maxd};
    uint32_t root = te.emit(top, 1);
    if (depth) *depth = maxd;
    return root;
}

}  // namespace rich
