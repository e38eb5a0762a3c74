// Scene construction: validation, instance grouping, BVH4 builds, FP32 upload.
#include "scene.h"

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <atomic>
#include <algorithm>
#include <map>

#include "bvh_build.h"
#include "kernels.h"

namespace rich {

static thread_local std::string g_last_error;

rich_status set_error(rich_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

const char *last_error() { return g_last_error.c_str(); }

namespace {

constexpr int kMaxMeshPlanes = 64;     // a fixed mesh of at most this many planes is grouped by plane

bool finite3(const double *p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

double norm3(const double *p) { return std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]); }

bool unit3(const double *p) { return finite3(p) && std::fabs(norm3(p) - 1.0) < 1e-9; }

rich_status check_table(int n, const double *x, const double *y, const char *what) {
    if (n < 1 || n > kMaxTable || !x || !y) return set_error(RICH_EINVAL, "%s: need 1..%d table nodes", what, kMaxTable);
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || y[i] < 0.0 || y[i] > 1.0)
            return set_error(RICH_EINVAL, "%s: node %d not finite or outside [0,1]", what, i);
        if (i > 0 && !(x[i] > x[i - 1])) return set_error(RICH_EINVAL, "%s: wavelengths must increase", what);
    }
    return RICH_OK;
}

rich_status validate(const rich_scene_desc *d) {
    if (d->n_materials < 1 || !d->materials) return set_error(RICH_EINVAL, "scene needs at least one material");
    for (int i = 0; i < d->n_materials; ++i) {
        const rich_material &m = d->materials[i];
        if (m.kind != RICH_MAT_MIRROR && m.kind != RICH_MAT_ABSORBER)
            return set_error(RICH_EINVAL, "material %d: unknown kind %d", i, m.kind);
        rich_status st = check_table(m.n_refl, m.refl_lambda, m.refl_value, "reflectivity table");
        if (st) return st;
    }
    if (d->n_segments < 0 || d->n_segments > RICH_MAX_SEGMENTS || (d->n_segments > 0 && !d->segments))
        return set_error(RICH_EINVAL, "n_segments must be in 0..%d", RICH_MAX_SEGMENTS);
    for (int k = 0; k < d->n_segments; ++k) {
        const rich_segment &s = d->segments[k];
        if (!finite3(s.pivot) || !unit3(s.u0) || !unit3(s.e1) || !unit3(s.e2) || !(s.radius0 > 0))
            return set_error(RICH_EINVAL, "segment %d: pivot must be finite, u0/e1/e2 unit, radius0 > 0", k);
        if (d->params) {
            for (int m = 0; m < 6; ++m)
                if (!std::isfinite(d->params[6 * k + m])) return set_error(RICH_EINVAL, "segment %d: parameter not finite", k);
            if (!(d->params[6 * k + 2] > 0)) return set_error(RICH_EINVAL, "segment %d: radius must be > 0", k);
        }
    }
    if (d->n_caps < 0 || (d->n_caps > 0 && !d->caps)) return set_error(RICH_EINVAL, "bad caps");
    for (int i = 0; i < d->n_caps; ++i) {
        const rich_cap &c = d->caps[i];
        if (c.segment < 0 || c.segment >= d->n_segments) return set_error(RICH_EINVAL, "cap %d: segment out of range", i);
        if (c.material < 0 || c.material >= d->n_materials) return set_error(RICH_EINVAL, "cap %d: bad material", i);
        if (!finite3(c.origin) || !unit3(c.axis_a) || !unit3(c.axis_b))
            return set_error(RICH_EINVAL, "cap %d: frame must be finite with unit axes", i);
        if (!(c.bounds[0] < c.bounds[1]) || !(c.bounds[2] < c.bounds[3]))
            return set_error(RICH_EINVAL, "cap %d: empty aperture cell", i);
    }
    if (d->n_rects < 0 || (d->n_rects > 0 && !d->rects)) return set_error(RICH_EINVAL, "bad rects");
    for (int i = 0; i < d->n_rects; ++i) {
        const rich_rect &r = d->rects[i];
        if (r.material < 0 || r.material >= d->n_materials) return set_error(RICH_EINVAL, "rect %d: bad material", i);
        if (!finite3(r.center) || !unit3(r.normal) || !unit3(r.axis_u) || !unit3(r.axis_v) || !(r.half[0] > 0) ||
            !(r.half[1] > 0))
            return set_error(RICH_EINVAL, "rect %d: bad frame or size", i);
    }
    if (d->n_meshes < 0 || (d->n_meshes > 0 && !d->meshes)) return set_error(RICH_EINVAL, "bad meshes");
    // Sizes first, before any vertex is read.  Traversal forms triangle and
    // node byte offsets in 32 bits (64-byte triangles, 128-byte nodes), so a
    // scene holds fewer than 2^26 triangles and 2^25 BVH nodes.
    int64_t total = 0;
    for (int i = 0; i < d->n_meshes; ++i) {
        const rich_mesh &m = d->meshes[i];
        if (m.n_tri < 0 || (m.n_tri > 0 && !m.vertices)) return set_error(RICH_EINVAL, "mesh %d: bad triangle array", i);
        if (m.material < 0 || m.material >= d->n_materials) return set_error(RICH_EINVAL, "mesh %d: bad material", i);
        if (m.segment < -1 || m.segment >= d->n_segments) return set_error(RICH_EINVAL, "mesh %d: segment out of range", i);
        total += m.n_tri;
        if (total >= kMaxTriangles) return set_error(RICH_EINVAL, "too many triangles (limit 2^26 - 1)");
    }
    for (int i = 0; i < d->n_meshes; ++i) {
        const rich_mesh &m = d->meshes[i];
        for (int64_t q = 0; q < 9 * m.n_tri; ++q)
            if (!std::isfinite(m.vertices[q])) return set_error(RICH_EINVAL, "mesh %d: non-finite vertex", i);
    }
    const rich_detector &t = d->detector;
    if (!finite3(t.center) || !unit3(t.normal) || !unit3(t.axis_u) || !unit3(t.axis_v) || !(t.half[0] > 0) ||
        !(t.half[1] > 0) || !(t.pitch > 0) || t.nx <= 0 || t.ny <= 0)
        return set_error(RICH_EINVAL, "detector: bad frame, size, pitch or pixel counts");
    rich_status st = check_table(t.n_qe, t.qe_lambda, t.qe_value, "QE table");
    if (st) return st;
    if (d->has_box) {
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(d->box_lo[a]) || !std::isfinite(d->box_hi[a]) || !(d->box_lo[a] < d->box_hi[a]))
                return set_error(RICH_EINVAL, "box: need finite lo < hi");
    }
    if (d->max_bounces < 0 || d->max_bounces > 1024) return set_error(RICH_EINVAL, "max_bounces must be in 0..1024");
    if (!(d->t_min >= 0) || !std::isfinite(d->t_min)) return set_error(RICH_EINVAL, "t_min must be finite and >= 0");
    return RICH_OK;
}

void to_f3(float *dst, const double *src) {
    dst[0] = (float)src[0];
    dst[1] = (float)src[1];
    dst[2] = (float)src[2];
}

template <class T>
rich_status upload(T **dptr, const T *host, size_t count, int64_t *bytes) {
    size_t sz = sizeof(T) * (count > 0 ? count : 1);
    if (hipMalloc(dptr, sz) != hipSuccess) return set_error(RICH_ENOMEM, "hipMalloc of %zu bytes failed", sz);
    *bytes += (int64_t)sz;
    if (count > 0 && hipMemcpy(*dptr, host, sizeof(T) * count, hipMemcpyHostToDevice) != hipSuccess)
        return set_error(RICH_EDEVICE, "hipMemcpy to the device failed");
    return RICH_OK;
}

struct InstanceBuild {
    int segment = -1;
    double origin[3] = {0, 0, 0};
    std::vector<BuildTri> tris;
};

}  // namespace

void free_scene(rich_scene *s) {
    if (!s) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    for (StreamWork &w : s->slots) {
        if (w.graph_exec) (void)hipGraphExecDestroy(w.graph_exec);
        if (w.graph) (void)hipGraphDestroy(w.graph);
        if (w.capture_stream) (void)hipStreamDestroy(w.capture_stream);
        if (w.partials) (void)hipFree(w.partials);
        if (w.order) (void)hipFree(w.order);
        if (w.sorted) (void)hipFree(w.sorted);
    }
    void *ptrs[] = {s->d_nodes, s->d_tris, s->d_inst, s->d_caps, s->d_caps_static, s->d_segs, s->d_rects,
                    s->d_mats, s->d_det, s->d_params, s->d_status, s->d_counters, s->d_tallies};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    (void)hipSetDevice(prev);
    delete s;
}

namespace {

// The body of build_scene; *made is the scene once allocated, so that a
// throw past this point can free it.
rich_status build_scene_impl(const rich_scene_desc *d, int device, rich_scene **out, rich_scene **made) {
    auto t0 = std::chrono::steady_clock::now();
    rich_status st = validate(d);
    if (st) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return set_error(RICH_EINVAL, "device %d not available (%d devices)", device, ndev);
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return set_error(RICH_EDEVICE, "hipSetDevice(%d) failed", device);

    // the no-allocation adjoint's partial-sum array: its address on this
    // device, looked up once while the device is current
    float *scratch_addr = nullptr;
    if (adjoint_scratch(device, &scratch_addr) != hipSuccess) {
        (void)hipSetDevice(prev);
        return set_error(RICH_EDEVICE, "device %d: address of the adjoint scratch array not found", device);
    }

    rich_scene *s = new rich_scene();
    *made = s;
    s->device = device;
    (void)hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, device);
    int64_t bytes = 0;

    // --- group meshes into instances
    std::vector<InstanceBuild> inst;
    std::vector<int> seg_inst(d->n_segments, -1);
    int static_inst = -1;
    // Every fixed mesh goes into one instance.  Its triangles are grouped:
    // per plane for a mesh made of a few planes (planes shared by several
    // meshes, like tiles of one flat mirror, form one group), and per mesh
    // for the others.  The BVH builder gives the large groups (an
    // enclosure's walls) subtrees of their own and the rest one subtree.
    std::map<PlaneKey, int> plane_group;
    int n_groups = 0;
    uint32_t tri_index = 0;
    for (int i = 0; i < d->n_meshes; ++i) {
        const rich_mesh &m = d->meshes[i];
        if (m.n_tri == 0) continue;
        int k;
        if (m.segment >= 0) {
            if (seg_inst[m.segment] < 0) {
                seg_inst[m.segment] = (int)inst.size();
                inst.emplace_back();
                inst.back().segment = m.segment;
            }
            k = seg_inst[m.segment];
        } else {
            if (static_inst < 0) {
                static_inst = (int)inst.size();
                inst.emplace_back();
            }
            k = static_inst;
        }
        std::vector<BuildTri> mt;
        mt.reserve((size_t)m.n_tri);
        for (int64_t q = 0; q < m.n_tri; ++q) {
            BuildTri t;
            const double *v = m.vertices + 9 * q;
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) t.v[a][c] = v[3 * a + c];
            double e1[3] = {t.v[1][0] - t.v[0][0], t.v[1][1] - t.v[0][1], t.v[1][2] - t.v[0][2]};
            double e2[3] = {t.v[2][0] - t.v[0][0], t.v[2][1] - t.v[0][1], t.v[2][2] - t.v[0][2]};
            double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
            double len = norm3(n);
            for (int a = 0; a < 3; ++a) t.n[a] = len > 0 ? n[a] / len : 0.0;
            t.index = tri_index++;
            t.material = (uint32_t)m.material;
            mt.push_back(t);
        }
        if (m.segment < 0) {
            std::vector<int> grp;
            if (plane_groups(mt, kMaxMeshPlanes, grp) > 0) {
                for (auto &t : mt) {
                    t.group = plane_group.emplace(plane_key(t), n_groups).first->second;
                    if (t.group == n_groups) ++n_groups;
                }
            } else {
                for (auto &t : mt) t.group = n_groups;
                ++n_groups;
            }
        }
        inst[k].tris.insert(inst[k].tris.end(), mt.begin(), mt.end());
    }
    // local frames: segment instances around the pivot, fixed ones around their box centre
    for (auto &in : inst) {
        if (in.segment >= 0) {
            for (int a = 0; a < 3; ++a) in.origin[a] = d->segments[in.segment].pivot[a];
        } else {
            double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
            for (auto &t : in.tris)
                for (int m = 0; m < 3; ++m)
                    for (int a = 0; a < 3; ++a) {
                        lo[a] = std::min(lo[a], t.v[m][a]);
                        hi[a] = std::max(hi[a], t.v[m][a]);
                    }
            for (int a = 0; a < 3; ++a) in.origin[a] = 0.5 * (lo[a] + hi[a]);
        }
        for (auto &t : in.tris)
            for (int m = 0; m < 3; ++m)
                for (int a = 0; a < 3; ++a) t.v[m][a] -= in.origin[a];
    }

    // --- BVHs: one per instance, then the top level in front
    std::vector<Node4> inst_nodes;
    std::vector<Tri> tris;
    std::vector<Instance> hinst(inst.size());
    std::vector<BuildBox> world_boxes(inst.size());
    std::vector<uint32_t> roots(inst.size());
    int max_inst_depth = 0;
    // instance BVHs are independent: build them on host threads into their own
    // arrays, then concatenate in instance order with node and triangle
    // offsets rebased, which gives the same arrays as building them in turn
    std::vector<std::vector<Node4>> knodes(inst.size());
    std::vector<std::vector<Tri>> ktris(inst.size());
    std::vector<int> kdepth(inst.size(), 0);
    std::vector<BuildBox> kbox(inst.size());
    {
        const size_t hw = std::max(1u, std::thread::hardware_concurrency());
        parallel_for(inst.size(), std::min<size_t>(hw, 16), [&](size_t k) {
            roots[k] = build_mesh_bvh4(inst[k].tris, knodes[k], ktris[k], &kdepth[k], &kbox[k]);
        });
    }
    for (size_t k = 0; k < inst.size(); ++k) {
        if (roots[k] == kEmpty) {
            free_scene(s);
            (void)hipSetDevice(prev);
            return set_error(RICH_EINVAL, "internal check failed: instance %zu's BVH has a leaf of 0 or more than %u triangles",
                             k, kLeafMaxTris);
        }
    }
    for (size_t k = 0; k < inst.size(); ++k) {
        const uint32_t node_base = (uint32_t)inst_nodes.size(), tri_base = (uint32_t)tris.size();
        for (Node4 nd : knodes[k]) {
            for (int c = 0; c < 4; ++c) {
                if (nd.child[c] == kEmpty) continue;
                nd.child[c] += (nd.child[c] & kLeafBit) ? tri_base : node_base;   // leaf: first triangle (< 2^27)
            }
            inst_nodes.push_back(nd);
        }
        tris.insert(tris.end(), ktris[k].begin(), ktris[k].end());
        std::vector<Node4>().swap(knodes[k]);
        std::vector<Tri>().swap(ktris[k]);
        roots[k] += node_base;
        const int depth = kdepth[k];
        const BuildBox &lb = kbox[k];
        max_inst_depth = std::max(max_inst_depth, depth);
        Instance &h = hinst[k];
        std::memset(&h, 0, sizeof h);
        for (int a = 0; a < 9; ++a) h.m[a] = h.rot[a] = (a % 4 == 0) ? 1.0f : 0.0f;
        to_f3(h.org, inst[k].origin);
        h.scale = 1.0f;
        h.segment = inst[k].segment;
        for (int a = 0; a < 3; ++a) {
            h.loc_lo[a] = lower_f32(lb.lo[a]);
            h.loc_hi[a] = upper_f32(lb.hi[a]);
            world_boxes[k].lo[a] = lb.lo[a] + inst[k].origin[a];
            world_boxes[k].hi[a] = lb.hi[a] + inst[k].origin[a];
            h.lo[a] = lower_f32(world_boxes[k].lo[a]);
            h.hi[a] = upper_f32(world_boxes[k].hi[a]);
        }
    }
    std::vector<Node4> nodes;
    int top_depth = 0;
    if (!inst.empty()) build_top_bvh4(world_boxes, nodes, &top_depth);
    uint32_t n_top = (uint32_t)nodes.size();
    for (auto &nd : inst_nodes) {
        for (int c = 0; c < 4; ++c)
            if (nd.child[c] != kEmpty && !(nd.child[c] & kLeafBit)) nd.child[c] += n_top;
        nodes.push_back(nd);
    }
    for (size_t k = 0; k < inst.size(); ++k) hinst[k].root = roots[k] + n_top;
    s->n_top = (int32_t)n_top;

    // --- analytic primitives, materials, detector, segments
    std::vector<MatDev> mats(d->n_materials);
    for (int i = 0; i < d->n_materials; ++i) {
        const rich_material &m = d->materials[i];
        MatDev &md = mats[i];
        std::memset(&md, 0, sizeof md);
        md.kind = m.kind;
        md.n = m.n_refl;
        for (int q = 0; q < m.n_refl; ++q) {
            md.x[q] = (float)m.refl_lambda[q];
            md.y[q] = (float)m.refl_value[q];
            if (q + 1 < m.n_refl)
                md.s[q] = (float)((m.refl_value[q + 1] - m.refl_value[q]) / (m.refl_lambda[q + 1] - m.refl_lambda[q]));
        }
    }
    std::vector<RectDev> rects(d->n_rects);
    for (int i = 0; i < d->n_rects; ++i) {
        const rich_rect &r = d->rects[i];
        RectDev &rd = rects[i];
        std::memset(&rd, 0, sizeof rd);
        to_f3(rd.c, r.center);
        to_f3(rd.n, r.normal);
        to_f3(rd.u, r.axis_u);
        to_f3(rd.v, r.axis_v);
        rd.material = r.material;
        rd.hu = (float)r.half[0];
        rd.hv = (float)r.half[1];
    }
    DetDev det;
    std::memset(&det, 0, sizeof det);
    const rich_detector &t = d->detector;
    to_f3(det.c, t.center);
    to_f3(det.n, t.normal);
    to_f3(det.u, t.axis_u);
    to_f3(det.v, t.axis_v);
    det.hu = (float)t.half[0];
    det.hv = (float)t.half[1];
    det.pitch = (float)t.pitch;
    det.act_hu = (float)(0.5 * t.nx * t.pitch);
    det.act_hv = (float)(0.5 * t.ny * t.pitch);
    det.nx = t.nx;
    det.ny = t.ny;
    det.n_qe = t.n_qe;
    det.inv_pitch = (float)(1.0 / t.pitch);
    for (int q = 0; q < t.n_qe; ++q) {
        det.qe_x[q] = (float)t.qe_lambda[q];
        det.qe_y[q] = (float)t.qe_value[q];
        if (q + 1 < t.n_qe)
            det.qe_s[q] = (float)((t.qe_value[q + 1] - t.qe_value[q]) / (t.qe_lambda[q + 1] - t.qe_lambda[q]));
    }
    std::vector<SegDev> segs(d->n_segments);
    std::vector<float> params(6 * (size_t)d->n_segments);
    for (int k = 0; k < d->n_segments; ++k) {
        const rich_segment &g = d->segments[k];
        for (int a = 0; a < 3; ++a) {
            segs[k].pivot[a] = g.pivot[a];
            segs[k].u0[a] = g.u0[a];
            segs[k].e1[a] = g.e1[a];
            segs[k].e2[a] = g.e2[a];
        }
        segs[k].r0 = g.radius0;
        for (int m = 0; m < 6; ++m)
            params[6 * k + m] = d->params ? (float)d->params[6 * k + m] : (m == 2 ? (float)g.radius0 : 0.0f);
    }
    std::vector<CapStatic> caps_static(d->n_caps);
    for (int i = 0; i < d->n_caps; ++i) {
        const rich_cap &c = d->caps[i];
        CapStatic &cs = caps_static[i];
        cs.segment = c.segment;
        cs.material = c.material;
        for (int a = 0; a < 3; ++a) {
            cs.O[a] = c.origin[a];
            cs.A[a] = c.axis_a[a];
            cs.B[a] = c.axis_b[a];
        }
        for (int a = 0; a < 4; ++a) cs.bounds[a] = c.bounds[a];
    }

    if (nodes.size() >= (size_t)kMaxNodes) {
        free_scene(s);
        (void)hipSetDevice(prev);
        return set_error(RICH_EINVAL, "BVH of %zu nodes (limit 2^25 - 1)", nodes.size());
    }

    // --- upload
    if ((st = upload(&s->d_nodes, nodes.data(), nodes.size(), &bytes)) ||
        (st = upload(&s->d_tris, tris.data(), tris.size(), &bytes)) ||
        (st = upload(&s->d_inst, hinst.data(), hinst.size(), &bytes)) ||
        (st = upload(&s->d_caps_static, caps_static.data(), caps_static.size(), &bytes)) ||
        (st = upload(&s->d_segs, segs.data(), segs.size(), &bytes)) ||
        (st = upload(&s->d_rects, rects.data(), rects.size(), &bytes)) ||
        (st = upload(&s->d_mats, mats.data(), mats.size(), &bytes)) ||
        (st = upload(&s->d_det, &det, 1, &bytes)) ||
        (st = upload(&s->d_params, params.data(), params.size(), &bytes))) {
        free_scene(s);
        (void)hipSetDevice(prev);
        return st;
    }
    std::vector<CapDev> zero_caps(d->n_caps);
    unsigned int zero_status = 0;
    std::vector<unsigned long long> zero_counter((size_t)kStreamSlots * kBatchCounters, 0ull);
    std::vector<unsigned long long> zero_tally((size_t)kStreamSlots * kTallyWords, 0ull);
    if ((st = upload(&s->d_caps, zero_caps.data(), zero_caps.size(), &bytes)) ||
        (st = upload(&s->d_status, &zero_status, 1, &bytes)) ||
        (st = upload(&s->d_counters, zero_counter.data(), zero_counter.size(), &bytes)) ||
        (st = upload(&s->d_tallies, zero_tally.data(), zero_tally.size(), &bytes))) {
        free_scene(s);
        (void)hipSetDevice(prev);
        return st;
    }
    for (int k = 0; k < kStreamSlots; ++k) {
        s->slots[k].counter = s->d_counters + (size_t)k * kBatchCounters;
        s->slots[k].tally = s->d_tallies + (size_t)k * kTallyWords;
    }
    PrepareArgs pa{s->d_segs, s->d_caps_static, s->d_params, s->d_caps, d->n_caps, s->d_inst,
                   (int32_t)inst.size(), s->d_nodes, (int32_t)n_top};
    if (launch_prepare(pa, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        free_scene(s);
        (void)hipSetDevice(prev);
        return set_error(RICH_EDEVICE, "parameter kernel failed");
    }

    DevScene &S = s->dev;
    S.caps = s->d_caps;
    S.rects = s->d_rects;
    S.mats = s->d_mats;
    S.nodes = s->d_nodes;
    S.tris = s->d_tris;
    S.inst = s->d_inst;
    S.det = s->d_det;
    S.status = s->d_status;
    S.tally = nullptr;   // the launching stream's fate-count slots, set per call
    S.n_caps = d->n_caps;
    S.n_rects = d->n_rects;
    S.n_mats = d->n_materials;
    S.n_inst = (int32_t)inst.size();
    S.has_mesh = inst.empty() ? 0 : 1;
    S.has_box = d->has_box ? 1 : 0;
    // a scene of one instance starts in it: the top-level node would only hold its box
    S.top_root = inst.size() == 1 ? make_inst(0) : 0;
    S.max_bounces = d->max_bounces;
    S.t_min = (float)d->t_min;
    S.prim_det = (uint32_t)(d->n_caps + d->n_rects);
    S.prim_box = S.prim_det + 1;
    S.prim_tri = S.prim_det + 2;
    for (int a = 0; a < 3; ++a) {
        S.box_lo[a] = (float)d->box_lo[a];
        S.box_hi[a] = (float)d->box_hi[a];
    }
    S.n_seg = d->n_segments;
    for (int i = 0; i < d->n_materials; ++i) s->mat_kind.push_back(d->materials[i].kind);
    s->n_segments = d->n_segments;
    s->nx = t.nx;
    s->ny = t.ny;

    s->stats.n_triangles = (int64_t)tris.size();
    s->stats.n_nodes = (int64_t)nodes.size();
    s->stats.n_instances = (int32_t)inst.size();
    s->stats.max_depth = inst.empty() ? 0 : top_depth + max_inst_depth;
    s->stats.device_bytes = bytes;
    s->stats.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    (void)hipSetDevice(prev);
    *out = s;
    return RICH_OK;
}

}  // namespace

rich_status build_scene(const rich_scene_desc *d, int device, rich_scene **out) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    rich_scene *made = nullptr;
    try {
        return build_scene_impl(d, device, out, &made);
    } catch (...) {
        // host allocation or thread failure during the build: free what was made
        if (made && *out != made) free_scene(made);
        (void)hipSetDevice(prev);
        throw;
    }
}

}  // namespace rich
