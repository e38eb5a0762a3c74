// C ABI of librich: argument checks, source set-up, launches, graph capture,
// autotuning and status.  No exception crosses these functions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/rich.h"
#include "kernels.h"
#include "scene.h"

namespace rich {
const char *last_error();
}

using namespace rich;

namespace {

// Makes the scene's device current for the lifetime of a call.
struct DeviceGuard {
    int prev = 0, dev = 0;
    explicit DeviceGuard(int d) : dev(d) {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev != dev) (void)hipSetDevice(prev);
    }
};

#define RICH_HIP(call)                                                                            \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return set_error(RICH_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

rich_status check_spectrum(double n, double lmin, double lmax) {
    if (!(n > 0) || !std::isfinite(n)) return set_error(RICH_EINVAL, "n_radiator must be finite and > 0");
    if (!(lmin > 0) || !(lmax > lmin) || !std::isfinite(lmax))
        return set_error(RICH_EINVAL, "need 0 < lambda_min < lambda_max");
    return RICH_OK;
}

double table_at(int n, const double *x, const double *y, double l) {
    if (l <= x[0]) return y[0];
    if (l >= x[n - 1]) return y[n - 1];
    int i = 0;
    while (i + 1 < n - 1 && l >= x[i + 1]) ++i;
    return y[i] + (y[i + 1] - y[i]) * (l - x[i]) / (x[i + 1] - x[i]);
}

rich_status check_dispersion(const rich_dispersion &dp) {
    if (dp.n_nodes < 0 || dp.n_nodes > kMaxTable) return set_error(RICH_EINVAL, "dispersion: 0..%d nodes", kMaxTable);
    if (dp.n_nodes == 0) return RICH_OK;
    if (!dp.lambda || !dp.index) return set_error(RICH_EINVAL, "dispersion: lambda and index arrays needed");
    for (int k = 0; k < dp.n_nodes; ++k) {
        if (!std::isfinite(dp.lambda[k]) || !std::isfinite(dp.index[k]) || !(dp.index[k] >= 1.0))
            return set_error(RICH_EINVAL, "dispersion: finite wavelengths and indices >= 1");
        if (k > 0 && !(dp.lambda[k] > dp.lambda[k - 1]))
            return set_error(RICH_EINVAL, "dispersion: wavelengths must increase");
    }
    return RICH_OK;
}

// Largest index over [lmin, lmax]: n is piecewise linear, so at an end or a node.
double dispersion_nmax(const rich_dispersion &dp, double lmin, double lmax) {
    double m = std::max(table_at(dp.n_nodes, dp.lambda, dp.index, lmin), table_at(dp.n_nodes, dp.lambda, dp.index, lmax));
    for (int k = 0; k < dp.n_nodes; ++k)
        if (dp.lambda[k] > lmin && dp.lambda[k] < lmax) m = std::max(m, dp.index[k]);
    return m;
}

// Device copy of a dispersion table: nodes, n - 1 (kept apart from the 1 so
// FP32 holds it to ~1e-10) and the segment slopes.
rich_status set_dispersion(const rich_dispersion &dp, double lmin, double lmax, DevSource &ds) {
    rich_status st = check_dispersion(dp);
    if (st) return st;
    ds.n_disp = dp.n_nodes;
    for (int k = 0; k < dp.n_nodes; ++k) {
        ds.disp_x[k] = (float)dp.lambda[k];
        ds.disp_m[k] = (float)(dp.index[k] - 1.0);
        ds.disp_s[k] = k + 1 < dp.n_nodes
                           ? (float)((dp.index[k + 1] - dp.index[k]) / (dp.lambda[k + 1] - dp.lambda[k]))
                           : 0.0f;
    }
    ds.disp_nmax = dp.n_nodes > 0 ? dispersion_nmax(dp, lmin, lmax) : 0.0;
    return RICH_OK;
}

// Host FP64 set-up of a single track source: unit direction, its orthonormal
// basis (Duff et al., JCGT 2017), the Cherenkov cone cos = 1/(n beta) and the
// wavelength inverse-CDF constants, rounded once to FP32.
rich_status make_track_source(const rich_source *src, DevSource &ds) {
    std::memset(&ds, 0, sizeof ds);
    if (src->kind == RICH_SRC_EXPLICIT) {
        if (!src->dev_o || !src->dev_d || !src->dev_lambda)
            return set_error(RICH_EINVAL, "explicit source needs dev_o, dev_d and dev_lambda");
        ds.kind = 2;
        ds.ex_o = src->dev_o;
        ds.ex_d = src->dev_d;
        ds.ex_l = src->dev_lambda;
        // group index for arrival times: n_radiator when it is a refractive index, else vacuum
        ds.ng_const = (std::isfinite(src->n_radiator) && src->n_radiator >= 1.0) ? (float)src->n_radiator : 1.0f;
        if (src->dispersion.n_nodes > 0) return set_dispersion(src->dispersion, 0.0, 0.0, ds);
        return RICH_OK;
    }
    if (src->kind != RICH_SRC_TRACK) return set_error(RICH_EINVAL, "unknown source kind %d", src->kind);
    rich_status st = check_spectrum(src->n_radiator, src->lambda_min, src->lambda_max);
    if (st) return st;
    const double *o = src->origin, *t = src->direction;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(o[a]) || !std::isfinite(t[a])) return set_error(RICH_EINVAL, "track origin/direction not finite");
    if (!std::isfinite(src->length) || src->length < 0) return set_error(RICH_EINVAL, "track length must be >= 0");
    double nb = src->n_radiator * src->beta;
    if (src->dispersion.n_nodes > 0) {
        // with dispersion the largest index over the band must be above threshold
        st = set_dispersion(src->dispersion, src->lambda_min, src->lambda_max, ds);
        if (st) return st;
        nb = ds.disp_nmax * src->beta;
    }
    if (!(nb > 1.0) || !std::isfinite(nb)) return set_error(RICH_EINVAL, "n*beta = %g: no Cherenkov light", nb);
    double len = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    if (!(len > 0)) return set_error(RICH_EINVAL, "track direction is zero");
    double T[3] = {t[0] / len, t[1] / len, t[2] / len};
    double sgn = std::copysign(1.0, T[2]);
    double a = -1.0 / (sgn + T[2]);
    double b = T[0] * T[1] * a;
    double E1[3] = {1.0 + sgn * T[0] * T[0] * a, sgn * b, -sgn * T[0]};
    double E2[3] = {b, sgn + T[1] * T[1] * a, -T[1]};
    double c = 1.0 / nb;
    ds.kind = 0;
    for (int q = 0; q < 3; ++q) {
        ds.P0[q] = (float)o[q];
        ds.T[q] = (float)T[q];
        ds.E1[q] = (float)E1[q];
        ds.E2[q] = (float)E2[q];
    }
    ds.length = (float)src->length;
    ds.beta = (float)src->beta;
    ds.ng_const = (float)src->n_radiator;
    ds.cos_t = (float)c;
    ds.sin_t = (float)std::sqrt((1.0 - c) * (1.0 + c));
    ds.inv_lmin = (float)(1.0 / src->lambda_min);
    ds.inv_span = (float)(1.0 / src->lambda_min - 1.0 / src->lambda_max);
    return RICH_OK;
}

rich_status set_prefilter(const rich_scene *s, const rich_prefilter &pf, DevSource &ds) {
    ds.prefilter = pf.enabled ? 1 : 0;
    ds.pf_n = 0;
    if (!pf.enabled) return RICH_OK;
    if (pf.n_materials < 0 || pf.n_materials > 4) return set_error(RICH_EINVAL, "prefilter: 0..4 materials");
    for (int k = 0; k < pf.n_materials; ++k) {
        int m = pf.materials[k];
        if (m < 0 || m >= s->dev.n_mats || s->mat_kind[m] != RICH_MAT_MIRROR)
            return set_error(RICH_EINVAL, "prefilter: material %d is not a mirror of this scene", m);
        ds.pf_mats[k] = m;
    }
    ds.pf_n = pf.n_materials;
    return RICH_OK;
}

rich_status make_batch_source(const rich_batch *b, DevSource &ds) {
    std::memset(&ds, 0, sizeof ds);
    if (!b->dev_tracks || !b->dev_offsets || b->n_tracks < 1)
        return set_error(RICH_EINVAL, "batch needs tracks, offsets and n_tracks >= 1");
    rich_status st = check_spectrum(b->n_radiator, b->lambda_min, b->lambda_max);
    if (st) return st;
    ds.kind = 1;
    ds.tracks = reinterpret_cast<const float *>(b->dev_tracks);
    ds.offsets = b->dev_offsets;
    ds.n_tracks = b->n_tracks;
    ds.n_radiator = b->n_radiator;
    ds.ng_const = (float)b->n_radiator;
    ds.inv_lmin = (float)(1.0 / b->lambda_min);
    ds.inv_span = (float)(1.0 / b->lambda_min - 1.0 / b->lambda_max);
    // per-track velocities live on the device: the tracks must be above
    // threshold (n_max beta > 1), which the host cannot check here
    if (b->dispersion.n_nodes > 0) return set_dispersion(b->dispersion, b->lambda_min, b->lambda_max, ds);
    return RICH_OK;
}

DevOutputs make_outputs(const rich_outputs *o) {
    DevOutputs d;
    std::memset(&d, 0, sizeof d);
    if (!o) return d;
    d.fate = o->fate;
    d.pixel = o->pixel;
    d.hit_xyz = o->hit_xyz;
    d.hit_uv = o->hit_uv;
    d.histogram = o->histogram;
    d.fate_counts = o->fate_counts;
    d.hit_list = o->hit_list;
    d.hit_count = o->hit_count;
    d.hit_capacity = o->hit_list_capacity;
    d.hit_time = o->hit_time;
    return d;
}

rich_status check_outputs(const rich_outputs *o) {
    if (!o) return RICH_OK;
    if (o->hit_list && !o->hit_count) return set_error(RICH_EINVAL, "hit_list needs hit_count");
    return RICH_OK;
}

// ------------------------------------------------------------- autotune cache

std::string arch_name(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    return std::string(p.gcnArchName);
}

std::string tune_key(const rich_scene *s, uint64_t n) {
    int tb = 0;
    for (int64_t x = s->stats.n_triangles; x > 1; x >>= 1) ++tb;
    int nb = 0;
    for (uint64_t x = n; x > 1; x >>= 1) ++nb;
    std::ostringstream k;
    k << arch_name(s->device) << "/cu" << s->n_cu << "/tri2^" << tb << "/caps" << s->dev.n_caps << "/n2^" << nb;
    return k.str();
}

bool load_tuning_file(const std::string &key, rich_tuning *t) {
    const char *path = std::getenv("RICH_TUNE_CACHE");
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        // one entry per line: "key": [block, chunk, blocks_per_cu],
        size_t q0 = line.find('"'), q1 = line.find('"', q0 + 1);
        if (q0 == std::string::npos || q1 == std::string::npos) continue;
        if (line.substr(q0 + 1, q1 - q0 - 1) != key) continue;
        int b, c, p;
        if (std::sscanf(line.c_str() + q1 + 1, " : [%d , %d , %d]", &b, &c, &p) == 3) {
            t->block = b;
            t->chunk = c;
            t->blocks_per_cu = p;
            return true;
        }
    }
    return false;
}

void store_tuning_file(const std::string &key, const rich_tuning &t) {
    const char *path = std::getenv("RICH_TUNE_CACHE");
    if (!path) return;
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line)) {
            size_t q0 = line.find('"'), q1 = line.find('"', q0 + 1);
            if (q0 == std::string::npos || q1 == std::string::npos) continue;
            if (line.substr(q0 + 1, q1 - q0 - 1) == key) continue;
            std::string e = line;
            while (!e.empty() && (e.back() == ',' || e.back() == ' ')) e.pop_back();
            keep.push_back(e);
        }
    }
    char buf[512];
    std::snprintf(buf, sizeof buf, "  \"%s\": [%d, %d, %d]", key.c_str(), t.block, t.chunk, t.blocks_per_cu);
    keep.push_back(buf);
    std::ofstream f(path);
    f << "{\n";
    for (size_t i = 0; i < keep.size(); ++i) f << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
    f << "}\n";
}

rich_status valid_tuning(const rich_tuning *t) {
    if (t->block != 64 && t->block != 128 && t->block != 256 && t->block != 512)
        return set_error(RICH_EINVAL, "tuning.block must be 64, 128, 256 or 512");
    if (t->chunk < 64 || t->chunk % 64 != 0 || t->chunk > 65536)
        return set_error(RICH_EINVAL, "tuning.chunk must be a multiple of 64 in 64..65536");
    if (t->blocks_per_cu < 1 || t->blocks_per_cu > 64) return set_error(RICH_EINVAL, "tuning.blocks_per_cu in 1..64");
    return RICH_OK;
}

int grid_of(const rich_scene *s, const rich_tuning &t) { return std::max(1, s->n_cu * t.blocks_per_cu); }

// The workspace of the launches on `stream`: the slot the stream took at its
// first launch on this scene, or a free one (no allocation: the counters
// and fate-count slots of every slot are made with the scene).  The caller
// holds the scene's lock.
rich_status stream_slot(rich_scene *s, hipStream_t stream, StreamWork **out) {
    for (StreamWork &w : s->slots)
        if (w.used && w.stream == stream) {
            *out = &w;
            return RICH_OK;
        }
    for (StreamWork &w : s->slots)
        if (!w.used) {
            w.used = true;
            w.stream = stream;
            *out = &w;
            return RICH_OK;
        }
    return set_error(RICH_ESTATE, "more than %d streams launch on this scene", kStreamSlots);
}

rich_status run_autotune(rich_scene *s, const DevSource &src, uint64_t n, uint64_t seed, rich_tuning *best_out) {
    uint64_t n_t = std::min<uint64_t>(n, 4000000ull);
    if (n_t == 0) {
        *best_out = rich_tuning{256, 256, 4, 0};
        return RICH_OK;
    }
    // scratch outputs so the caller's accumulating outputs stay untouched
    uint8_t *fate = nullptr;
    int32_t *pixel = nullptr;
    float *xyz = nullptr, *uv = nullptr, *time = nullptr;
    uint32_t *hist = nullptr;
    unsigned long long *counts = nullptr, *counter = nullptr, *tally = nullptr;
    size_t nh = (size_t)s->nx * s->ny;
    hipError_t e = hipSuccess;
    e = e == hipSuccess ? hipMalloc(&fate, n_t) : e;
    e = e == hipSuccess ? hipMalloc(&pixel, 4 * n_t) : e;
    e = e == hipSuccess ? hipMalloc(&xyz, 12 * n_t) : e;
    e = e == hipSuccess ? hipMalloc(&uv, 8 * n_t) : e;
    e = e == hipSuccess ? hipMalloc(&time, 4 * n_t) : e;
    e = e == hipSuccess ? hipMalloc(&hist, 4 * nh) : e;
    e = e == hipSuccess ? hipMalloc(&counts, 8 * RICH_N_FATES) : e;
    e = e == hipSuccess ? hipMalloc(&counter, 8 * kBatchCounters) : e;
    e = e == hipSuccess ? hipMalloc(&tally, 8 * kTallyWords) : e;
    e = e == hipSuccess ? hipMemset(tally, 0, 8 * kTallyWords) : e;
    hipEvent_t a = nullptr, b = nullptr;
    e = e == hipSuccess ? hipEventCreate(&a) : e;
    e = e == hipSuccess ? hipEventCreate(&b) : e;
    rich_status st = RICH_OK;
    if (e != hipSuccess) {
        st = set_error(RICH_ENOMEM, "autotune scratch allocation failed: %s", hipGetErrorString(e));
    } else {
        DevOutputs out;
        std::memset(&out, 0, sizeof out);
        out.fate = fate;
        out.pixel = pixel;
        out.hit_xyz = xyz;
        out.hit_uv = uv;
        out.hit_time = time;
        out.histogram = hist;
        out.fate_counts = counts;
        DevScene dv = s->dev;   // fate-count slots of its own
        dv.tally = tally;
        float best = INFINITY;
        rich_tuning bt{256, 256, 4, 0};
        const int blocks[] = {64, 128, 256, 512};
        const int chunks[] = {64, 128, 256, 512, 1024};
        for (int blk : blocks) {
            int max_bpc = (int)std::min<long>(16, (160L * 1024) / (long)batch_lds_bytes(blk));
            for (int bpc = 1; bpc <= max_bpc; bpc *= 2) {
                for (int ch : chunks) {
                    rich_tuning t{blk, ch, bpc, 0};
                    float tmin = INFINITY;
                    for (int rep = 0; rep < 3 && st == RICH_OK; ++rep) {
                        hipError_t r1 = launch_fill_u64(counter, kBatchCounters, nullptr);
                        (void)hipEventRecord(a, nullptr);
                        hipError_t r2 = launch_batch(dv, src, out, n_t, seed, counter, blk, ch, grid_of(s, t), false, nullptr);
                        (void)hipEventRecord(b, nullptr);
                        if (r1 != hipSuccess || r2 != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
                            st = set_error(RICH_EDEVICE, "autotune launch failed");
                            break;
                        }
                        float ms = 0;
                        (void)hipEventElapsedTime(&ms, a, b);
                        if (rep > 0) tmin = std::min(tmin, ms);
                    }
                    if (st != RICH_OK) break;
                    if (tmin < best) {
                        best = tmin;
                        bt = t;
                    }
                }
            }
        }
        *best_out = bt;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    void *ptrs[] = {fate, pixel, xyz, uv, time, hist, counts, counter, tally};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    return st;
}

}  // namespace

extern "C" {

const char *rich_last_error(void) { return last_error(); }

const char *rich_version(void) { return "richprop 0.1 (gfx950)"; }

rich_status rich_build_scene(const rich_scene_desc *desc, int device, rich_scene **out) {
    if (!out) return set_error(RICH_EINVAL, "out is NULL");
    *out = nullptr;
    if (!desc) return set_error(RICH_EINVAL, "desc is NULL");
    try {
        return build_scene(desc, device, out);
    } catch (const std::bad_alloc &) {
        return set_error(RICH_ENOMEM, "host allocation failed while building the scene");
    } catch (...) {
        return set_error(RICH_EINVAL, "scene build failed");
    }
}

rich_status rich_destroy_scene(rich_scene *s) {
    if (!s) return set_error(RICH_EINVAL, "scene is NULL");
    free_scene(s);
    return RICH_OK;
}

rich_status rich_scene_info(const rich_scene *s, rich_scene_stats *out) {
    if (!s || !out) return set_error(RICH_EINVAL, "scene and out must not be NULL");
    *out = s->stats;
    return RICH_OK;
}

rich_status rich_set_mirror_params(rich_scene *s, const float *dev_params, hipStream_t stream) {
    if (!s) return set_error(RICH_EINVAL, "scene is NULL");
    if (s->n_segments == 0) return set_error(RICH_ESTATE, "scene has no parametrised segments");
    if (!dev_params) return set_error(RICH_EINVAL, "dev_params is NULL");
    DeviceGuard g(s->device);
    RICH_HIP(hipMemcpyAsync(s->d_params, dev_params, sizeof(float) * 6 * s->n_segments, hipMemcpyDeviceToDevice,
                            stream));
    PrepareArgs pa{s->d_segs, s->d_caps_static, s->d_params, s->d_caps, s->dev.n_caps, s->d_inst, s->dev.n_inst,
                   s->d_nodes, s->n_top};
    RICH_HIP(launch_prepare(pa, stream));
    return RICH_OK;
}

rich_status rich_fit_step(rich_scene *s, const rich_fit *fit, const float *dev_p0, const float *dev_grad,
                          const float *dev_loss, float *dev_state, float *dev_params, float *dev_losses,
                          float *dev_cut, hipStream_t stream) {
    if (!s || !fit) return set_error(RICH_EINVAL, "scene and fit must not be NULL");
    if (s->n_segments == 0) return set_error(RICH_ESTATE, "scene has no parametrised segments");
    if (!dev_p0 || !dev_grad || !dev_loss || !dev_state)
        return set_error(RICH_EINVAL, "dev_p0, dev_grad, dev_loss and dev_state are needed");
    if (fit->n_steps < 1) return set_error(RICH_EINVAL, "fit: n_steps >= 1");
    if (!(fit->lr >= 0) || !(fit->lr_final >= 0) || !std::isfinite(fit->lr) || !std::isfinite(fit->lr_final))
        return set_error(RICH_EINVAL, "fit: finite step sizes >= 0");
    if (!(fit->beta1 >= 0 && fit->beta1 < 1) || !(fit->beta2 >= 0 && fit->beta2 < 1))
        return set_error(RICH_EINVAL, "fit: beta1 and beta2 in [0, 1)");
    if (!(fit->eps > 0) || !std::isfinite(fit->eps)) return set_error(RICH_EINVAL, "fit: eps > 0");
    for (int c = 0; c < 6; ++c)
        if (!(fit->scale[c] > 0) || !std::isfinite(fit->scale[c])) return set_error(RICH_EINVAL, "fit: scale > 0");
    if (dev_cut && (!std::isfinite(fit->outlier_cut) || !std::isfinite(fit->cut_floor)))
        return set_error(RICH_EINVAL, "fit: finite outlier_cut and cut_floor");
    DeviceGuard g(s->device);
    FitArgs a;
    a.n_par = 6 * s->n_segments;
    a.n_steps = fit->n_steps;
    a.lr = fit->lr;
    a.lr_final = fit->lr_final;
    a.beta1 = fit->beta1;
    a.beta2 = fit->beta2;
    a.eps = fit->eps;
    for (int c = 0; c < 6; ++c) {
        a.scale[c] = (float)fit->scale[c];
        a.free[c] = fit->free[c] ? 1 : 0;
    }
    a.outlier_cut = (float)fit->outlier_cut;
    a.cut_floor = (float)fit->cut_floor;
    a.p0 = dev_p0;
    a.grad = dev_grad;
    a.loss = dev_loss;
    a.state = dev_state;
    a.params = s->d_params;
    a.params_out = dev_params;
    a.losses = dev_losses;
    a.cut = dev_cut;
    RICH_HIP(launch_fit_step(a, stream));
    PrepareArgs pa{s->d_segs, s->d_caps_static, s->d_params, s->d_caps, s->dev.n_caps, s->d_inst, s->dev.n_inst,
                   s->d_nodes, s->n_top};
    RICH_HIP(launch_prepare(pa, stream));
    return RICH_OK;
}

rich_status rich_propagate(rich_scene *s, const rich_source *src, uint64_t n_photons, uint64_t seed,
                           uint64_t first_photon_id, const rich_outputs *out, hipStream_t stream) {
    if (!s || !src) return set_error(RICH_EINVAL, "scene and source must not be NULL");
    if (first_photon_id + n_photons < first_photon_id) return set_error(RICH_ERANGE, "photon id range wraps 2^64");
    if (n_photons > (1ull << 40)) return set_error(RICH_ERANGE, "n_photons too large for one call");
    rich_status st = check_outputs(out);
    if (st) return st;
    DevSource ds;
    if ((st = make_track_source(src, ds))) return st;
    if ((st = set_prefilter(s, src->prefilter, ds))) return st;
    if (n_photons == 0) return RICH_OK;
    try {
        std::lock_guard<std::mutex> lock(s->mu);
        StreamWork *w = nullptr;
        if ((st = stream_slot(s, stream, &w))) return st;
        DeviceGuard g(s->device);
        DevScene dv = s->dev;
        dv.tally = w->tally;
        if (forward_sorted(dv, ds)) {
            // the stream's order buffer, grown to the largest chunk so far
            const uint64_t need = n_photons < kSortedChunk ? n_photons : kSortedChunk;
            if (need > w->sorted_count) {
                if (w->sorted) (void)hipFree(w->sorted);
                w->sorted = nullptr;
                w->sorted_count = 0;
                if (hipMalloc(&w->sorted, need * sizeof(uint32_t)) != hipSuccess)
                    return set_error(RICH_ENOMEM, "forward order buffer allocation failed");
                w->sorted_count = need;
            }
        }
        RICH_HIP(launch_forward(dv, ds, make_outputs(out), n_photons, first_photon_id, seed, s->n_cu, w->sorted,
                                w->counter, stream));
        return RICH_OK;
    } catch (...) {
        return set_error(RICH_EDEVICE, "forward launch failed");
    }
}

rich_status rich_autotune(rich_scene *s, const rich_batch *batch, uint64_t n_photons, uint64_t seed,
                          rich_tuning *out) {
    if (!s || !batch || !out) return set_error(RICH_EINVAL, "scene, batch and out must not be NULL");
    DevSource ds;
    rich_status st = make_batch_source(batch, ds);
    if (st) return st;
    if ((st = set_prefilter(s, batch->prefilter, ds))) return st;
    std::lock_guard<std::mutex> lock(s->mu);
    DeviceGuard g(s->device);
    try {
        return run_autotune(s, ds, n_photons, seed, out);
    } catch (...) {
        return set_error(RICH_ENOMEM, "autotune failed");
    }
}

rich_status rich_propagate_batch(rich_scene *s, const rich_batch *batch, uint64_t n_photons, uint64_t seed,
                                 const rich_outputs *out, const rich_tuning *tune, hipStream_t stream) {
    if (!s || !batch) return set_error(RICH_EINVAL, "scene and batch must not be NULL");
    if (n_photons > (1ull << 40)) return set_error(RICH_ERANGE, "n_photons too large for one call");
    rich_status st = check_outputs(out);
    if (st) return st;
    DevSource ds;
    if ((st = make_batch_source(batch, ds))) return st;
    if ((st = set_prefilter(s, batch->prefilter, ds))) return st;
    if (n_photons == 0) return RICH_OK;
    std::lock_guard<std::mutex> lock(s->mu);
    StreamWork *w = nullptr;
    if ((st = stream_slot(s, stream, &w))) return st;
    DeviceGuard g(s->device);
    try {
        DevScene dv = s->dev;
        dv.tally = w->tally;
        rich_tuning t;
        if (tune) {
            if ((st = valid_tuning(tune))) return st;
            t = *tune;
        } else {
            std::string key = tune_key(s, n_photons);
            auto it = s->tuned.find(key);
            if (it != s->tuned.end()) {
                t = it->second;
            } else if (!load_tuning_file(key, &t) || valid_tuning(&t) != RICH_OK) {
                RICH_HIP(hipStreamSynchronize(stream));
                if ((st = run_autotune(s, ds, n_photons, seed, &t))) return st;
                store_tuning_file(key, t);
                s->tuned[key] = t;
            } else {
                s->tuned[key] = t;
            }
        }
        DevOutputs dout = make_outputs(out);
        // Large batches on meshed scenes are processed in an order of the
        // tracks by direction dealt to the id partitions (each XCD's tracks in
        // flight then point the same way, and share L2 lines); photon ids and
        // results do not change.  Small batches do not repay its five launches.
        const bool ordered = s->dev.has_mesh && n_photons >= (1ull << 21) && batch->n_tracks >= 64;
        if (ordered) {
            const size_t need = order_buffer_bytes(batch->n_tracks);
            if (need > w->order_bytes) {
                if (w->order) (void)hipFree(w->order);
                w->order = nullptr;
                w->order_bytes = 0;
                if (hipMalloc(&w->order, need) != hipSuccess)
                    return set_error(RICH_ENOMEM, "batch order buffer allocation failed");
                w->order_bytes = need;
            }
            set_order(ds, w->order);
        }
        // the graph is reused while every launch argument is the same: compare
        // their bytes (both structs are zero-filled before they are set)
        std::string k2;
        auto put = [&](const void *p, size_t bytes) { k2.append(reinterpret_cast<const char *>(p), bytes); };
        put(&ds, sizeof ds);
        put(&dout, sizeof dout);
        put(&n_photons, sizeof n_photons);
        put(&seed, sizeof seed);
        put(&t, sizeof t);
        if (!w->graph_exec || w->graph_key != k2) {
            if (w->graph_exec) {
                (void)hipGraphExecDestroy(w->graph_exec);
                w->graph_exec = nullptr;
            }
            if (w->graph) {
                (void)hipGraphDestroy(w->graph);
                w->graph = nullptr;
            }
            if (!w->capture_stream) RICH_HIP(hipStreamCreateWithFlags(&w->capture_stream, hipStreamNonBlocking));
            RICH_HIP(hipStreamBeginCapture(w->capture_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e0 = ordered ? launch_order(ds, batch_parts(grid_of(s, t)), w->order, w->capture_stream)
                                    : hipSuccess;
            hipError_t e1 = launch_fill_u64(w->counter, kBatchCounters, w->capture_stream);
            hipError_t e2 = launch_batch(dv, ds, dout, n_photons, seed, w->counter, t.block, t.chunk,
                                         grid_of(s, t), true, w->capture_stream);
            hipGraph_t gr = nullptr;
            hipError_t e3 = hipStreamEndCapture(w->capture_stream, &gr);
            if (e0 != hipSuccess || e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
                if (gr) (void)hipGraphDestroy(gr);
                return set_error(RICH_EDEVICE, "graph capture failed");
            }
            w->graph = gr;
            RICH_HIP(hipGraphInstantiate(&w->graph_exec, w->graph, nullptr, nullptr, 0));
            w->graph_key = k2;
        }
        RICH_HIP(hipGraphLaunch(w->graph_exec, stream));
        return RICH_OK;
    } catch (...) {
        return set_error(RICH_ENOMEM, "batch launch failed");
    }
}

// Shared by both adjoint entry points: argument checks, source set-up, the
// grid, and the partial-sum buffer (the scene's, grown with hipMalloc, or the
// static per-device array when noalloc is set).
static rich_status adjoint_call(rich_scene *s, const rich_source *src, const rich_batch *batch, uint64_t n_photons,
                                uint64_t seed, uint64_t first_photon_id, const float *dev_grad_uv,
                                const float *dev_targets, const uint8_t *dev_mask, const float *dev_residual_cut,
                                float *dev_grad_params, float *dev_loss, hipStream_t stream, bool noalloc) {
    if (!s) return set_error(RICH_EINVAL, "scene is NULL");
    if ((src == nullptr) == (batch == nullptr)) return set_error(RICH_EINVAL, "give exactly one of src and batch");
    if ((dev_grad_uv == nullptr) == (dev_targets == nullptr))
        return set_error(RICH_EINVAL, "give exactly one of dev_grad_uv and dev_targets");
    if (dev_residual_cut && !dev_targets) return set_error(RICH_EINVAL, "dev_residual_cut needs dev_targets");
    if (!dev_grad_params) return set_error(RICH_EINVAL, "dev_grad_params is NULL");
    if (s->n_segments == 0) return set_error(RICH_ESTATE, "scene has no parametrised segments");
    if (first_photon_id + n_photons < first_photon_id) return set_error(RICH_ERANGE, "photon id range wraps 2^64");
    if (n_photons > (1ull << 40)) return set_error(RICH_ERANGE, "n_photons too large for one call");
    DevSource ds;
    rich_status st = src ? make_track_source(src, ds) : make_batch_source(batch, ds);
    if (st) return st;
    if ((st = set_prefilter(s, src ? src->prefilter : batch->prefilter, ds))) return st;
    if (batch && first_photon_id != 0) return set_error(RICH_EINVAL, "batch photons start at id 0");
    std::lock_guard<std::mutex> lock(s->mu);
    DeviceGuard g(s->device);
    int n_par = 6 * s->n_segments;
    const AdjointPlan plan = adjoint_plan(n_photons, n_par, s->n_cu, dev_mask != nullptr);
    float *work = nullptr;
    if (noalloc) {
        if (plan.bytes > kAdjScratchFloats * sizeof(float))
            return set_error(RICH_ERANGE,
                             "no-allocation adjoint: %zu bytes of partial sums and mask counts exceed its %zu "
                             "(fewer segments or photons, or rich_propagate_adjoint)",
                             plan.bytes, kAdjScratchFloats * sizeof(float));
        hipError_t e = adjoint_scratch(s->device, &work);
        if (e != hipSuccess)
            return set_error(RICH_EDEVICE, "adjoint scratch address: %s", hipGetErrorString(e));
    } else {
        // the stream's buffer, grown to its largest call so far: partial
        // sums, mask counts and offsets
        StreamWork *w = nullptr;
        if ((st = stream_slot(s, stream, &w))) return st;
        const size_t need = (plan.bytes + sizeof(float) - 1) / sizeof(float);
        if (need > w->partials_floats) {
            if (w->partials) (void)hipFree(w->partials);
            w->partials = nullptr;
            w->partials_floats = 0;
            if (hipMalloc(&w->partials, need * sizeof(float)) != hipSuccess)
                return set_error(RICH_ENOMEM, "adjoint work buffer allocation failed");
            w->partials_floats = need;
        }
        work = w->partials;
    }
    AdjointArgs a{dev_grad_uv, dev_targets, dev_mask, dev_residual_cut, nullptr, dev_grad_params, dev_loss, n_par,
                  nullptr, nullptr};
    RICH_HIP(launch_adjoint(s->dev, ds, a, n_photons, first_photon_id, seed, plan, work, stream));
    return RICH_OK;
}

rich_status rich_propagate_adjoint(rich_scene *s, const rich_source *src, const rich_batch *batch,
                                   uint64_t n_photons, uint64_t seed, uint64_t first_photon_id,
                                   const float *dev_grad_uv, const float *dev_targets, const uint8_t *dev_mask,
                                   const float *dev_residual_cut, float *dev_grad_params, float *dev_loss,
                                   hipStream_t stream) {
    try {
        return adjoint_call(s, src, batch, n_photons, seed, first_photon_id, dev_grad_uv, dev_targets, dev_mask,
                            dev_residual_cut, dev_grad_params, dev_loss, stream, false);
    } catch (...) {
        return set_error(RICH_EDEVICE, "adjoint launch failed");
    }
}

rich_status rich_propagate_adjoint_noalloc(rich_scene *s, const rich_source *src, const rich_batch *batch,
                                           uint64_t n_photons, uint64_t seed, uint64_t first_photon_id,
                                           const float *dev_grad_uv, const float *dev_targets,
                                           const uint8_t *dev_mask, const float *dev_residual_cut,
                                           float *dev_grad_params, float *dev_loss, hipStream_t stream) {
    try {
        return adjoint_call(s, src, batch, n_photons, seed, first_photon_id, dev_grad_uv, dev_targets, dev_mask,
                            dev_residual_cut, dev_grad_params, dev_loss, stream, true);
    } catch (...) {
        return set_error(RICH_EDEVICE, "adjoint launch failed");
    }
}

// Gauss-Legendre rule on [-1, 1]: nodes are the roots of P_n, found by Newton
// iteration from Chebyshev-like starting points; w = 2 / ((1 - x^2) P_n'(x)^2).
static void gauss_legendre(int n, double *x, double *w) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;               // P_0, P_1, then the three-term recurrence
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

rich_status rich_cherenkov_yield(const rich_dispersion *dispersion, double n_radiator, double beta,
                                 double lambda_min, double lambda_max, double *photons_per_mm) {
    if (!photons_per_mm) return set_error(RICH_EINVAL, "photons_per_mm is NULL");
    if (!(beta > 0) || !std::isfinite(beta)) return set_error(RICH_EINVAL, "beta must be finite and > 0");
    rich_dispersion none{0, 0, nullptr, nullptr};
    const rich_dispersion &dp = dispersion ? *dispersion : none;
    rich_status st = check_dispersion(dp);
    if (st) return st;
    if (dp.n_nodes == 0 && (st = check_spectrum(n_radiator, lambda_min, lambda_max))) return st;
    if (!(lambda_min > 0) || !(lambda_max > lambda_min) || !std::isfinite(lambda_max))
        return set_error(RICH_EINVAL, "need 0 < lambda_min < lambda_max");
    auto index = [&](double l) { return dp.n_nodes > 0 ? table_at(dp.n_nodes, dp.lambda, dp.index, l) : n_radiator; };
    auto weight = [&](double l) {
        double n = index(l), w = 1.0 - 1.0 / (beta * beta * n * n);
        return w > 0.0 ? w / (l * l) : 0.0;
    };
    // pieces on which n is linear: the band split at the table nodes, each
    // split again where n beta crosses 1 (the integrand has a kink there)
    std::vector<double> cuts{lambda_min};
    for (int k = 0; k < dp.n_nodes; ++k)
        if (dp.lambda[k] > lambda_min && dp.lambda[k] < lambda_max) cuts.push_back(dp.lambda[k]);
    cuts.push_back(lambda_max);
    constexpr int kPoints = 16;
    double gx[kPoints], gw[kPoints];
    gauss_legendre(kPoints, gx, gw);
    double integral = 0.0;   // of w / lambda^2 over lambda in nm
    for (size_t q = 0; q + 1 < cuts.size(); ++q) {
        double lo = cuts[q], hi = cuts[q + 1];
        double nlo = index(lo), nhi = index(hi);
        double pieces[3] = {lo, hi, hi};
        int np = 2;
        if ((nlo * beta > 1.0) != (nhi * beta > 1.0)) {
            pieces[1] = lo + (1.0 / beta - nlo) / (nhi - nlo) * (hi - lo);
            np = 3;
        }
        for (int p = 0; p + 1 < np; ++p) {
            double a = pieces[p], b = pieces[p + 1], half = 0.5 * (b - a), mid = 0.5 * (a + b);
            double sum = 0.0;
            for (int i = 0; i < kPoints; ++i) sum += gw[i] * weight(mid + half * gx[i]);
            integral += half * sum;
        }
    }
    const double alpha = 1.0 / 137.035999084, pi = 3.14159265358979323846;
    // lambda in mm: the nm integral times 1e6
    *photons_per_mm = 2.0 * pi * alpha * 1e6 * integral;
    return RICH_OK;
}

rich_status rich_film_readout(const rich_film *film, const uint8_t *dev_fate, const float *dev_hit_uv,
                              uint64_t n_photons, float *dev_image, uint8_t *dev_hits, hipStream_t stream) {
    if (!film || !dev_image) return set_error(RICH_EINVAL, "film and dev_image must not be NULL");
    if (n_photons && (!dev_fate || !dev_hit_uv)) return set_error(RICH_EINVAL, "dev_fate and dev_hit_uv needed");
    if (film->width < 1 || film->height < 1 || (int64_t)film->width * film->height > (1ll << 31))
        return set_error(RICH_EINVAL, "film size out of range");
    const double pi = 3.14159265358979323846;
    if (!(film->distance > 0) || !std::isfinite(film->distance) || !(film->fov > 0) || !(film->fov < pi) ||
        !(film->sigma > 0) || !(film->sigma < 64) || !std::isfinite(film->threshold))
        return set_error(RICH_EINVAL, "film: distance > 0, 0 < fov < pi, 0 < sigma < 64, finite threshold");
    const double f = 0.5 * film->width / std::tan(0.5 * film->fov);
    FilmArgs a;
    a.width = film->width;
    a.height = film->height;
    a.cx = (float)(0.5 * film->width);
    a.cy = (float)(0.5 * film->height);
    a.scale = (float)(f / film->distance);
    a.radius = (float)(4.0 * film->sigma);
    a.inv_2s2 = (float)(1.0 / (2.0 * film->sigma * film->sigma));
    a.threshold = (float)film->threshold;
    RICH_HIP(launch_film(a, dev_fate, dev_hit_uv, n_photons, dev_image, dev_hits, stream));
    return RICH_OK;
}

rich_status rich_get_status(rich_scene *s, hipStream_t stream, uint32_t *flags) {
    if (!s) return set_error(RICH_EINVAL, "scene is NULL");
    DeviceGuard g(s->device);
    RICH_HIP(hipStreamSynchronize(stream));
    unsigned int f = 0;
    RICH_HIP(hipMemcpy(&f, s->d_status, sizeof f, hipMemcpyDeviceToHost));
    unsigned int zero = 0;
    RICH_HIP(hipMemcpy(s->d_status, &zero, sizeof zero, hipMemcpyHostToDevice));
    if (flags) *flags = f;
    if (f) return set_error(RICH_EOVERFLOW, "device flags 0x%x raised", f);
    return RICH_OK;
}

}  // extern "C"
