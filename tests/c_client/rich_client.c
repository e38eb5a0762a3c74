/*
 * A plain C program that drives librich.so through include/rich.h only:
 * reads an analytic scene and a track source from a text file, builds the
 * scene, propagates photons 0..n-1 into hipMalloc'd buffers, reads the device
 * flags and writes the per-photon results to a binary file.  It also checks
 * two error paths of the ABI (a NULL source, a wrapping id range).
 *
 *   rich_client <scene.txt> <n_photons> <seed> <out.bin>
 *
 * out.bin: fate u8[n], pixel i32[n], hit_uv f32[n][2], fate_counts u64[7],
 *          histogram-total u64.
 * Exit status 0 on success; the failing call is printed otherwise.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rich.h"

#define CHECK_HIP(x)                                                              \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));        \
            return 3;                                                             \
        }                                                                         \
    } while (0)

#define CHECK_RICH(x)                                                             \
    do {                                                                          \
        rich_status s_ = (x);                                                     \
        if (s_ != RICH_OK) {                                                      \
            fprintf(stderr, "%s returned %d: %s\n", #x, s_, rich_last_error());   \
            return 4;                                                             \
        }                                                                         \
    } while (0)

static FILE *g_in;

static int expect(const char *word) {
    char buf[64];
    if (fscanf(g_in, "%63s", buf) != 1 || strcmp(buf, word) != 0) {
        fprintf(stderr, "scene file: expected '%s'\n", word);
        return 0;
    }
    return 1;
}

static int read_d(double *x, int n) {
    for (int i = 0; i < n; ++i)
        if (fscanf(g_in, "%lf", &x[i]) != 1) {
            fprintf(stderr, "scene file: number expected\n");
            return 0;
        }
    return 1;
}

static int read_i(int32_t *x) {
    if (fscanf(g_in, "%d", x) != 1) {
        fprintf(stderr, "scene file: integer expected\n");
        return 0;
    }
    return 1;
}

/* A table of n nodes: n lambdas then n values, in fresh host arrays. */
static int read_table(int32_t *n, double **lam, double **val) {
    if (!read_i(n) || *n < 1 || *n > RICH_MAX_TABLE) return 0;
    *lam = (double *)malloc(sizeof(double) * *n);
    *val = (double *)malloc(sizeof(double) * *n);
    return *lam && *val && read_d(*lam, *n) && read_d(*val, *n);
}

int main(int argc, char **argv) {
    if (argc != 5) {
        fprintf(stderr, "usage: %s scene.txt n_photons seed out.bin\n", argv[0]);
        return 2;
    }
    uint64_t n = strtoull(argv[2], NULL, 10);
    uint64_t seed = strtoull(argv[3], NULL, 10);
    g_in = fopen(argv[1], "r");
    if (!g_in) {
        perror(argv[1]);
        return 2;
    }

    rich_scene_desc d;
    memset(&d, 0, sizeof d);
    rich_material mats[8];
    rich_segment segs[8];
    double params[8 * 6];
    rich_cap caps[8];
    rich_rect rects[8];
    memset(mats, 0, sizeof mats);
    memset(segs, 0, sizeof segs);
    memset(caps, 0, sizeof caps);
    memset(rects, 0, sizeof rects);

    if (!expect("materials") || !read_i(&d.n_materials) || d.n_materials < 1 || d.n_materials > 8) return 2;
    for (int i = 0; i < d.n_materials; ++i) {
        double *lam, *val;
        if (!read_i(&mats[i].kind) || !read_table(&mats[i].n_refl, &lam, &val)) return 2;
        mats[i].refl_lambda = lam;
        mats[i].refl_value = val;
    }
    d.materials = mats;

    if (!expect("segments") || !read_i(&d.n_segments) || d.n_segments < 0 || d.n_segments > 8) return 2;
    for (int k = 0; k < d.n_segments; ++k)
        if (!read_d(segs[k].pivot, 3) || !read_d(segs[k].u0, 3) || !read_d(segs[k].e1, 3) ||
            !read_d(segs[k].e2, 3) || !read_d(&segs[k].radius0, 1) || !read_d(&params[6 * k], 6))
            return 2;
    d.segments = segs;
    d.params = d.n_segments ? params : NULL;

    if (!expect("caps") || !read_i(&d.n_caps) || d.n_caps < 0 || d.n_caps > 8) return 2;
    for (int i = 0; i < d.n_caps; ++i)
        if (!read_i(&caps[i].segment) || !read_i(&caps[i].material) || !read_d(caps[i].origin, 3) ||
            !read_d(caps[i].axis_a, 3) || !read_d(caps[i].axis_b, 3) || !read_d(caps[i].bounds, 4))
            return 2;
    d.caps = caps;

    if (!expect("rects") || !read_i(&d.n_rects) || d.n_rects < 0 || d.n_rects > 8) return 2;
    for (int i = 0; i < d.n_rects; ++i)
        if (!read_i(&rects[i].material) || !read_d(rects[i].center, 3) || !read_d(rects[i].normal, 3) ||
            !read_d(rects[i].axis_u, 3) || !read_d(rects[i].axis_v, 3) || !read_d(rects[i].half, 2))
            return 2;
    d.rects = rects;

    rich_detector *det = &d.detector;
    double *qlam, *qval, pix[2];
    if (!expect("detector") || !read_d(det->center, 3) || !read_d(det->normal, 3) || !read_d(det->axis_u, 3) ||
        !read_d(det->axis_v, 3) || !read_d(det->half, 2) || !read_d(&det->pitch, 1) || !read_d(pix, 2) ||
        !read_table(&det->n_qe, &qlam, &qval))
        return 2;
    det->nx = (int32_t)pix[0];
    det->ny = (int32_t)pix[1];
    det->qe_lambda = qlam;
    det->qe_value = qval;

    if (!expect("box") || !read_i(&d.has_box) || !read_d(d.box_lo, 3) || !read_d(d.box_hi, 3)) return 2;
    double mb;
    if (!expect("limits") || !read_d(&mb, 1) || !read_d(&d.t_min, 1)) return 2;
    d.max_bounces = (int32_t)mb;

    rich_source src;
    memset(&src, 0, sizeof src);
    src.kind = RICH_SRC_TRACK;
    if (!expect("source") || !read_d(src.origin, 3) || !read_d(src.direction, 3) || !read_d(&src.length, 1) ||
        !read_d(&src.beta, 1) || !read_d(&src.n_radiator, 1) || !read_d(&src.lambda_min, 1) ||
        !read_d(&src.lambda_max, 1))
        return 2;
    fclose(g_in);

    rich_scene *scene = NULL;
    CHECK_RICH(rich_build_scene(&d, 0, &scene));
    rich_scene_stats st;
    CHECK_RICH(rich_scene_info(scene, &st));
    printf("scene: %lld BVH nodes, %lld device bytes, built in %.3f s\n", (long long)st.n_nodes,
           (long long)st.device_bytes, st.build_seconds);

    const uint64_t npix = (uint64_t)det->nx * (uint64_t)det->ny;
    uint8_t *d_fate;
    int32_t *d_pixel;
    float *d_xyz, *d_uv;
    uint32_t *d_hist;
    unsigned long long *d_counts;
    CHECK_HIP(hipMalloc((void **)&d_fate, n ? n : 1));
    CHECK_HIP(hipMalloc((void **)&d_pixel, 4 * (n ? n : 1)));
    CHECK_HIP(hipMalloc((void **)&d_xyz, 12 * (n ? n : 1)));
    CHECK_HIP(hipMalloc((void **)&d_uv, 8 * (n ? n : 1)));
    CHECK_HIP(hipMalloc((void **)&d_hist, 4 * npix));
    CHECK_HIP(hipMalloc((void **)&d_counts, 8 * RICH_N_FATES));
    CHECK_HIP(hipMemset(d_hist, 0, 4 * npix));
    CHECK_HIP(hipMemset(d_counts, 0, 8 * RICH_N_FATES));

    rich_outputs out;
    memset(&out, 0, sizeof out);
    out.fate = d_fate;
    out.pixel = d_pixel;
    out.hit_xyz = d_xyz;
    out.hit_uv = d_uv;
    out.histogram = d_hist;
    out.fate_counts = d_counts;

    hipStream_t stream;
    CHECK_HIP(hipStreamCreate(&stream));

    /* error paths: reported synchronously, nothing launched */
    rich_status e1 = rich_propagate(scene, NULL, n, seed, 0, &out, stream);
    rich_status e2 = rich_propagate(scene, &src, 16, seed, UINT64_MAX - 4, &out, stream);
    if (e1 != RICH_EINVAL || e2 != RICH_ERANGE || rich_last_error()[0] == '\0') {
        fprintf(stderr, "error paths: got %d and %d, expected %d and %d\n", e1, e2, RICH_EINVAL, RICH_ERANGE);
        return 5;
    }

    CHECK_RICH(rich_propagate(scene, &src, n, seed, 0, &out, stream));
    uint32_t flags = 0xffffffffu;
    CHECK_RICH(rich_get_status(scene, stream, &flags));
    if (flags != 0) {
        fprintf(stderr, "device flags 0x%x\n", flags);
        return 6;
    }

    uint8_t *fate = (uint8_t *)malloc(n ? n : 1);
    int32_t *pixel = (int32_t *)malloc(4 * (n ? n : 1));
    float *uv = (float *)malloc(8 * (n ? n : 1));
    uint32_t *hist = (uint32_t *)malloc(4 * npix);
    unsigned long long counts[RICH_N_FATES];
    if (!fate || !pixel || !uv || !hist) return 2;
    CHECK_HIP(hipMemcpy(fate, d_fate, n, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(pixel, d_pixel, 4 * n, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(uv, d_uv, 8 * n, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(hist, d_hist, 4 * npix, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(counts, d_counts, sizeof counts, hipMemcpyDeviceToHost));
    unsigned long long hist_total = 0;
    for (uint64_t i = 0; i < npix; ++i) hist_total += hist[i];

    FILE *f = fopen(argv[4], "wb");
    if (!f) {
        perror(argv[4]);
        return 2;
    }
    int ok = fwrite(fate, 1, n, f) == n && fwrite(pixel, 4, n, f) == n && fwrite(uv, 8, n, f) == n &&
             fwrite(counts, 8, RICH_N_FATES, f) == RICH_N_FATES && fwrite(&hist_total, 8, 1, f) == 1;
    if (fclose(f) != 0 || !ok) {
        fprintf(stderr, "writing %s failed\n", argv[4]);
        return 2;
    }

    CHECK_HIP(hipStreamDestroy(stream));
    CHECK_HIP(hipFree(d_fate));
    CHECK_HIP(hipFree(d_pixel));
    CHECK_HIP(hipFree(d_xyz));
    CHECK_HIP(hipFree(d_uv));
    CHECK_HIP(hipFree(d_hist));
    CHECK_HIP(hipFree(d_counts));
    CHECK_RICH(rich_destroy_scene(scene));
    printf("%s: %llu photons, %llu detected\n", rich_version(), (unsigned long long)n, counts[RICH_DETECTED]);
    return 0;
}
