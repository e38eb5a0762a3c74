// Film read-out emulation (Section 4.4): the paper images the detector plane
// with a pinhole camera and a film, and counts pixels above an intensity
// threshold as hits.  Detected photons are projected onto the film and
// splatted with a Gaussian reconstruction filter; a second pass thresholds.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "rich_dev.h"

namespace rich {

namespace {

constexpr int kFilmBlock = 256;

// One thread per photon: project (u, v) and add 255 exp(-r^2 / 2 sigma^2)
// to the pixels whose centres lie within 4 sigma in x and in y.
__global__ __launch_bounds__(kFilmBlock) void film_splat_kernel(FilmArgs a, const uint8_t *fate, const float *uv,
                                                                uint64_t n, float *image) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        if (fate[p] != 0) continue;   // DETECTED only
        const float x = fmaf(a.scale, uv[2 * p], a.cx), y = fmaf(a.scale, uv[2 * p + 1], a.cy);
        if (!(fabsf(x) < 1e9f && fabsf(y) < 1e9f)) continue;   // NaN or far outside: nothing to add
        const int i0 = max((int)ceilf(x - a.radius - 0.5f), 0), i1 = min((int)floorf(x + a.radius - 0.5f), a.width - 1);
        const int j0 = max((int)ceilf(y - a.radius - 0.5f), 0), j1 = min((int)floorf(y + a.radius - 0.5f), a.height - 1);
        for (int j = j0; j <= j1; ++j) {
            const float dy = (float)j + 0.5f - y;
            for (int i = i0; i <= i1; ++i) {
                const float dx = (float)i + 0.5f - x;
                atomicAdd(image + (size_t)j * a.width + i, 255.0f * __expf(-(dx * dx + dy * dy) * a.inv_2s2));
            }
        }
    }
}

__global__ __launch_bounds__(kFilmBlock) void film_threshold_kernel(const float *image, uint64_t n_pix, float threshold,
                                                                    uint8_t *hits) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_pix; k += stride)
        hits[k] = fminf(image[k], 255.0f) >= threshold ? 1 : 0;
}

}  // namespace

hipError_t launch_film(const FilmArgs &a, const uint8_t *fate, const float *uv, uint64_t n, float *image,
                       uint8_t *hits, hipStream_t st) {
    if (n > 0) {
        uint64_t blocks = (n + kFilmBlock - 1) / kFilmBlock;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(film_splat_kernel, dim3((unsigned)blocks), dim3(kFilmBlock), 0, st, a, fate, uv, n, image);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (hits) {
        const uint64_t n_pix = (uint64_t)a.width * a.height;
        uint64_t blocks = (n_pix + kFilmBlock - 1) / kFilmBlock;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(film_threshold_kernel, dim3((unsigned)blocks), dim3(kFilmBlock), 0, st, image, n_pix,
                           a.threshold, hits);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace rich
