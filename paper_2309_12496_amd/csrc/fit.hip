// Alignment-fit optimiser step on the device: Adam (Kingma and Ba, ICLR 2015)
// over the segment parameters in normalised coordinates z = (p - p0) / scale,
// with a cosine-decayed step size.  It records the step's loss, sets the
// residual cut for the next adjoint launch and writes the new parameters
// into the scene, so that a whole fit step (adjoint, reduction, this kernel,
// the parameter refresh) stays on the device and can be captured in a graph.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace rich {

namespace {

constexpr int kFitBlock = 256;

__global__ __launch_bounds__(kFitBlock) void fit_step_kernel(FitArgs a) {
    const int n = a.n_par;
    const float taken = a.state[3 * n];          // steps before this one
    const double t = (double)taken + 1.0;
    const double pi = 3.14159265358979323846;
    // step size at step t = 1, 2, ...: lr at t = 1, decaying towards lr_final
    const double size = a.lr_final + 0.5 * (a.lr - a.lr_final) * (1.0 + cos(pi * (t - 1.0) / a.n_steps));
    const float bc1 = (float)(1.0 - pow(a.beta1, t));   // bias corrections of the two moments
    const float bc2 = (float)(1.0 - pow(a.beta2, t));
    const float b1 = (float)a.beta1, b2 = (float)a.beta2, eps = (float)a.eps, lr_t = (float)size;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int col = j % 6;
        const float sc = a.scale[col];
        const float g = a.free[col] ? a.grad[j] * sc : 0.0f;   // gradient with respect to z
        float m = a.state[n + j], v = a.state[2 * n + j], z = a.state[j];
        m = b1 * m + (1.0f - b1) * g;
        v = b2 * v + (1.0f - b2) * (g * g);
        z -= lr_t * (m / bc1) / (sqrtf(v / bc2) + eps);
        a.state[j] = z;
        a.state[n + j] = m;
        a.state[2 * n + j] = v;
        const float p = fmaf(z, sc, a.p0[j]);
        a.params[j] = p;
        if (a.params_out) a.params_out[j] = p;
    }
    __syncthreads();   // every thread has read the step count
    if (threadIdx.x == 0) {
        const float loss = *a.loss;
        a.state[3 * n] = (float)t;
        if (a.losses && taken >= 0.0f && taken < (float)a.n_steps) a.losses[(int)taken] = loss;
        if (a.cut) *a.cut = loss > 0.0f ? fmaf(sqrtf(loss), a.outlier_cut, a.cut_floor) : INFINITY;
    }
}

}  // namespace

hipError_t launch_fit_step(const FitArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(fit_step_kernel, dim3(1), dim3(kFitBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace rich
