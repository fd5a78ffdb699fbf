// adam.hip -- the per-Gaussian optimiser step of the calibration loop: Adam (the
// optimiser of Sec. IV-B) over several parameter arrays in one launch, fused with
// the activation the render applies (sigmoid opacity, exp scale, identity colour
// and rotation): the gradient with respect to the activated value is chained to the
// raw parameter, the parameter updated, its activation rewritten for the next step
// and the gradient cleared for the next adjoint, which adds into it.  Memory-bound:
// per element 4 + 4 + 4 + 4 (+4) bytes read and 4 + 4 + 4 + 4 (+4) written.
#include "common.hpp"

#include <math.h>

namespace splat {
namespace {

struct AdamArgs {
    splat_adam_group g[SPLAT_ADAM_MAX_GROUPS];
    int n_groups;
    float b1, b2, eps;
};

// blockIdx.y = group (its fields are workgroup-uniform), blocks stride over its elements
__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a, const float *step) {
    const int k = blockIdx.y;
    if (k >= a.n_groups) return;
    const splat_adam_group G = a.g[k];
    const float t = *step + 1.f;
    // bias corrections in float64 (b^t for t up to 1e6 steps), applied in float32
    const float bc1 = (float)(1.0 - pow((double)a.b1, (double)t));
    const float rbc2 = (float)(1.0 / sqrt(1.0 - pow((double)a.b2, (double)t)));
    const float lr = *G.lr;
    const float step_size = lr / bc1;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < G.n; j += (int64_t)gridDim.x * blockDim.x) {
        float g = G.grad[j];
        float v = 0.f;
        if (G.act != SPLAT_ACT_IDENTITY) v = G.value[j];
        if (G.act == SPLAT_ACT_SIGMOID) g *= v * (1.f - v);
        else if (G.act == SPLAT_ACT_EXP) g *= v;
        const float m = a.b1 * G.exp_avg[j] + (1.f - a.b1) * g;
        const float s = a.b2 * G.exp_avg_sq[j] + (1.f - a.b2) * g * g;
        const float p = G.param[j] - step_size * m / (sqrtf(s) * rbc2 + a.eps);
        G.exp_avg[j] = m;
        G.exp_avg_sq[j] = s;
        G.param[j] = p;
        G.grad[j] = 0.f;
        if (G.act == SPLAT_ACT_SIGMOID) G.value[j] = 1.f / (1.f + expf(-p));
        else if (G.act == SPLAT_ACT_EXP) G.value[j] = expf(p);
    }
}

__global__ void adam_advance_kernel(float *step) { *step += 1.f; }

}  // namespace

int launch_adam(const splat_adam_group *groups, int n_groups, double beta1, double beta2, double eps, float *step,
                hipStream_t st) {
    AdamArgs a;
    a.n_groups = n_groups;
    a.b1 = (float)beta1;
    a.b2 = (float)beta2;
    a.eps = (float)eps;
    int64_t nmax = 0;
    for (int i = 0; i < SPLAT_ADAM_MAX_GROUPS; ++i) {
        a.g[i] = i < n_groups ? groups[i] : splat_adam_group{};
        if (i < n_groups && groups[i].n > nmax) nmax = groups[i].n;
    }
    if (nmax > 0) {
        int64_t nb = (nmax + 255) / 256;
        if (nb > 2048) nb = 2048;
        hipLaunchKernelGGL(adam_kernel, dim3((unsigned)nb, (unsigned)n_groups), dim3(256), 0, st, a,
                           (const float *)step);
        int rc = launch_status("adam");
        if (rc) return rc;
    }
    hipLaunchKernelGGL(adam_advance_kernel, dim3(1), dim3(1), 0, st, step);
    return launch_status("adam_advance");
}

}  // namespace splat
