// loss.hip -- the L1 term of the photometric loss (paper Eq. 4), the scale
// regulariser (Sec. III-C) and their gradients.
//
// dL/dimg = sign(img - target) / N with sign(0) = 0, and L = sum |img - target| / N,
// where N = views * 3 * (H - roi_y0) * W: the rows above the region of interest and
// masked pixels (mask[v][p] != 0) contribute nothing.  Also the scale regulariser.
// The loss is accumulated in float64 with one atomic per workgroup.
#include "common.hpp"

namespace splat {
namespace {

__global__ __launch_bounds__(256) void l1_kernel(const float *img, const float *target, const uint8_t *mask,
                                                int64_t n_views, int32_t width, int32_t height, int32_t roi_y0,
                                                double inv_n, float *dimg, double *loss) {
    __shared__ double part[4];
    const int64_t hw = (int64_t)width * height;
    const int64_t n = n_views * 3 * hw;
    const int64_t top = (int64_t)roi_y0 * width;  // pixels above the region of interest
    double acc = 0.0;
    float g = (float)inv_n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t v = i / (3 * hw);
        int64_t p = i - v * 3 * hw;
        p -= (p / hw) * hw;
        float d = img[i] - target[i];
        if (p < top || (mask && mask[v * hw + p])) d = 0.f;
        float sg = d > 0.f ? g : (d < 0.f ? -g : 0.f);
        dimg[i] = sg;
        acc += (double)fabsf(d);
    }
    acc = wave_sum(acc);
    if (__lane_id() == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0 && loss) atomicAdd(loss, (part[0] + part[1] + part[2] + part[3]) * inv_n);
}

// Scale regulariser (Sec. III-C): per Gaussian m = mean of the three scales (float64),
// L += lambda * sum_k |s_k - m|, dL/ds_k = lambda * (sign(s_k - m) - mean_j sign(s_j - m)).
__global__ __launch_bounds__(256) void scale_reg_kernel(const float *scale, int64_t n, double lambda, float *dscale,
                                                       double *loss) {
    __shared__ double part[4];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s0 = scale[i], s1 = scale[n + i], s2 = scale[2 * n + i];
        double m = (s0 + s1 + s2) / 3.0;
        double d0 = s0 - m, d1 = s1 - m, d2 = s2 - m;
        double g0 = (d0 > 0) - (d0 < 0), g1 = (d1 > 0) - (d1 < 0), g2 = (d2 > 0) - (d2 < 0);
        double gm = (g0 + g1 + g2) / 3.0;
        dscale[i] += (float)(lambda * (g0 - gm));
        dscale[n + i] += (float)(lambda * (g1 - gm));
        dscale[2 * n + i] += (float)(lambda * (g2 - gm));
        acc += fabs(d0) + fabs(d1) + fabs(d2);
    }
    acc = wave_sum(acc);
    if (__lane_id() == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0 && loss) atomicAdd(loss, lambda * (part[0] + part[1] + part[2] + part[3]));
}

}  // namespace

int launch_l1(const float *img, const float *target, const uint8_t *mask, int64_t n_views, int32_t width,
              int32_t height, int32_t roi_y0, double inv_n, float *dimg, double *loss, hipStream_t st) {
    int64_t n = n_views * 3 * (int64_t)width * height;
    int64_t nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(l1_kernel, dim3((unsigned)nb), dim3(256), 0, st, img, target, mask, n_views, width, height,
                       roi_y0, inv_n, dimg, loss);
    return launch_status("l1");
}

int launch_scale_reg(const float *scale, int64_t n, double lambda, float *dscale, double *loss, hipStream_t st) {
    int64_t nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(scale_reg_kernel, dim3((unsigned)nb), dim3(256), 0, st, scale, n, lambda, dscale, loss);
    return launch_status("scale_reg");
}

}  // namespace splat
