// loss.hip -- the L1 term of the photometric loss (paper Eq. 4) and its gradient.
//
// dL/dimg = sign(img - target) / N with sign(0) = 0, and L = sum |img - target| / N,
// where N = views * 3 * H * W.  Masked pixels (mask[v][p] != 0) contribute nothing.
// The loss is accumulated in float64 with one atomic per workgroup.
#include "common.hpp"

namespace splat {
namespace {

__global__ __launch_bounds__(256) void l1_kernel(const float *img, const float *target, const uint8_t *mask,
                                                int64_t n_views, int64_t hw, double inv_n, float *dimg,
                                                double *loss) {
    __shared__ double part[4];
    int64_t n = n_views * 3 * hw;
    double acc = 0.0;
    float g = (float)inv_n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float d = img[i] - target[i];
        if (mask) {
            int64_t v = i / (3 * hw);
            int64_t p = i - v * 3 * hw;
            p -= (p / hw) * hw;
            if (mask[v * hw + p]) d = 0.f;
        }
        float sg = d > 0.f ? g : (d < 0.f ? -g : 0.f);
        dimg[i] = sg;
        acc += (double)fabsf(d);
    }
    acc = wave_sum(acc);
    if (__lane_id() == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0 && loss) atomicAdd(loss, (part[0] + part[1] + part[2] + part[3]) * inv_n);
}

}  // namespace

int launch_l1(const float *img, const float *target, const uint8_t *mask, int64_t n_views, int64_t hw, double inv_n,
              float *dimg, double *loss, hipStream_t st) {
    int64_t n = n_views * 3 * hw;
    int64_t nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(l1_kernel, dim3((unsigned)nb), dim3(256), 0, st, img, target, mask, n_views, hw, inv_n, dimg,
                       loss);
    return launch_status("l1");
}

}  // namespace splat
