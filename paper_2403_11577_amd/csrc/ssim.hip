// ssim.hip -- the D-SSIM term of the photometric loss (paper Eq. 4) and its gradient.
//
// SSIM of the rendered image x against the target y with an 11 x 11 Gaussian
// window (sigma 1.5, normalised), zero padding and C1 = 0.01^2, C2 = 0.03^2, per
// channel, over the rows [roi_y0, H) (the image is cropped to the region of
// interest first).  With the raw window moments m1 = w*x, m2 = w*y, m11 = w*x^2,
// m22 = w*y^2, m12 = w*xy and
//   S = (2 m1 m2 + C1)(2 (m12 - m1 m2) + C2) / ((m1^2 + m2^2 + C1)((m11 - m1^2) + (m22 - m2^2) + C2)),
// the loss term is weight * (1 - mean S) and, the window being symmetric,
//   dL/dx = w*G1 + 2 x (w*G11) + y (w*G12),   G = dL/dS * (dS/dm1, dS/dm11, dS/dm12).
// Two launches: ssim_fwd forms the moments (separable filter through LDS, float64
// accumulation: the stage is bandwidth-bound, so float64 costs nothing and keeps
// m11 - m1^2 free of float32 cancellation) and stores G per pixel; ssim_bwd
// filters G and adds the gradient into dL/dimg.
#include "common.hpp"

namespace splat {
namespace {

constexpr int SR = 5;                 // window radius
constexpr int SW = 2 * SR + 1;        // window width
constexpr int STX = 32, STY = 16;     // output tile
constexpr int SLX = STX + 2 * SR, SLY = STY + 2 * SR;
constexpr double SC1 = 0.01 * 0.01, SC2 = 0.03 * 0.03;

struct SsimArgs {
    int W, H, roi, Hc;       // Hc = H - roi rows in the region
    int64_t hw, hwc;         // H*W, Hc*W
    double g[SW];            // normalised 1-D window
};

__device__ inline int64_t plane_px(const SsimArgs &a, int plane, int r, int c) {
    // image index of row r (region coordinates) and column c of plane (view, channel)
    return (int64_t)plane * a.hw + (int64_t)(r + a.roi) * a.W + c;
}

__global__ __launch_bounds__(256) void ssim_fwd_kernel(SsimArgs a, const float *x, const float *y, double fscale,
                                                      double weight, float *G, double *loss) {
    __shared__ float sx[SLY][SLX], sy[SLY][SLX];
    __shared__ double hm[5][SLY][STX];
    __shared__ double part[4];
    const int t = threadIdx.x, plane = blockIdx.z;
    const int x0 = blockIdx.x * STX, y0 = blockIdx.y * STY;
    for (int i = t; i < SLY * SLX; i += 256) {
        int r = i / SLX, c = i - r * SLX;
        int gr = y0 + r - SR, gc = x0 + c - SR;
        bool in = gr >= 0 && gr < a.Hc && gc >= 0 && gc < a.W;
        int64_t o = in ? plane_px(a, plane, gr, gc) : 0;
        sx[r][c] = in ? x[o] : 0.f;
        sy[r][c] = in ? y[o] : 0.f;
    }
    __syncthreads();
    for (int i = t; i < SLY * STX; i += 256) {
        int r = i / STX, c = i - r * STX;
        double m1 = 0, m2 = 0, m11 = 0, m22 = 0, m12 = 0;
#pragma unroll
        for (int k = 0; k < SW; ++k) {
            double xv = sx[r][c + k], yv = sy[r][c + k], gk = a.g[k];
            m1 += gk * xv;
            m2 += gk * yv;
            m11 += gk * (xv * xv);
            m22 += gk * (yv * yv);
            m12 += gk * (xv * yv);
        }
        hm[0][r][c] = m1; hm[1][r][c] = m2; hm[2][r][c] = m11; hm[3][r][c] = m22; hm[4][r][c] = m12;
    }
    __syncthreads();
    double ssum = 0.0;
    const int64_t gbase = (int64_t)plane * a.hwc;
    for (int i = t; i < STY * STX; i += 256) {
        int r = i / STX, c = i - r * STX;
        int gr = y0 + r, gc = x0 + c;
        if (gr >= a.Hc || gc >= a.W) continue;
        double m1 = 0, m2 = 0, m11 = 0, m22 = 0, m12 = 0;
#pragma unroll
        for (int k = 0; k < SW; ++k) {
            double gk = a.g[k];
            m1 += gk * hm[0][r + k][c];
            m2 += gk * hm[1][r + k][c];
            m11 += gk * hm[2][r + k][c];
            m22 += gk * hm[3][r + k][c];
            m12 += gk * hm[4][r + k][c];
        }
        double A = 2.0 * m1 * m2 + SC1;
        double B = 2.0 * (m12 - m1 * m2) + SC2;
        double C = m1 * m1 + m2 * m2 + SC1;
        double D = (m11 - m1 * m1) + (m22 - m2 * m2) + SC2;
        double S = (A * B) / (C * D);
        ssum += S;
        // dS/dm1 = S (2 m2 / A - 2 m2 / B - 2 m1 / C + 2 m1 / D), dS/dm11 = -S / D, dS/dm12 = 2 S / B
        double d1 = S * (2.0 * m2 / A - 2.0 * m2 / B - 2.0 * m1 / C + 2.0 * m1 / D);
        double d11 = -S / D, d12 = 2.0 * S / B;
        int64_t o = gbase + (int64_t)gr * a.W + gc;
        G[o] = (float)(fscale * d1);
        G[(int64_t)gridDim.z * a.hwc + o] = (float)(fscale * d11);
        G[2 * (int64_t)gridDim.z * a.hwc + o] = (float)(fscale * d12);
    }
    ssum = wave_sum(ssum);
    if ((t & 63) == 0) part[t >> 6] = ssum;
    __syncthreads();
    if (t == 0 && loss) {
        double s = ((part[0] + part[1]) + part[2]) + part[3];
        double add = fscale * s;  // fscale = -weight / N
        if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0) add += weight;
        atomicAdd(loss, add);
    }
}

__global__ __launch_bounds__(256) void ssim_bwd_kernel(SsimArgs a, const float *x, const float *y, const float *G,
                                                      float *dimg) {
    __shared__ float sg[3][SLY][SLX];
    __shared__ double hm[3][SLY][STX];
    const int t = threadIdx.x, plane = blockIdx.z;
    const int x0 = blockIdx.x * STX, y0 = blockIdx.y * STY;
    const int64_t np = (int64_t)gridDim.z * a.hwc;
    for (int i = t; i < SLY * SLX; i += 256) {
        int r = i / SLX, c = i - r * SLX;
        int gr = y0 + r - SR, gc = x0 + c - SR;
        bool in = gr >= 0 && gr < a.Hc && gc >= 0 && gc < a.W;
        int64_t o = in ? (int64_t)plane * a.hwc + (int64_t)gr * a.W + gc : 0;
        sg[0][r][c] = in ? G[o] : 0.f;
        sg[1][r][c] = in ? G[np + o] : 0.f;
        sg[2][r][c] = in ? G[2 * np + o] : 0.f;
    }
    __syncthreads();
    for (int i = t; i < SLY * STX; i += 256) {
        int r = i / STX, c = i - r * STX;
        double f1 = 0, f11 = 0, f12 = 0;
#pragma unroll
        for (int k = 0; k < SW; ++k) {
            double gk = a.g[k];
            f1 += gk * sg[0][r][c + k];
            f11 += gk * sg[1][r][c + k];
            f12 += gk * sg[2][r][c + k];
        }
        hm[0][r][c] = f1; hm[1][r][c] = f11; hm[2][r][c] = f12;
    }
    __syncthreads();
    for (int i = t; i < STY * STX; i += 256) {
        int r = i / STX, c = i - r * STX;
        int gr = y0 + r, gc = x0 + c;
        if (gr >= a.Hc || gc >= a.W) continue;
        double f1 = 0, f11 = 0, f12 = 0;
#pragma unroll
        for (int k = 0; k < SW; ++k) {
            double gk = a.g[k];
            f1 += gk * hm[0][r + k][c];
            f11 += gk * hm[1][r + k][c];
            f12 += gk * hm[2][r + k][c];
        }
        int64_t o = plane_px(a, plane, gr, gc);
        double xv = x[o], yv = y[o];
        dimg[o] += (float)(f1 + 2.0 * xv * f11 + yv * f12);
    }
}

}  // namespace

size_t dssim_ws_bytes(int64_t n_views, int32_t width, int32_t height, int32_t roi_y0) {
    return (size_t)3 * (size_t)(n_views * 3) * (size_t)(height - roi_y0) * (size_t)width * sizeof(float);
}

int launch_dssim(const float *img, const float *target, int64_t n_views, int32_t width, int32_t height,
                 int32_t roi_y0, double weight, void *ws, float *dimg, double *loss, hipStream_t st) {
    SsimArgs a;
    a.W = width;
    a.H = height;
    a.roi = roi_y0;
    a.Hc = height - roi_y0;
    a.hw = (int64_t)width * height;
    a.hwc = (int64_t)width * a.Hc;
    double sum = 0.0;
    for (int k = 0; k < SW; ++k) {
        double d = (double)(k - SR);
        a.g[k] = exp(-(d * d) / (2.0 * 1.5 * 1.5));
        sum += a.g[k];
    }
    for (int k = 0; k < SW; ++k) a.g[k] /= sum;
    double n = 3.0 * (double)n_views * (double)a.hwc;
    double fscale = -weight / n;
    dim3 grid((width + STX - 1) / STX, (a.Hc + STY - 1) / STY, (unsigned)(n_views * 3));
    float *G = static_cast<float *>(ws);
    hipLaunchKernelGGL(ssim_fwd_kernel, grid, dim3(256), 0, st, a, img, target, fscale, weight, G, loss);
    int rc = launch_status("ssim_fwd");
    if (rc) return rc;
    hipLaunchKernelGGL(ssim_bwd_kernel, grid, dim3(256), 0, st, a, img, target, G, dimg);
    return launch_status("ssim_bwd");
}

}  // namespace splat
