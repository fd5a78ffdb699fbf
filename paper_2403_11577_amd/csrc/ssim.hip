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
// accumulation, which keeps m11 - m1^2 free of float32 cancellation) and stores G
// per pixel; ssim_bwd filters G and adds the gradient into dL/dimg.  Workgroups
// take 32 x 21 output tiles: the row pass then has exactly one item (4 outputs of
// one of the 31 halo rows) per thread and the column pass 3 outputs per thread,
// and three workgroups fit a compute unit's LDS.  The workgroups are persistent and
// fetch the next tile's inputs while they filter the current one.
#include <mutex>

#include "common.hpp"

// Gradient maps of the allocation-free entry point, one copy per GPU.  In host code
// the name is only a host-side stand-in: kernels receive the device address that
// hipGetSymbolAddress returns (dssim_scratch below).
static __device__ __align__(256) float scratch[3 * (size_t)SPLAT_DSSIM_NOALLOC_MAX_PX];

namespace splat {
namespace {

constexpr int SR = 5;                 // window radius
constexpr int SW = 2 * SR + 1;        // window width
constexpr int OX = 32, OY = 21;       // output tile
constexpr int IX = OX + 2 * SR, IY = OY + 2 * SR;
constexpr int RC = 4;                 // outputs per row-pass item (along x)
constexpr int CC = 3;                 // outputs per column-pass thread (along y)
constexpr int NCT = OX * (OY / CC);   // threads of the column pass
static_assert(OY % CC == 0 && OX % RC == 0 && IY * (OX / RC) <= 256 && NCT <= 256, "tile shape");
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

// The separable filter, both passes: a thread filters C + 10 consecutive inputs held in
// registers into C consecutive outputs (11 taps each), so every input is read from LDS once
// per thread rather than once per tap.
template <int NM, int C>
__device__ __forceinline__ void filter_cpt(const double (&g)[SW], const double (&v)[NM][C + 2 * SR],
                                           double (&out)[NM][C]) {
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int o = 0; o < C; ++o) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < SW; ++k) acc = fma(g[k], v[m][o + k], acc);
            out[m][o] = acc;
        }
}

// Tiles are numbered plane-major, then tile row, then tile column; workgroups are persistent
// and walk their tiles as TileWalk below orders them.  A tile's inputs (its 42 x 31 halo, PF values per
// thread) are fetched into registers during the previous tile's filtering, so that the load
// latency is not exposed between the passes.
constexpr int NIN = IY * IX;                 // halo inputs per plane and tile
constexpr int PF = (NIN + 255) / 256;        // inputs per thread

struct TileIdx {
    int plane, x0, y0;
};

__device__ inline TileIdx tile_at(int tile, int ntx, int nty) {
    TileIdx ti;
    const int per = ntx * nty;
    ti.plane = tile / per;
    const int r = tile - ti.plane * per;
    const int ty = r / ntx;
    ti.y0 = ty * OY;
    ti.x0 = (r - ty * ntx) * OX;
    return ti;
}

// The tiles a workgroup takes.  Workgroups are handed to the eight XCDs in turn (workgroup b
// to XCD b mod 8), and each XCD has its own L2; when the grid is a multiple of 8 the tiles are
// cut into eight contiguous ranges, one per XCD, so that neighbouring tiles -- which share
// halo inputs -- run on the same XCD.
struct TileWalk {
    int base, chunk, step, k, ntiles;
    __device__ TileWalk(int ntiles_) : ntiles(ntiles_) {
        const bool xm = (gridDim.x & 7u) == 0u;
        chunk = xm ? (ntiles + 7) / 8 : ntiles;
        base = xm ? (int)(blockIdx.x & 7u) * chunk : 0;
        step = xm ? (int)(gridDim.x >> 3) : (int)gridDim.x;
        k = xm ? (int)(blockIdx.x >> 3) : (int)blockIdx.x;
    }
    // tile number kk of this workgroup's sequence, or -1 past its end
    __device__ int at(int kk) const { return kk < chunk && base + kk < ntiles ? base + kk : -1; }
};

// halo input i of the tile (row-major over IY x IX): index into the plane arrays, or -1 outside
__device__ inline int64_t halo_src(const SsimArgs &a, const TileIdx &ti, int i, int64_t plane_stride, int row_off) {
    const int r = i / IX, c = i - r * IX;
    const int gr = ti.y0 + r - SR, gc = ti.x0 + c - SR;
    if (i >= NIN || gr < 0 || gr >= a.Hc || gc < 0 || gc >= a.W) return -1;
    return (int64_t)ti.plane * plane_stride + (int64_t)(gr + row_off) * a.W + gc;
}

__global__ __launch_bounds__(256) void ssim_fwd_kernel(SsimArgs a, const float *x, const float *y, double fscale,
                                                      double weight, float *G, double *loss, int ntx, int nty,
                                                      int ntiles) {
    __shared__ float sx[IY][IX + 1], sy[IY][IX + 1];
    __shared__ double hm[5][IY][OX];
    __shared__ double part[4];
    const int64_t np = (int64_t)(ntiles / (ntx * nty)) * a.hwc;
    double g[SW];
#pragma unroll
    for (int k = 0; k < SW; ++k) g[k] = a.g[k];
    float fx[PF], fy[PF];
    auto fetch = [&](int tile, int t) {
        const TileIdx ti = tile_at(tile, ntx, nty);
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int64_t o = halo_src(a, ti, t + 256 * j, a.hw, a.roi);
            fx[j] = o >= 0 ? x[o] : 0.f;
            fy[j] = o >= 0 ? y[o] : 0.f;
        }
    };
    TileWalk tw(ntiles);
    int tile = tw.at(tw.k);
    if (tile >= 0) fetch(tile, threadIdx.x);
    double ssum = 0.0;
    for (; tile >= 0; tw.k += tw.step, tile = tw.at(tw.k)) {
        // the thread index, opaque to the compiler: the indices derived from it are formed
        // again in every iteration instead of being kept in registers across the loop
        int t = threadIdx.x;
        asm volatile("" : "+v"(t));
        const TileIdx ti = tile_at(tile, ntx, nty);
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int i = t + 256 * j;
            if (i < NIN) {
                const int r = i / IX, c = i - r * IX;
                sx[r][c] = fx[j];
                sy[r][c] = fy[j];
            }
        }
        // the inputs are staged, and every thread has left the previous tile's column pass
        __syncthreads();
        if (tw.at(tw.k + tw.step) >= 0) fetch(tw.at(tw.k + tw.step), t);
        // rows: the five raw moments x, y, x^2, y^2, xy of every halo row, RC columns per item,
        // one moment at a time (the inputs stay as float32 in registers)
        if (t < IY * (OX / RC)) {
            const int r = t / (OX / RC), c0 = (t - r * (OX / RC)) * RC;
            float xs[RC + 2 * SR], ys[RC + 2 * SR];
#pragma unroll
            for (int k = 0; k < RC + 2 * SR; ++k) {
                xs[k] = sx[r][c0 + k];
                ys[k] = sy[r][c0 + k];
            }
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                double v[1][RC + 2 * SR];
#pragma unroll
                for (int k = 0; k < RC + 2 * SR; ++k) {
                    const double xv = xs[k], yv = ys[k];
                    v[0][k] = m == 0 ? xv : m == 1 ? yv : m == 2 ? xv * xv : m == 3 ? yv * yv : xv * yv;
                }
                double out[1][RC];
                filter_cpt<1, RC>(g, v, out);
#pragma unroll
                for (int o = 0; o < RC; ++o) hm[m][r][c0 + o] = out[0][o];
            }
        }
        // the row moments are complete (and the staged inputs free for the next tile)
        __syncthreads();
        // columns: CC rows of one column per thread, then SSIM and its partials
        if (t < NCT) {
            const int c = t % OX, r0 = (t / OX) * CC;
            double mo[5][CC];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                double v[1][CC + 2 * SR], out[1][CC];
#pragma unroll
                for (int k = 0; k < CC + 2 * SR; ++k) v[0][k] = hm[m][r0 + k][c];
                filter_cpt<1, CC>(g, v, out);
#pragma unroll
                for (int o = 0; o < CC; ++o) mo[m][o] = out[0][o];
                // one moment's 13 reads in flight at a time: the registers of all 65 would halve
                // the waves per SIMD
                asm volatile("" ::: "memory");
            }
            const int64_t gbase = (int64_t)ti.plane * a.hwc;
            const int gc = ti.x0 + c;
#pragma unroll
            for (int o = 0; o < CC; ++o) {
                const int gr = ti.y0 + r0 + o;
                if (gr >= a.Hc || gc >= a.W) continue;
                const double m1 = mo[0][o], m2 = mo[1][o], m11 = mo[2][o], m22 = mo[3][o], m12 = mo[4][o];
                const double A = 2.0 * m1 * m2 + SC1;
                const double B = 2.0 * (m12 - m1 * m2) + SC2;
                const double C = m1 * m1 + m2 * m2 + SC1;
                const double D = (m11 - m1 * m1) + (m22 - m2 * m2) + SC2;
                // one division for the four reciprocals
                const double AB = A * B, CD = C * D, P = 1.0 / (AB * CD);
                const double rA = B * CD * P, rB = A * CD * P, rC = AB * D * P, rD = AB * C * P;
                const double S = AB * AB * P;
                ssum += S;
                // dS/dm1 = S (2 m2 / A - 2 m2 / B - 2 m1 / C + 2 m1 / D), dS/dm11 = -S / D, dS/dm12 = 2 S / B
                const double d1 = 2.0 * S * (m2 * (rA - rB) + m1 * (rD - rC));
                const double d11 = -S * rD, d12 = 2.0 * S * rB;
                const int64_t q = gbase + (int64_t)gr * a.W + gc;
                G[q] = (float)(fscale * d1);
                G[np + q] = (float)(fscale * d11);
                G[2 * np + q] = (float)(fscale * d12);
            }
        }
    }
    ssum = wave_sum(ssum);
    const int t = threadIdx.x;
    if ((t & 63) == 0) part[t >> 6] = ssum;
    __syncthreads();
    if (t == 0 && loss) {
        double sm = ((part[0] + part[1]) + part[2]) + part[3];
        double add = fscale * sm;  // fscale = -weight / N
        if (blockIdx.x == 0) add += weight;
        atomicAdd(loss, add);
    }
}

__global__ __launch_bounds__(256, 4) void ssim_bwd_kernel(SsimArgs a, const float *x, const float *y, const float *G,
                                                      float *dimg, int ntx, int nty, int ntiles) {
    __shared__ float sg[3][IY][IX + 1];
    __shared__ double hm[3][IY][OX];
    const int64_t np = (int64_t)(ntiles / (ntx * nty)) * a.hwc;
    double g[SW];
#pragma unroll
    for (int k = 0; k < SW; ++k) g[k] = a.g[k];
    float f0[PF], f1[PF], f2[PF];
    auto fetch = [&](int tile, int t) {
        const TileIdx ti = tile_at(tile, ntx, nty);
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int64_t o = halo_src(a, ti, t + 256 * j, a.hwc, 0);
            f0[j] = o >= 0 ? G[o] : 0.f;
            f1[j] = o >= 0 ? G[np + o] : 0.f;
            f2[j] = o >= 0 ? G[2 * np + o] : 0.f;
        }
    };
    TileWalk tw(ntiles);
    int tile = tw.at(tw.k);
    if (tile >= 0) fetch(tile, threadIdx.x);
    for (; tile >= 0; tw.k += tw.step, tile = tw.at(tw.k)) {
        int t = threadIdx.x;  // opaque, as in the forward
        asm volatile("" : "+v"(t));
        const TileIdx ti = tile_at(tile, ntx, nty);
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int i = t + 256 * j;
            if (i < NIN) {
                const int r = i / IX, c = i - r * IX;
                sg[0][r][c] = f0[j];
                sg[1][r][c] = f1[j];
                sg[2][r][c] = f2[j];
            }
        }
        __syncthreads();
        if (tw.at(tw.k + tw.step) >= 0) fetch(tw.at(tw.k + tw.step), t);
        if (t < IY * (OX / RC)) {
            const int r = t / (OX / RC), c0 = (t - r * (OX / RC)) * RC;
            double v[3][RC + 2 * SR];
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int k = 0; k < RC + 2 * SR; ++k) v[m][k] = sg[m][r][c0 + k];
            double out[3][RC];
            filter_cpt<3, RC>(g, v, out);
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int o = 0; o < RC; ++o) hm[m][r][c0 + o] = out[m][o];
        }
        __syncthreads();
        if (t < NCT) {
            const int c = t % OX, r0 = (t / OX) * CC;
            double f[3][CC];
            {
                double v[3][CC + 2 * SR];
#pragma unroll
                for (int m = 0; m < 3; ++m)
#pragma unroll
                    for (int k = 0; k < CC + 2 * SR; ++k) v[m][k] = hm[m][r0 + k][c];
                filter_cpt<3, CC>(g, v, f);
            }
            const int gc = ti.x0 + c;
#pragma unroll
            for (int o = 0; o < CC; ++o) {
                const int gr = ti.y0 + r0 + o;
                if (gr >= a.Hc || gc >= a.W) continue;
                const int64_t q = plane_px(a, ti.plane, gr, gc);
                const double xv = x[q], yv = y[q];
                dimg[q] += (float)(f[0][o] + 2.0 * xv * f[1][o] + yv * f[2][o]);
            }
        }
    }
}

// persistent workgroups: as many as fit the GPU at once (looked up once per device), at most
// one per tile
template <typename Kern>
int resident_groups(Kern k, int ntiles, int *out) {
    static int cache[64][2];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SPLAT_ELAUNCH;
    const int which = (void *)k == (void *)ssim_fwd_kernel ? 0 : 1;
    if (cache[dev][which] == 0) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, 256, 0) != hipSuccess || cus < 1 || per < 1) {
            set_error("dssim: occupancy query failed");
            return SPLAT_ELAUNCH;
        }
        cache[dev][which] = cus * per;
    }
    int g = ntiles < cache[dev][which] ? ntiles : cache[dev][which];
    if (g >= 8) g &= ~7;  // a multiple of 8: one tile range per XCD
    *out = g;
    return 0;
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
    const int ntx = (width + OX - 1) / OX, nty = (a.Hc + OY - 1) / OY;
    const int64_t nt64 = (int64_t)ntx * nty * n_views * 3;
    if (nt64 >= ((int64_t)1 << 31)) { set_error("dssim: too many tiles"); return SPLAT_EUNSUPPORTED; }
    const int ntiles = (int)nt64;
    int gf = 0, gb = 0;
    int rc = resident_groups(ssim_fwd_kernel, ntiles, &gf);
    if (rc || (rc = resident_groups(ssim_bwd_kernel, ntiles, &gb))) return rc;
    float *G = static_cast<float *>(ws);
    hipLaunchKernelGGL(ssim_fwd_kernel, dim3(gf), dim3(256), 0, st, a, img, target, fscale, weight, G, loss, ntx, nty,
                       ntiles);
    rc = launch_status("ssim_fwd");
    if (rc) return rc;
    hipLaunchKernelGGL(ssim_bwd_kernel, dim3(gb), dim3(256), 0, st, a, img, target, G, dimg, ntx, nty, ntiles);
    return launch_status("ssim_bwd");
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch[kMaxDevices];  // device address of each GPU's scratch array, once looked up
}  // namespace

// Device address of the current GPU's scratch array: looked up on the first call on that
// device (with it current) and kept; every later call reuses it.
int dssim_scratch(float **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error("dssim_loss_grad_noalloc: no current device below %d", kMaxDevices);
        return SPLAT_ELAUNCH;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("dssim_loss_grad_noalloc: hipGetSymbolAddress of the scratch array failed on device %d: %s",
                      dev, hipGetErrorString(e));
            return SPLAT_ELAUNCH;
        }
        g_scratch[dev] = static_cast<float *>(p);
    }
    *out = g_scratch[dev];
    return 0;
}

}  // namespace splat
