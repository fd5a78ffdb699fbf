// common.hpp -- internal helpers of the gfx950 splatting library.
// Not part of the public ABI (see include/splat.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/splat.h"

namespace splat {

constexpr int kWave = 64;

// digit width of the LSD radix sort of the instance keys
#ifndef SPLAT_RADIX_BITS
#define SPLAT_RADIX_BITS 9
#endif
constexpr int kRadixBits = SPLAT_RADIX_BITS;
constexpr int kRadixDigits = 1 << kRadixBits;
constexpr int kDw2cStages = 32;  // workgroups per view summing the W2C gradient partials
constexpr int kL1Span = 4096;    // work-item partials of the forward's L1 term summed per workgroup
constexpr size_t kCamBytes = 144;  // per-view camera constants of the projection (f64[8], f32[20])

// workspace views --------------------------------------------------------------
template <typename T>
__host__ __device__ inline T *ws_at(void *ws, size_t off) {
    return reinterpret_cast<T *>(reinterpret_cast<char *>(ws) + off);
}

struct alignas(8) Rect16 {
    uint16_t x0, x1, y0, y1;
};

// counter indices in off_counts
enum { CNT_SLOTS = 0, CNT_INST = 1, CNT_WORK = 2, CNT_NSPLIT = 3, CNT_NCHUNK = 4, CNT_BITEMS = 5, CNT_PREP = 6,
       CNT_RUNS = 7 };
// counts[CNT_PREP]: the bin sort the last projection wrote its per-slot inputs for
constexpr uint32_t kPrepSlotSort = 0x534C4F54u, kPrepInstSort = 0x494E5354u;

// float <-> bits
__device__ inline uint32_t f2u(float f) { return __float_as_uint(f); }

// wave-level helpers -------------------------------------------------------------
__device__ inline int lane_id() { return __lane_id(); }

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

// exclusive rank of this lane among the set bits of mask below it
__device__ inline uint32_t rank_in(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// host side ------------------------------------------------------------------------
void set_error(const char *fmt, ...);
int launch_status(const char *what);

// internal launchers (one per translation unit)
int launch_pose_fwd(int32_t K, const double *kt, const double *kq, const double *kp, int32_t C,
                    const double *R0, const double *t0, const double *xi, const double *delta,
                    int32_t V, const int32_t *vcam, const double *vt, double *w2c, uint32_t *status,
                    hipStream_t st);
int launch_pose_bwd(int32_t K, const double *kt, const double *kq, const double *kp, int32_t C,
                    const double *R0, const double *t0, const double *xi, const double *delta,
                    int32_t V, const int32_t *vcam, const double *vt, const double *dw2c,
                    double *dxi, double *ddelta, hipStream_t st);
int launch_slot_meta(const splat_plan &p, void *ws, hipStream_t st);
int launch_project(const splat_plan &p, void *ws, const splat_gaussians &g, const double *w2c,
                   const double *intr, hipStream_t st);
int launch_project_bwd(const splat_plan &p, void *ws, const splat_gaussians &g, const double *w2c,
                       const double *intr, float *dquat, float *dscale, float *dopac,
                       float *dcolor, float *dmean, double *dw2c, hipStream_t st);
int launch_bin_sort(const splat_plan &p, void *ws, hipStream_t st);
// The L1 term fused into the forward's output stage (target null: not fused): per pixel of the
// region of interest d = img - target (0 where mask is set), dimg = sign(d) inv_n, *loss +=
// sum |d| inv_n, as launch_l1 computes them.
struct L1Fuse {
    const float *target;
    const uint8_t *mask;
    float *dimg;
    double *loss;
    double inv_n;
};
int launch_render_fwd(const splat_plan &p, void *ws, float *img, float *T, int32_t *last,
                      uint64_t *stats, hipStream_t st, const L1Fuse *l1 = nullptr);
int launch_render_bwd(const splat_plan &p, void *ws, const float *dimg, const float *T,
                      const int32_t *last, uint64_t *stats, hipStream_t st);
int launch_l1(const float *img, const float *target, const uint8_t *mask, int64_t n_views, int32_t width,
              int32_t height, int32_t roi_y0, double inv_n, float *dimg, double *loss, hipStream_t st);
int launch_scale_reg(const float *scale, int64_t n, double lambda, float *dscale, double *loss, hipStream_t st);
int launch_adam(const splat_adam_group *groups, int n_groups, double beta1, double beta2, double eps, float *step,
                hipStream_t st);
size_t dssim_ws_bytes(int64_t n_views, int32_t width, int32_t height, int32_t roi_y0);
size_t ngp_ws_bytes(int64_t n);
int launch_ngp_fwd(const splat_ngp &m, const float *mean, int64_t n, float *quat, float *scale, float *opac,
                   float *color, hipStream_t st);
int launch_ngp_bwd(const splat_ngp &m, const float *mean, int64_t n, const float *dquat, const float *dscale,
                   const float *dopac, const float *dcolor, void *ws, float *dtables, float *dw1, float *db1,
                   float *dw2, float *db2, float *dw3, float *db3, hipStream_t st);
size_t ngp_index_bytes(const splat_ngp &m, int64_t n);
size_t ngp_index_ws_bytes(const splat_ngp &m, int64_t n);
int launch_ngp_index_build(const splat_ngp &m, const float *mean, int64_t n, void *index, void *ws, hipStream_t st);
int launch_ngp_bwd_indexed(const splat_ngp &m, const float *mean, int64_t n, const void *index, const float *dquat,
                           const float *dscale, const float *dopac, const float *dcolor, void *ws, float *dtables,
                           float *dw1, float *db1, float *dw2, float *db2, float *dw3, float *db3, hipStream_t st);
int launch_ngp_fwd_train(const splat_ngp &m, const float *mean, int64_t n, float *quat, float *scale, float *opac,
                         float *color, void *ws, hipStream_t st);
int launch_ngp_bwd_saved(const splat_ngp &m, int64_t n, const void *index, const float *dquat, const float *dscale,
                         const float *dopac, const float *dcolor, void *ws, float *dtables, float *dw1, float *db1,
                         float *dw2, float *db2, float *dw3, float *db3, hipStream_t st);
int launch_dssim(const float *img, const float *target, int64_t n_views, int32_t width, int32_t height,
                 int32_t roi_y0, double weight, void *ws, float *dimg, double *loss, hipStream_t st);
// device address of the current GPU's D-SSIM scratch array (allocation-free entry point)
int dssim_scratch(float **out);

// device exclusive scan of u32 (binsort.hip): out[i] = sum in[0..i), out[n] = total;
// n is read from *n_dev (clamped to n_cap); partials needs scan_partials(n_cap) u32.
size_t scan_partials(int64_t n_cap);
int launch_scan_u32(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, int64_t n_cap,
                    uint32_t *partials, uint32_t *total_dst, hipStream_t st);
int launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
// stable LSD radix sort of (k0, v0) by key bits [bit0, bit0 + bits), n = counts[CNT_INST];
// hist needs 2^kRadixBits * nparts + 1 u32, partials scan_partials of that
int launch_radix_sort_u64(uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, const uint32_t *counts, int bit0,
                          int bits, int nparts, uint32_t *hist, uint32_t *partials, hipStream_t st, int *sorted_in_1);
// the same sort, where the passes after the first whose remaining digits fit 32 bits above
// a shift S <= max_shift carry u32 keys (key >> S); *key_shift = S, or -1 when none does
int launch_radix_sort_keys(uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, const uint32_t *counts, int bit0,
                           int bits, int nparts, uint32_t *hist, uint32_t *partials, hipStream_t st, int *sorted_in_1,
                           int max_shift, int *key_shift);
size_t voxel_ws_bytes(int64_t n);
int launch_voxel_downsample(const float *pts, int64_t n, const double *lo, double voxel, void *ws, int32_t *keep,
                            uint32_t *n_keep, uint32_t *status, hipStream_t st);

}  // namespace splat
