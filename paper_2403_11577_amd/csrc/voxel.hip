// voxel.hip -- voxel downsampling of the accumulated LiDAR cloud (Sec. III-C: one
// point per voxel; the coarse-to-fine schedule runs it at 10, 5 and 2 cm).
//
// Voxel of a point: floor((x - lo) / voxel) per axis in float64, 21 bits per axis,
// packed as its Morton (Z-curve) code: bit b of x, y, z goes to bit 3b, 3b+1, 3b+2.
// A stable radix sort of (code, index) puts every voxel's points together in index
// order, so the first of each run is the point with the lowest index; those are
// compacted in Z-curve order of their voxels, which keeps points that are close in
// space close in memory (the hash-grid adjoint's scattered updates then share
// cache lines and wave-level combining).
#include "common.hpp"

namespace splat {
namespace {

constexpr int VB = 21;                       // bits per axis
constexpr int64_t VMAX = ((int64_t)1 << VB) - 1;

struct VoxelLayout {
    size_t counts, keys, vals, flags, hist, partials, end;
    int nparts;
};

VoxelLayout voxel_layout(int64_t n) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    VoxelLayout L;
    int64_t np = (n + 8191) / 8192;
    L.nparts = (int)(np < 1 ? 1 : (np > 2048 ? 2048 : np));
    size_t nh = (size_t)kRadixDigits * L.nparts + 1;
    size_t o = 0;
    L.counts = o; o = al(o + 8 * 4);
    L.keys = o; o = al(o + (size_t)2 * n * 8);
    L.vals = o; o = al(o + (size_t)2 * n * 4);
    L.flags = o; o = al(o + (size_t)(n + 1) * 4);
    L.hist = o; o = al(o + nh * 4);
    size_t np1 = scan_partials(n + 1), np2 = scan_partials((int64_t)nh);
    L.partials = o; o = al(o + (np1 > np2 ? np1 : np2) * 4);
    L.end = o;
    return L;
}

// spreads the low 21 bits of v to bits 0, 3, 6, ..., 60
__device__ inline uint64_t spread3(uint64_t v) {
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x001F00000000FFFFull;
    v = (v | (v << 16)) & 0x001F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__global__ void voxel_key_kernel(const float *pts, int64_t n, double lo0, double lo1, double lo2, double voxel,
                                 uint64_t *keys, uint32_t *vals, uint32_t *counts, uint32_t *status) {
    if (blockIdx.x == 0 && threadIdx.x == 0) counts[CNT_INST] = (uint32_t)n;
    bool clamped = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double lo[3] = {lo0, lo1, lo2};
        uint64_t key = 0;
        for (int d = 0; d < 3; ++d) {
            double c = floor(((double)pts[d * n + i] - lo[d]) / voxel);
            if (!(c >= 0.0)) { c = 0.0; clamped = true; }          // below the box (or NaN)
            if (c > (double)VMAX) { c = (double)VMAX; clamped = true; }
            key |= spread3((uint64_t)c) << d;
        }
        keys[i] = key;
        vals[i] = (uint32_t)i;
    }
    if (__ballot(clamped) && __lane_id() == 0) atomicOr(status, SPLAT_ST_RANGE);
}

__global__ void voxel_flag_kernel(const uint64_t *keys, int64_t n, uint32_t *flags) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ void voxel_compact_kernel(const uint64_t *keys, const uint32_t *vals, const uint32_t *offs, int64_t n,
                                     int32_t *keep) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (i == 0 || keys[i] != keys[i - 1]) keep[offs[i]] = (int32_t)vals[i];
}

int grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

size_t voxel_ws_bytes(int64_t n) { return voxel_layout(n).end; }

int launch_voxel_downsample(const float *pts, int64_t n, const double *lo, double voxel, void *ws, int32_t *keep,
                            uint32_t *n_keep, uint32_t *status, hipStream_t st) {
    VoxelLayout L = voxel_layout(n);
    uint32_t *counts = ws_at<uint32_t>(ws, L.counts);
    uint64_t *k0 = ws_at<uint64_t>(ws, L.keys), *k1 = k0 + n;
    uint32_t *v0 = ws_at<uint32_t>(ws, L.vals), *v1 = v0 + n;
    uint32_t *flags = ws_at<uint32_t>(ws, L.flags);
    hipLaunchKernelGGL(voxel_key_kernel, dim3(grid_for(n)), dim3(256), 0, st, pts, n, lo[0], lo[1], lo[2], voxel, k0, v0,
                       counts, status);
    int rc = launch_status("voxel_key");
    if (rc) return rc;
    int in1 = 0;
    rc = launch_radix_sort_u64(k0, k1, v0, v1, counts, 0, 3 * VB, L.nparts, ws_at<uint32_t>(ws, L.hist),
                               ws_at<uint32_t>(ws, L.partials), st, &in1);
    if (rc) return rc;
    uint64_t *ks = in1 ? k1 : k0;
    uint32_t *vs = in1 ? v1 : v0;
    hipLaunchKernelGGL(voxel_flag_kernel, dim3(grid_for(n)), dim3(256), 0, st, ks, n, flags);
    if ((rc = launch_status("voxel_flag"))) return rc;
    rc = launch_scan_u32(flags, flags, nullptr, n, ws_at<uint32_t>(ws, L.partials), n_keep, st);
    if (rc) return rc;
    hipLaunchKernelGGL(voxel_compact_kernel, dim3(grid_for(n)), dim3(256), 0, st, ks, vs, flags, n, keep);
    return launch_status("voxel_compact");
}

}  // namespace splat
