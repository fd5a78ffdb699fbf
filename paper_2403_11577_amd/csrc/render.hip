// render.hip -- per-tile front-to-back alpha compositing and its reverse-order adjoint.
//
// The splatting function Phi of Eq. (5) (EWA splatting) evaluates, for every
// pixel, the sorted Gaussians of its tile: alpha = min(alpha_max, o exp(power))
// with power = -d^T Q d / 2, skips alpha < alpha_min, stops before a blend that
// would take the transmittance below t_min and accumulates C += c alpha T.  The
// backward pass (gradients to the Gaussians and, through them, to the pose; end
// of Sec. III-B) walks the same lists in reverse from the saved last
// contributor, recovers T by division from the saved final transmittance, and
// accumulates per-slot gradients with one wave-reduced atomic group per
// (tile, Gaussian).
//
// gfx950 mapping: one wave64 workgroup per (view, tile) work item, TW*TH/64
// pixels per lane.  A batch of 64 Gaussian records is gathered one record per
// lane (the next batch is in flight while the current one is evaluated) and
// broadcast to the whole wave with v_readlane into scalar registers, so the
// pair loop needs no LDS and no barrier.  The wave leaves a tile as soon as
// every lane is saturated (ballot).  Work items come from a queue ordered by
// decreasing list length; the hardware dispatcher hands them out in order, or
// persistent waves pull them from a counter.
//
// Both kernels evaluate alpha with the same inline function, with float
// contraction disabled, so the backward pass sees exactly the forward decisions,
// and means are taken relative to the enclosing 32x32 pixel block so the
// arithmetic is identical for every supported tile shape.
#include "common.hpp"

namespace splat {
namespace {

constexpr float LOG2E = 1.4426950408889634f;
constexpr float LN2 = 0.6931471805599453f;

struct RenderArgs {
    const float4 *rec;
    const uint32_t *vals;       // sorted slot ids
    const uint2 *ranges;        // [V*T]
    const uint32_t *queue;      // [V*T] work items in decreasing cost
    uint32_t *work;             // persistent work counter
    const uint32_t *counts;     // device counts (slots, instances)
    unsigned long long *stats;  // pair counters of the instrumented variant
    int n_items, T, tiles_x, W, H, persistent;
    float amin, amax, tmin;
    float bg0, bg1, bg2;
};

// one Gaussian as staged for a tile: block-relative mean, conic pre-scaled by
// -1/2 log2(e) (A, Cc) and -log2(e) (Bc), opacity, colour
struct Stage {
    float mx, my, A, Bc, Cc, o, r, g, b;
    uint32_t slot;
};

__device__ __forceinline__ Stage stage_load(const RenderArgs &a, uint32_t idx, uint32_t end, uint32_t nslots,
                                            float xb, float yb) {
    Stage s;
    s.mx = s.my = s.A = s.Bc = s.Cc = s.o = s.r = s.g = s.b = 0.f;
    s.slot = 0xFFFFFFFFu;
    if (idx < end) {
        uint32_t slot = a.vals[idx];
        // (a slot id outside the slot count cannot come out of the sort; it stays transparent)
        if (slot < nslots) {
            float4 r0 = a.rec[3 * (size_t)slot + 0];
            float4 r1 = a.rec[3 * (size_t)slot + 1];
            float4 r2 = a.rec[3 * (size_t)slot + 2];
            s.mx = (r0.x - xb) + r0.z;
            s.my = (r0.y - yb) + r0.w;
            s.A = -0.5f * LOG2E * r1.x;
            s.Bc = -LOG2E * r1.y;
            s.Cc = -0.5f * LOG2E * r1.z;
            s.o = r1.w;
            s.r = r2.x;
            s.g = r2.y;
            s.b = r2.z;
            s.slot = slot;
        }
    }
    return s;
}

__device__ __forceinline__ float bcast(float v, int j) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

// exponent in log2 units: A dx^2 + Bc dx dy + Cc dy^2
__device__ __forceinline__ float power2(float dx, float dy, float A, float Bc, float Cc) {
    return __fmaf_rn(dx, __fmaf_rn(A, dx, Bc * dy), (Cc * dy) * dy);
}

__device__ __forceinline__ float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }

// wave64 sum with DPP (quad swaps, half-row and row mirrors, row broadcasts);
// the total ends up in lane 63
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xF, false));
}

__device__ __forceinline__ float wave_sum63(float x) {
    x += dpp_f<0xB1, 0xF>(x);   // quad_perm [1,0,3,2]
    x += dpp_f<0x4E, 0xF>(x);   // quad_perm [2,3,0,1]
    x += dpp_f<0x141, 0xF>(x);  // row_half_mirror
    x += dpp_f<0x140, 0xF>(x);  // row_mirror
    x += dpp_f<0x142, 0xA>(x);  // row_bcast:15 into rows 1, 3
    x += dpp_f<0x143, 0xC>(x);  // row_bcast:31 into rows 2, 3
    return x;
}

__device__ __forceinline__ float lane63(float x) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

__device__ inline void stat_add(unsigned long long *dst, unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    if (__lane_id() == 0 && v) atomicAdd(dst, v);
}

__device__ __forceinline__ bool next_item(const RenderArgs &a, int iter, int &item) {
    if (a.persistent) {
        uint32_t it = 0;
        if (__lane_id() == 0) it = atomicAdd(a.work, 1u);
        item = __builtin_amdgcn_readfirstlane((int)it);
    } else {
        if (iter > 0) return false;
        item = blockIdx.x;
    }
    return item < a.n_items;
}

// STATS = true is the instrumented variant (pair counters for the roofline);
// it computes exactly the same outputs.
template <int TW, int TH, bool STATS>
__global__ __launch_bounds__(64) void render_fwd_kernel(RenderArgs a, float *img, float *Tout, int32_t *lastout) {
    constexpr int PPT = TW * TH / 64;
    const int lane = threadIdx.x;
    const size_t HW = (size_t)a.W * a.H;
    const uint32_t nslots = a.counts[CNT_SLOTS];
    unsigned long long n_eval = 0, n_blend = 0;
    int item;
    for (int iter = 0; next_item(a, iter, item); ++iter) {
        int tid = (int)a.queue[item];
        int v = tid / a.T, tile = tid - v * a.T;
        int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
        int x0 = tx * TW, y0 = ty * TH;
        int xb = x0 & ~31, yb = y0 & ~31;
        uint2 rg = a.ranges[tid];
        float Tr[PPT], C0[PPT], C1[PPT], C2[PPT], px[PPT], py[PPT];
        int last[PPT];
        bool alive[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            int p = lane + 64 * k;
            int lx = p % TW, ly = p / TW;
            px[k] = (float)(x0 - xb + lx) + 0.5f;
            py[k] = (float)(y0 - yb + ly) + 0.5f;
            Tr[k] = 1.f;
            C0[k] = C1[k] = C2[k] = 0.f;
            last[k] = -1;
            alive[k] = (x0 + lx < a.W) && (y0 + ly < a.H);
        }
        Stage cur = stage_load(a, rg.x + lane, rg.y, nslots, (float)xb, (float)yb);
        for (uint32_t b = rg.x; b < rg.y; b += 64) {
            bool any = false;
#pragma unroll
            for (int k = 0; k < PPT; ++k) any |= alive[k];
            if (__ballot(any) == 0) break;
            Stage nxt = stage_load(a, b + 64 + lane, rg.y, nslots, (float)xb, (float)yb);
            int n = (int)min(64u, rg.y - b);
            for (int j = 0; j < n; ++j) {
                float mx = bcast(cur.mx, j), my = bcast(cur.my, j);
                float A = bcast(cur.A, j), Bc = bcast(cur.Bc, j), Cc = bcast(cur.Cc, j);
                float o = bcast(cur.o, j);
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    if (!alive[k]) continue;
                    if (STATS) ++n_eval;
                    float dx = px[k] - mx, dy = py[k] - my;
                    float al = fminf(a.amax, o * exp2_hw(power2(dx, dy, A, Bc, Cc)));
                    if (al < a.amin) continue;
                    float Tn = Tr[k] * (1.f - al);
                    if (Tn < a.tmin) {
                        alive[k] = false;
                        continue;
                    }
                    if (STATS) ++n_blend;
                    float w = al * Tr[k];
                    C0[k] = __fmaf_rn(bcast(cur.r, j), w, C0[k]);
                    C1[k] = __fmaf_rn(bcast(cur.g, j), w, C1[k]);
                    C2[k] = __fmaf_rn(bcast(cur.b, j), w, C2[k]);
                    Tr[k] = Tn;
                    last[k] = (int)(b + j);
                }
            }
            cur = nxt;
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            int p = lane + 64 * k;
            int gx = x0 + p % TW, gy = y0 + p / TW;
            if (gx >= a.W || gy >= a.H) continue;
            size_t o = (size_t)gy * a.W + gx;
            size_t vo = (size_t)v * HW;
            img[3 * vo + o] = __fmaf_rn(Tr[k], a.bg0, C0[k]);
            img[3 * vo + HW + o] = __fmaf_rn(Tr[k], a.bg1, C1[k]);
            img[3 * vo + 2 * HW + o] = __fmaf_rn(Tr[k], a.bg2, C2[k]);
            Tout[vo + o] = Tr[k];
            lastout[vo + o] = last[k];
        }
    }
    if (STATS) {
        stat_add(a.stats + 0, n_eval);
        stat_add(a.stats + 1, n_blend);
    }
}

template <int TW, int TH, bool STATS>
__global__ __launch_bounds__(64) void render_bwd_kernel(RenderArgs a, const float *dimg, const float *Tin,
                                                       const int32_t *lastin, float *grad2d) {
    constexpr int PPT = TW * TH / 64;
    const int lane = threadIdx.x;
    const size_t HW = (size_t)a.W * a.H;
    const uint32_t nslots = a.counts[CNT_SLOTS];
    unsigned long long n_eval = 0, n_contrib = 0, n_atomic = 0;
    int item;
    for (int iter = 0; next_item(a, iter, item); ++iter) {
        int tid = (int)a.queue[item];
        int v = tid / a.T, tile = tid - v * a.T;
        int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
        int x0 = tx * TW, y0 = ty * TH;
        int xb = x0 & ~31, yb = y0 & ~31;
        uint2 rg = a.ranges[tid];
        float Tr[PPT], S0[PPT], S1[PPT], S2[PPT], gc0[PPT], gc1[PPT], gc2[PPT], px[PPT], py[PPT];
        int last[PPT];
        int mymax = -1;
        size_t vo = (size_t)v * HW;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            int p = lane + 64 * k;
            int lx = p % TW, ly = p / TW;
            px[k] = (float)(x0 - xb + lx) + 0.5f;
            py[k] = (float)(y0 - yb + ly) + 0.5f;
            int gx = x0 + lx, gy = y0 + ly;
            last[k] = -1;
            Tr[k] = 1.f;
            gc0[k] = gc1[k] = gc2[k] = 0.f;
            if (gx < a.W && gy < a.H) {
                size_t o = (size_t)gy * a.W + gx;
                last[k] = lastin[vo + o];
                // a position outside this tile's list cannot come from render_fwd; ignore it
                if (last[k] < (int)rg.x || last[k] >= (int)rg.y) last[k] = -1;
                Tr[k] = Tin[vo + o];
                gc0[k] = dimg[3 * vo + o];
                gc1[k] = dimg[3 * vo + HW + o];
                gc2[k] = dimg[3 * vo + 2 * HW + o];
            }
            S0[k] = Tr[k] * a.bg0;
            S1[k] = Tr[k] * a.bg1;
            S2[k] = Tr[k] * a.bg2;
            mymax = max(mymax, last[k]);
        }
        // walk [rg.x, hi) backwards, hi = 1 + the wave's last contributor
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mymax = max(mymax, __shfl_xor(mymax, o, kWave));
        int hi = mymax + 1;
        if (hi <= (int)rg.x) continue;
        int e = hi;
        int bs = max((int)rg.x, e - 64);
        Stage cur = stage_load(a, (uint32_t)(bs + lane), (uint32_t)e, nslots, (float)xb, (float)yb);
        while (e > (int)rg.x) {
            int n = e - bs;
            int e2 = bs, bs2 = max((int)rg.x, bs - 64);
            Stage nxt = stage_load(a, (uint32_t)(bs2 + lane), (uint32_t)e2, nslots, (float)xb, (float)yb);
            for (int j = n - 1; j >= 0; --j) {
                int idx = bs + j;
                float mx = bcast(cur.mx, j), my = bcast(cur.my, j);
                float A = bcast(cur.A, j), Bc = bcast(cur.Bc, j), Cc = bcast(cur.Cc, j);
                float o = bcast(cur.o, j);
                float cr = bcast(cur.r, j), cg = bcast(cur.g, j), cb = bcast(cur.b, j);
                float gmx = 0.f, gmy = 0.f, ga = 0.f, gb = 0.f, gcc = 0.f, go = 0.f, gr = 0.f, gg = 0.f, gbl = 0.f;
                bool hit = false;
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    if (idx > last[k]) continue;
                    if (STATS) ++n_eval;
                    float dx = px[k] - mx, dy = py[k] - my;
                    float ex = exp2_hw(power2(dx, dy, A, Bc, Cc));
                    float av = o * ex;
                    float al = fminf(a.amax, av);
                    if (al < a.amin) continue;
                    if (STATS) ++n_contrib;
                    hit = true;
                    float iom = __builtin_amdgcn_rcpf(1.f - al);
                    float Tj = Tr[k] * iom;
                    float w = al * Tj;
                    gr = __fmaf_rn(w, gc0[k], gr);
                    gg = __fmaf_rn(w, gc1[k], gg);
                    gbl = __fmaf_rn(w, gc2[k], gbl);
                    float dal = gc0[k] * __fmaf_rn(cr, Tj, -S0[k] * iom) + gc1[k] * __fmaf_rn(cg, Tj, -S1[k] * iom) +
                                gc2[k] * __fmaf_rn(cb, Tj, -S2[k] * iom);
                    S0[k] = __fmaf_rn(cr, w, S0[k]);
                    S1[k] = __fmaf_rn(cg, w, S1[k]);
                    S2[k] = __fmaf_rn(cb, w, S2[k]);
                    Tr[k] = Tj;
                    if (av < a.amax) {
                        go = __fmaf_rn(dal, ex, go);
                        float dp = dal * al;
                        float hdx = 0.5f * dx, hdy = 0.5f * dy;
                        ga = __fmaf_rn(-dp * hdx, dx, ga);
                        gb = __fmaf_rn(-dp * dx, dy, gb);
                        gcc = __fmaf_rn(-dp * hdy, dy, gcc);
                        // d power / d mu = (a dx + b dy, b dx + c dy) with a = -2 ln2 A, b = -ln2 Bc, c = -2 ln2 Cc
                        gmx = __fmaf_rn(dp, -LN2 * __fmaf_rn(2.f * A, dx, Bc * dy), gmx);
                        gmy = __fmaf_rn(dp, -LN2 * __fmaf_rn(Bc, dx, 2.f * Cc * dy), gmy);
                    }
                }
                if (__ballot(hit) == 0) continue;
                float s0 = lane63(wave_sum63(gmx)), s1 = lane63(wave_sum63(gmy));
                float s2 = lane63(wave_sum63(ga)), s3 = lane63(wave_sum63(gb)), s4 = lane63(wave_sum63(gcc));
                float s5 = lane63(wave_sum63(go));
                float s6 = lane63(wave_sum63(gr)), s7 = lane63(wave_sum63(gg)), s8 = lane63(wave_sum63(gbl));
                uint32_t slot = (uint32_t)__builtin_amdgcn_readlane((int)cur.slot, j);
                if (STATS && lane == 0) ++n_atomic;
                if (lane < 9) {
                    float val = lane == 0 ? s0 : lane == 1 ? s1 : lane == 2 ? s2 : lane == 3 ? s3 :
                                lane == 4 ? s4 : lane == 5 ? s5 : lane == 6 ? s6 : lane == 7 ? s7 : s8;
                    atomicAdd(grad2d + 9 * (size_t)slot + lane, val);
                }
            }
            cur = nxt;
            e = e2;
            bs = bs2;
        }
    }
    if (STATS) {
        stat_add(a.stats + 2, n_eval);
        stat_add(a.stats + 3, n_contrib);
        stat_add(a.stats + 4, n_atomic);
    }
}

__global__ void zero_grad2d_kernel(const uint32_t *counts, float *g) {
    uint64_t n = (uint64_t)counts[CNT_SLOTS] * 9;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        g[i] = 0.f;
}

__global__ void reset_work_kernel(uint32_t *w) { *w = 0u; }

RenderArgs make_args(const splat_plan &p, void *ws, unsigned long long *stats) {
    RenderArgs a;
    a.rec = ws_at<float4>(ws, p.off_rec);
    a.vals = ws_at<uint32_t>(ws, p.off_vals) + (p.sorted_buf ? p.inst_cap : 0);
    a.ranges = ws_at<uint2>(ws, p.off_ranges);
    a.queue = ws_at<uint32_t>(ws, p.off_queue);
    a.work = ws_at<uint32_t>(ws, p.off_counts) + CNT_WORK;
    a.counts = ws_at<uint32_t>(ws, p.off_counts);
    a.stats = stats;
    a.n_items = p.n_views * p.tiles_per_view;
    a.T = p.tiles_per_view;
    a.tiles_x = p.tiles_x;
    a.W = p.width;
    a.H = p.height;
    a.persistent = p.s.persistent;
    a.amin = (float)p.s.alpha_min;
    a.amax = (float)p.s.alpha_max;
    a.tmin = (float)p.s.t_min;
    a.bg0 = (float)p.s.bg[0];
    a.bg1 = (float)p.s.bg[1];
    a.bg2 = (float)p.s.bg[2];
    return a;
}

int persistent_grid(int n_items, int wg_per_cu) {
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    int g = ncu * wg_per_cu;
    return g < n_items ? g : n_items;
}

template <int TW, int TH>
int fwd_impl(const splat_plan &p, void *ws, float *img, float *T, int32_t *last, unsigned long long *stats,
             hipStream_t st) {
    RenderArgs a = make_args(p, ws, stats);
    if (a.n_items == 0) return 0;
    int grid = a.n_items;
    if (a.persistent) {
        hipLaunchKernelGGL(reset_work_kernel, dim3(1), dim3(1), 0, st, a.work);
        int rc = launch_status("reset_work");
        if (rc) return rc;
        grid = persistent_grid(a.n_items, 32);
    }
    if (stats)
        hipLaunchKernelGGL((render_fwd_kernel<TW, TH, true>), dim3(grid), dim3(64), 0, st, a, img, T, last);
    else
        hipLaunchKernelGGL((render_fwd_kernel<TW, TH, false>), dim3(grid), dim3(64), 0, st, a, img, T, last);
    return launch_status("render_fwd");
}

template <int TW, int TH>
int bwd_impl(const splat_plan &p, void *ws, const float *dimg, const float *T, const int32_t *last,
             unsigned long long *stats, hipStream_t st) {
    RenderArgs a = make_args(p, ws, stats);
    float *g2 = ws_at<float>(ws, p.off_grad2d);
    uint32_t *counts = ws_at<uint32_t>(ws, p.off_counts);
    int zb = (int)((p.slot_cap * 9 + 255) / 256);
    if (zb > 8192) zb = 8192;
    hipLaunchKernelGGL(zero_grad2d_kernel, dim3(zb), dim3(256), 0, st, counts, g2);
    int rc = launch_status("zero_grad2d");
    if (rc || a.n_items == 0) return rc;
    int grid = a.n_items;
    if (a.persistent) {
        hipLaunchKernelGGL(reset_work_kernel, dim3(1), dim3(1), 0, st, a.work);
        if ((rc = launch_status("reset_work"))) return rc;
        grid = persistent_grid(a.n_items, 32);
    }
    if (stats)
        hipLaunchKernelGGL((render_bwd_kernel<TW, TH, true>), dim3(grid), dim3(64), 0, st, a, dimg, T, last, g2);
    else
        hipLaunchKernelGGL((render_bwd_kernel<TW, TH, false>), dim3(grid), dim3(64), 0, st, a, dimg, T, last, g2);
    return launch_status("render_bwd");
}

}  // namespace

int launch_render_fwd(const splat_plan &p, void *ws, float *img, float *T, int32_t *last, uint64_t *stats,
                      hipStream_t st) {
    int tw = p.s.tile_w, th = p.s.tile_h;
    auto *s = reinterpret_cast<unsigned long long *>(stats);
    if (tw == 16 && th == 16) return fwd_impl<16, 16>(p, ws, img, T, last, s, st);
    if (tw == 8 && th == 8) return fwd_impl<8, 8>(p, ws, img, T, last, s, st);
    if (tw == 16 && th == 32) return fwd_impl<16, 32>(p, ws, img, T, last, s, st);
    if (tw == 32 && th == 16) return fwd_impl<32, 16>(p, ws, img, T, last, s, st);
    set_error("render_fwd: unsupported tile %dx%d", tw, th);
    return SPLAT_EUNSUPPORTED;
}

int launch_render_bwd(const splat_plan &p, void *ws, const float *dimg, const float *T, const int32_t *last,
                      uint64_t *stats, hipStream_t st) {
    int tw = p.s.tile_w, th = p.s.tile_h;
    auto *s = reinterpret_cast<unsigned long long *>(stats);
    if (tw == 16 && th == 16) return bwd_impl<16, 16>(p, ws, dimg, T, last, s, st);
    if (tw == 8 && th == 8) return bwd_impl<8, 8>(p, ws, dimg, T, last, s, st);
    if (tw == 16 && th == 32) return bwd_impl<16, 32>(p, ws, dimg, T, last, s, st);
    if (tw == 32 && th == 16) return bwd_impl<32, 16>(p, ws, dimg, T, last, s, st);
    set_error("render_bwd: unsupported tile %dx%d", tw, th);
    return SPLAT_EUNSUPPORTED;
}

}  // namespace splat
