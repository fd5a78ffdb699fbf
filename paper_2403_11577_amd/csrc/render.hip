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
// gfx950 mapping: one wave64 workgroup per work item, TW*TH/64 pixels per lane
// (lane l owns pixel (l mod 8, l div 8) of every 8x8 sub-block).  A batch of 64
// Gaussian records is gathered one record per lane (the next batch is in flight
// while the current one is evaluated), staged in LDS and read back with
// wave-uniform addresses; a workgroup is one wave, so no barrier is needed.  The
// forward leaves a tile as soon as every pixel has stopped, skips sub-blocks
// that no live pixel of it can see, and takes two Gaussians per pass.  Work items
// come from a queue ordered by decreasing list length; the hardware dispatcher
// hands them out in order, or persistent waves pull them from a counter.
//
// Long lists.  A list of at least split_len instances is cut into chunks.  The
// forward records every pixel's (T, C) where each chunk starts, so the adjoint
// walks the chunks as separate work items; optionally the forward also
// composites chunks 1.. on their own and joins them (see the forward kernel).
// The forward also leaves, per instance, the sub-blocks it was blended into;
// the adjoint evaluates only those.
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
    const uint32_t *counts;     // device counts (slots, instances, split lists, adjoint items)
    const uint4 *bitems;        // adjoint work items (tile, chunk, first checkpoint slot, -)
    const uint32_t *boff;       // first checkpoint slot of each split queue position
    float4 *chk;                // checkpoints: per-pixel (T, C) of the split lists
    int32_t *chklast;           // last blended instance of a chunk composited on its own
    uint8_t *bmask;             // per instance: sub-blocks it was blended into (forward writes)
    float4 *g2z;                // the slots' gradient sums, cleared by the forward for the adjoint
    L1Fuse l1;                  // the L1 term at the forward's output stage (l1.target null: off)
    double *l1part;             // its sum of |C - target| per (view, tile)
    unsigned long long *stats;  // pair counters of the instrumented variant
    int n_items, T, tiles_x, W, H, persistent, roi_y0;
    uint32_t lc, chk_cap;       // split length, checkpoint slots
    float amin, amax, tmin, lamin2;  // lamin2 = log2(alpha_min)
    float bg0, bg1, bg2;
};

// One Gaussian as staged for a tile: mean relative to the enclosing 32x32
// block, conic pre-scaled by -1/2 log2(e) (A, Cc) and -log2(e) (Bc), log2 of the
// opacity (folded into the exponent: alpha = min(alpha_max, 2^(power2 + lo2))),
// 1/opacity, colour, and the mask of the tile's 8x8 sub-blocks that its
// alpha >= alpha_min footprint can reach (padded by 1% + 0.6 px; a sub-block
// outside it only ever evaluates alpha < alpha_min).
struct Stage {
    float mx, my, A, Bc, Cc, lo2, r, g, b;
    uint32_t slot, mask;
};

// The gather of a batch is split so that it can be in flight while the previous
// batch is evaluated: slot ids two batches ahead, raw records one batch ahead,
// and the derivation of the staged values after the evaluation loop.
struct Raw {
    float4 r0, r1, r2;
    uint32_t slot;
    uint32_t bm;  // adjoint: the sub-blocks the forward blended this instance into
};

__device__ __forceinline__ uint32_t load_slot(const RenderArgs &a, uint32_t idx, uint32_t end) {
    uint32_t v = a.vals[idx < end ? idx : 0u];  // vals[0] exists whenever this runs (end > 0)
    return idx < end ? v : 0xFFFFFFFFu;
}

__device__ __forceinline__ uint32_t load_bm(const RenderArgs &a, uint32_t idx, uint32_t end) {
    uint32_t v = a.bmask[idx < end ? idx : 0u];
    return idx < end ? v : 0u;
}

// Unconditional gather (a branch here would make the compiler wait for the data
// to merge registers): an invalid slot reads record 0, which always exists, and
// is marked invalid.  (A slot id outside the slot count cannot come out of the
// sort; it is treated as transparent.)
__device__ __forceinline__ Raw load_raw(const RenderArgs &a, uint32_t slot, uint32_t nslots) {
    Raw r;
    bool ok = slot < nslots;
    size_t s = ok ? (size_t)slot : 0;
    r.slot = ok ? slot : 0xFFFFFFFFu;
    r.bm = 0u;
    r.r0 = a.rec[3 * s + 0];
    r.r1 = a.rec[3 * s + 1];
    r.r2 = a.rec[3 * s + 2];
    return r;
}

// The adjoint (BM = true) takes the forward's blend mask instead of the footprint mask: a
// Gaussian reaches a pixel's colour only through a blend, so the mask is exact and tighter.
template <int TW, int TH, bool BM = false>
__device__ __forceinline__ Stage derive(const RenderArgs &a, const Raw &raw, float xb, float yb, float ox, float oy) {
    constexpr int SBX = TW / 8, NSB = TW * TH / 64;
    Stage s;
    s.slot = raw.slot;
    s.mx = (raw.r0.x - xb) + raw.r0.z;
    s.my = (raw.r0.y - yb) + raw.r0.w;
    s.A = -0.5f * LOG2E * raw.r1.x;
    s.Bc = -LOG2E * raw.r1.y;
    s.Cc = -0.5f * LOG2E * raw.r1.z;
    float o = raw.r1.w;
    bool valid = raw.slot != 0xFFFFFFFFu && o > 0.f;
    s.lo2 = valid ? __log2f(o) : -256.f;
    s.r = raw.r2.x;
    s.g = raw.r2.y;
    s.b = raw.r2.z;
    if (BM) {
        s.mask = valid ? raw.bm : 0u;
        asm volatile("" : "+v"(s.mx), "+v"(s.my), "+v"(s.A), "+v"(s.Bc), "+v"(s.Cc), "+v"(s.lo2));
        asm volatile("" : "+v"(s.r), "+v"(s.g), "+v"(s.b), "+v"(s.slot), "+v"(s.mask));
        return s;
    }
    // footprint box: half-widths k sqrt(Sigma2_ii), Sigma2 = conic^-1, k^2 = 2 ln(o / alpha_min)
    float ca = raw.r1.x, cb = raw.r1.y, cc = raw.r1.z;
    float idet = __builtin_amdgcn_rcpf(fmaxf(ca * cc - cb * cb, 1e-30f));
    float k2 = fmaxf(2.f * LN2 * (s.lo2 - a.lamin2), 0.f);
    float rx = sqrtf(k2 * cc * idet) * 1.01f + 0.6f;
    float ry = sqrtf(k2 * ca * idet) * 1.01f + 0.6f;
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < NSB; ++k) {
        float bx = ox + 8.f * (float)(k % SBX) + 0.5f;  // first pixel centre of the sub-block
        float by = oy + 8.f * (float)(k / SBX) + 0.5f;
        bool hit = (s.mx + rx >= bx) && (s.mx - rx <= bx + 7.f) && (s.my + ry >= by) && (s.my - ry <= by + 7.f);
        m |= hit ? (1u << k) : 0u;
    }
    s.mask = valid ? m : 0u;
    // keep the derived values materialised here: otherwise the compiler may
    // recompute them from the raw registers at the top of the next evaluation
    // loop, after the next gather has been issued, and wait for that gather
    asm volatile("" : "+v"(s.mx), "+v"(s.my), "+v"(s.A), "+v"(s.Bc), "+v"(s.Cc), "+v"(s.lo2));
    asm volatile("" : "+v"(s.r), "+v"(s.g), "+v"(s.b), "+v"(s.slot), "+v"(s.mask));
    return s;
}

__device__ __forceinline__ float bcast(float v, int j) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

__device__ __forceinline__ uint32_t bcast_u(uint32_t v, int j) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, j);
}

// A batch is staged in LDS as three float4 per Gaussian: (mx, my, A, Bc), (Cc, lo2, r, g),
// (b, -, slot, -); the pair loops read Gaussian j back with a wave-uniform address (one
// broadcast read per float4) instead of a readlane per value.  The workgroup is one wave,
// whose LDS accesses complete in order, so no barrier is needed between the batches.
__device__ __forceinline__ void put_stage(float4 (*sg)[3], const Stage &s, int lane) {
    sg[lane][0] = make_float4(s.mx, s.my, s.A, s.Bc);
    sg[lane][1] = make_float4(s.Cc, s.lo2, s.r, s.g);
    sg[lane][2] = make_float4(s.b, 0.f, __uint_as_float(s.slot), 0.f);
}

// exponent in log2 units including log2(opacity): A dx^2 + Bc dx dy + Cc dy^2 + lo2
__device__ __forceinline__ float power2(float dx, float dy, float A, float Bc, float Cc, float lo2) {
    return __fmaf_rn(dx, __fmaf_rn(A, dx, Bc * dy), __fmaf_rn(Cc * dy, dy, lo2));
}

__device__ __forceinline__ float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }

// alpha = min(alpha_max, 2^power) as one median-of-three: 2^power is never negative or NaN
// here (culled Gaussians carry finite parameters), where the result equals fminf's
__device__ __forceinline__ float alpha_of(float pw, float amax) {
    return __builtin_amdgcn_fmed3f(exp2_hw(pw), 0.f, amax);
}

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

// Work items: persistent waves pull them from a counter; otherwise workgroup b takes items
// b, b + grid, ... (the grid covers the forward's items; the adjoint can have a few more).
__device__ __forceinline__ bool next_item(const RenderArgs &a, int iter, int n, int &item) {
    if (a.persistent) {
        uint32_t it = 0;
        if (__lane_id() == 0) it = atomicAdd(a.work, 1u);
        item = __builtin_amdgcn_readfirstlane((int)it);
    } else {
        item = (int)blockIdx.x + iter * (int)gridDim.x;
    }
    return item < n;
}

// checkpoint of a split list: the per-pixel (T, C) of one tile
template <int NSB>
__device__ __forceinline__ void put_chk(const RenderArgs &a, uint32_t slot, const float (&T)[NSB],
                                        const float (&C0)[NSB], const float (&C1)[NSB], const float (&C2)[NSB],
                                        int lane) {
    if (slot >= a.chk_cap) return;  // cannot happen: the capacity bounds every split list's chunks
    float4 *d = a.chk + (size_t)slot * (NSB * 64) + lane;
#pragma unroll
    for (int k = 0; k < NSB; ++k) d[k * 64] = make_float4(T[k], C0[k], C1[k], C2[k]);
}

// Pixel layout: lane l covers pixel (l & 7, l >> 3) of every 8x8 sub-block k of
// the tile (k row-major over the TW/8 x TH/8 sub-blocks).
//
// Forward state per pixel: the transmittance T and its live copy L, equal to T
// while the pixel composites and 0 once it has stopped.  The weight of a pair is
// alpha L, so a stopped pixel runs the same instructions without effect; when a
// blend would take T below t_min, L drops to 0 and T keeps its value.  Sub-blocks
// whose 64 pixels have all stopped are skipped from the next batch on.
//
// STATS = true is the instrumented variant (pair counters for the roofline);
// it computes exactly the same outputs.
//
// MODE 0 composites every list in order.  A split list (at least split_len
// instances) records (T, C) where each of its chunks starts, for the adjoint.
// MODE 1 composites chunks 1.. of every split list on their own, from T = 1 with
// the same stop rule, and stores per pixel (T_chunk or -1 if the pixel stopped
// inside the chunk, C_chunk) and the chunk's last blended instance in the chunk's
// checkpoint slot.  MODE 2 is MODE 0 that, at the start of chunk c >= 1, joins the
// chunk's own result instead of walking it (C += T C_chunk, T *= T_chunk, last =
// last_chunk) unless some live pixel of the tile could reach t_min inside it:
// T T_chunk >= t_min (1 + margin) with T_chunk >= t_min guarantees that the
// sequential walk (T decreasing monotonically) stops nowhere in the chunk, the
// margin covering the rounding by which the sequential product can differ.
template <int TW, int TH, bool STATS, int MODE, int NB>
__global__ __launch_bounds__(64) void render_fwd_kernel(RenderArgs a, float *img, float *Tout, int32_t *lastout) {
    constexpr int NSB = TW * TH / 64, SBX = TW / 8, NPIX = TW * TH;
    constexpr int R = NB >= 64 ? NB / 64 : 1;      // sub-batches of 64 staged at once
    __shared__ float4 sg[R * 64][3];  // the staged batch, read back with wave-uniform addresses
    const int lane = threadIdx.x;
    const int lx = lane & 7, ly = lane >> 3;
    const bool stager = NB >= 64 || lane < NB;     // lanes that gather a Gaussian of the batch
    const size_t HW = (size_t)a.W * a.H;
    const uint32_t nslots = a.counts[CNT_SLOTS];
    const uint32_t nsplit = a.counts[CNT_NSPLIT];
    const int n_items = MODE == 1 ? (int)min(a.counts[CNT_NCHUNK], a.chk_cap) : a.n_items;
    const float thr = a.tmin * (1.001f + 1.2e-7f * (float)a.lc);
    unsigned long long n_eval = 0, n_blend = 0, w_eval = 0, w_blend = 0;
    int item;
    for (int iter = 0; MODE == 1 ? (item = (int)blockIdx.x + iter * (int)gridDim.x) < n_items
                                  : next_item(a, iter, n_items, item);
         ++iter) {
        if (MODE != 1) {
            // the adjoint adds into the slots' nine gradient sums: work item i clears its share of
            // them (the kernel is bound by its instructions, the stores cost it little; the
            // region is padded to 256 bytes, so the last float4 stays inside it)
            const uint32_t n4 = (a.counts[CNT_SLOTS] * 9u + 3u) / 4u;
            const uint32_t per = (n4 + (uint32_t)n_items - 1u) / (uint32_t)n_items;
            const uint32_t q1 = min((uint32_t)item * per + per, n4);
            for (uint32_t q = (uint32_t)item * per + lane; q < q1; q += 64u) a.g2z[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        int tid;
        uint32_t lo, hi, lslot = 0;
        uint2 rg;
        if (MODE == 1) {
            const uint4 it = a.bitems[item];
            if (it.y == 0u || it.z == 0xFFFFFFFFu) continue;  // the first chunk is walked by MODE 2
            tid = (int)it.x;
            rg = a.ranges[tid];
            lo = rg.x + it.y * a.lc;
            hi = min(rg.y, lo + a.lc);
            lslot = it.z + it.y;
            if (lo >= rg.y || lslot >= a.chk_cap) continue;  // cannot happen
        } else {
            tid = (int)a.queue[item];
            rg = a.ranges[tid];
            lo = rg.x;
            hi = rg.y;
        }
        int v = tid / a.T, tile = tid - v * a.T;
        int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
        int x0 = tx * TW, y0 = ty * TH;
        int xb = x0 & ~31, yb = y0 & ~31;
        float T[NSB], L[NSB], C0[NSB], C1[NSB], C2[NSB], px[NSB], py[NSB];
        int last[NSB];
#pragma unroll
        for (int k = 0; k < NSB; ++k) {
            int qx = 8 * (k % SBX) + lx, qy = 8 * (k / SBX) + ly;
            px[k] = (float)(x0 - xb + qx) + 0.5f;
            py[k] = (float)(y0 - yb + qy) + 0.5f;
            T[k] = (x0 + qx < a.W && y0 + qy < a.H) ? 1.f : 0.f;
            L[k] = y0 + qy >= a.roi_y0 ? T[k] : 0.f;  // above the region of interest: background, T = 1
            C0[k] = C1[k] = C2[k] = 0.f;
            last[k] = -1;
        }
        const float fxb = (float)xb, fyb = (float)yb, fox = (float)(x0 - xb), foy = (float)(y0 - yb);
        // the batch [b, b + NB): sub-batch r holds instances b + 64 r + lane; the staged values go to
        // LDS, each lane keeps the sub-block masks of its Gaussians
        uint32_t cmask[R], sl_next[R];
        auto slot_at = [&](uint32_t base, int r) {
            return stager ? load_slot(a, base + 64u * r + lane, hi) : 0xFFFFFFFFu;
        };
        auto stage = [&](uint32_t base) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                Stage c = derive<TW, TH>(a, load_raw(a, slot_at(base, r), nslots), fxb, fyb, fox, foy);
                put_stage(sg + 64 * r, c, lane);
                cmask[r] = c.mask;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) sl_next[r] = slot_at(base + NB, r);
        };
        stage(lo);
        // a split list records (T, C) where each of its chunks starts (chunks are whole batches)
        const bool split = MODE != 1 && (uint32_t)item < nsplit;
        const uint32_t cslot = split ? a.boff[item] : 0u;
        uint32_t bnext = split ? rg.x + a.lc : 0xFFFFFFFFu, cnext = cslot + 1;
        // MODE 2, a chunk walked in order: its live pixels that cannot stop in it are joined at
        // once and parked (L = 0) until the chunk ends at park_end; the walk ends early when
        // the other pixels have stopped
        bool parked = false;
        uint32_t park_end = 0u;
        float parkL[NSB];
#pragma unroll
        for (int k = 0; k < NSB; ++k) parkL[k] = 0.f;
        for (uint32_t b = lo; b < hi; b += NB) {
            if (MODE == 2 && parked && b == park_end) {
#pragma unroll
                for (int k = 0; k < NSB; ++k) L[k] = parkL[k] > 0.f ? parkL[k] : L[k];
                parked = false;
            }
            if (b == bnext) {
                bool joined = false, wrote = false;
                if (MODE == 2 && cnext < a.chk_cap) {
                    const float4 *src = a.chk + (size_t)cnext * NPIX + lane;
                    bool need = false;
#pragma unroll
                    for (int k = 0; k < NSB; ++k) need |= L[k] > 0.f && !(T[k] * src[k * 64].x >= thr);
                    joined = __ballot(need) == 0ull;
                    const int32_t *lsrc = a.chklast + (size_t)cnext * NPIX + lane;
                    float4 *dst = a.chk + (size_t)cnext * NPIX + lane;
                    bool any_park = false;
#pragma unroll
                    for (int k = 0; k < NSB; ++k) {
                        const float4 q = src[k * 64];
                        const int ll = lsrc[k * 64];
                        dst[k * 64] = make_float4(T[k], C0[k], C1[k], C2[k]);  // state where chunk c starts
                        const bool jk = L[k] > 0.f && T[k] * q.x >= thr;    // cannot stop in the chunk
                        if (jk) {
                            C0[k] = __fmaf_rn(L[k], q.y, C0[k]);
                            C1[k] = __fmaf_rn(L[k], q.z, C1[k]);
                            C2[k] = __fmaf_rn(L[k], q.w, C2[k]);
                            T[k] = T[k] * q.x;
                            L[k] = T[k];
                            last[k] = ll >= 0 ? ll : last[k];
                        }
                        if (!joined) {
                            parkL[k] = jk ? L[k] : 0.f;
                            L[k] = jk ? 0.f : L[k];
                            any_park |= jk;
                        }
                    }
                    wrote = true;
                    if (!joined && __ballot(any_park) != 0ull) {
                        parked = true;
                        park_end = bnext + a.lc;
                    }
                }
                if (!wrote) put_chk<NSB>(a, cnext, T, C0, C1, C2, lane);
                ++cnext;
                bnext += a.lc;
                if (joined) {
                    // continue at the next chunk: restage its first batch
                    const uint32_t bn = b + a.lc;
                    stage(bn);
                    b = bn - NB;
                    continue;
                }
            }
            uint32_t live = 0;  // sub-blocks with a pixel still compositing
#pragma unroll
            for (int k = 0; k < NSB; ++k) live |= __ballot(L[k] > 0.f) ? (1u << k) : 0u;
            if (live == 0) {
                if (MODE == 2 && parked && park_end < hi) {
                    // the walking pixels have stopped: the parked ones resume where the chunk ends
                    stage(park_end);
                    b = park_end - NB;
                    continue;
                }
                break;  // every pixel has stopped (parked ones already hold the state at the list end)
            }
            Raw raw_next[R];
            uint32_t sl_after[R];
#pragma unroll
            for (int r = 0; r < R; ++r) raw_next[r] = load_raw(a, sl_next[r], nslots);  // records of batch b + NB
#pragma unroll
            for (int r = 0; r < R; ++r) sl_after[r] = slot_at(b + 2 * NB, r);         // slot ids of batch b + 2 NB
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r > 0) {
                    live = 0;
#pragma unroll
                    for (int k = 0; k < NSB; ++k) live |= __ballot(L[k] > 0.f) ? (1u << k) : 0u;
                }
                const uint32_t bb = b + 64u * r;   // first instance of the sub-batch
                const float4(*sgr)[3] = sg + 64 * r;
                uint64_t blended[NSB];  // per sub-block: the Gaussians of the sub-batch that blended into it
#pragma unroll
                for (int k = 0; k < NSB; ++k) blended[k] = 0ull;
                // the Gaussians of the sub-batch that reach a live sub-block, in order (lanes past the
                // list end carry an empty mask)
                uint64_t todo = __ballot((cmask[r] & live) != 0u);
                // two Gaussians per pass: the staged values of both are read before the first is
                // evaluated, so the second read is in flight meanwhile (without a second one the pass
                // evaluates the first again with zero opacity, which blends nothing)
                auto blend = [&](int j, const float4 q0, const float4 q1, const float cb, bool real) {
                    // with one sub-block every Gaussian of the ballot reaches it
                    const uint32_t m = NSB == 1 ? 1u : bcast_u(cmask[r], j) & live;
                    const float mx = q0.x, my = q0.y, A = q0.z, Bc = q0.w, Cc = q1.x, lo2 = q1.y;
                    const float cr = q1.z, cg = q1.w;
                    const int idx = (int)(bb + j);
#pragma unroll
                    for (int k = 0; k < NSB; ++k) {
                        if (!(m & (1u << k))) continue;  // wave-uniform
                        if (STATS) n_eval += real && L[k] > 0.f;
                        if (STATS) w_eval += lane == 0;
                        float dx = px[k] - mx, dy = py[k] - my;
                        const float pw = power2(dx, dy, A, Bc, Cc, lo2);
                        // no live pixel of the sub-block within reach of alpha_min: nothing blends
                        // (2^(log2 alpha_min - 0.01) is below alpha_min by far more than the rounding)
                        if (__ballot(L[k] > 0.f && pw >= a.lamin2 - 0.01f) == 0ull) continue;
                        if (STATS) w_blend += lane == 0;
                        float al = alpha_of(pw, a.amax);
                        al = al >= a.amin ? al : 0.f;
                        float w = al * L[k];
                        float Tn = T[k] - w;
                        bool stop = Tn < a.tmin;  // cannot hold for a stopped pixel: its T stays >= t_min
                        w = stop ? 0.f : w;
                        T[k] = stop ? T[k] : Tn;
                        L[k] = stop ? 0.f : L[k] - w;
                        if (STATS) n_blend += w > 0.f;
                        C0[k] = __fmaf_rn(cr, w, C0[k]);
                        C1[k] = __fmaf_rn(cg, w, C1[k]);
                        C2[k] = __fmaf_rn(cb, w, C2[k]);
                        last[k] = w > 0.f ? idx : last[k];
                        blended[k] |= __ballot(w > 0.f) ? (1ull << j) : 0ull;
                    }
                };
                while (todo) {
                    const int j1 = __ffsll((long long)todo) - 1;
                    todo &= todo - 1ull;
                    const bool two = todo != 0ull;
                    const int j2 = two ? __ffsll((long long)todo) - 1 : j1;
                    todo &= todo - 1ull;
                    const float4 a0 = sgr[j1][0], a1 = sgr[j1][1], b0 = sgr[j2][0];
                    float4 b1 = sgr[j2][1];
                    const float a2 = sgr[j1][2].x, b2 = sgr[j2][2].x;
                    b1.y = two ? b1.y : -256.f;  // log2 of the opacity: alpha = 0 < alpha_min
                    blend(j1, a0, a1, a2, true);
                    blend(j2, b0, b1, b2, two);
                }
                if (stager) {
                    uint32_t bm = 0;
#pragma unroll
                    for (int k = 0; k < NSB; ++k) bm |= ((blended[k] >> lane) & 1ull) ? (1u << k) : 0u;
                    // with parked pixels the chunk's own pass holds their blends (a superset is exact)
                    if (MODE == 2 && parked && bb + lane < hi) bm |= a.bmask[bb + lane];
                    if (bb + lane < hi) a.bmask[bb + lane] = (uint8_t)bm;
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                Stage c = derive<TW, TH>(a, raw_next[r], fxb, fyb, fox, foy);
                put_stage(sg + 64 * r, c, lane);
                cmask[r] = c.mask;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) sl_next[r] = sl_after[r];
        }
        if (MODE == 1) {
            // the chunk on its own: (T_chunk, C_chunk), T_chunk = -1 where the pixel stopped in it
            float4 *d = a.chk + (size_t)lslot * NPIX + lane;
            int32_t *dl = a.chklast + (size_t)lslot * NPIX + lane;
#pragma unroll
            for (int k = 0; k < NSB; ++k) {
                bool inside = x0 + 8 * (k % SBX) + lx < a.W && y0 + 8 * (k / SBX) + ly < a.H && y0 + 8 * (k / SBX) + ly >= a.roi_y0;
                d[k * 64] = make_float4(inside && !(L[k] > 0.f) ? -1.f : T[k], C0[k], C1[k], C2[k]);
                dl[k * 64] = last[k];
            }
            continue;
        }
        if (split) {
            // chunks after an early exit start from the final state, which the first slot also holds
            const uint32_t cend = cslot + (rg.y - rg.x + a.lc - 1) / a.lc;
            for (; cnext < cend; ++cnext) put_chk<NSB>(a, cnext, T, C0, C1, C2, lane);
            put_chk<NSB>(a, cslot, T, C0, C1, C2, lane);
        }
        size_t vo = (size_t)v * HW;
        double l1acc = 0.0;
#pragma unroll
        for (int k = 0; k < NSB; ++k) {
            int gx = x0 + 8 * (k % SBX) + lx, gy = y0 + 8 * (k / SBX) + ly;
            if (gx >= a.W || gy >= a.H) continue;
            size_t o = (size_t)gy * a.W + gx;
            float Tfin = T[k];
            const float c[3] = {__fmaf_rn(Tfin, a.bg0, C0[k]), __fmaf_rn(Tfin, a.bg1, C1[k]),
                                __fmaf_rn(Tfin, a.bg2, C2[k])};
            img[3 * vo + o] = c[0];
            img[3 * vo + HW + o] = c[1];
            img[3 * vo + 2 * HW + o] = c[2];
            Tout[vo + o] = Tfin;
            lastout[vo + o] = last[k];
            if (a.l1.target) {
                // the L1 term of this pixel, as the loss kernel forms it from the stored image
                const bool in = gy >= a.roi_y0 && !(a.l1.mask && a.l1.mask[vo + o]);
                const float g = (float)a.l1.inv_n;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const size_t q = 3 * vo + (size_t)ch * HW + o;
                    float d = c[ch] - a.l1.target[q];
                    d = in ? d : 0.f;
                    a.l1.dimg[q] = d > 0.f ? g : (d < 0.f ? -g : 0.f);
                    l1acc += (double)fabsf(d);
                }
            }
        }
        if (a.l1.target && a.l1.loss) {
            // one partial per (view, tile), summed in that order after the launch (the work
            // queue's order within a cost class varies between calls; a device-wide atomic per
            // item on one address serialises at the memory side)
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) l1acc += __shfl_xor(l1acc, off, kWave);
            if (lane == 0) a.l1part[tid] = l1acc;
        }
    }
    if (STATS) {
        stat_add(a.stats + 0, n_eval);
        stat_add(a.stats + 1, n_blend);
        stat_add(a.stats + 5, w_eval);
        stat_add(a.stats + 6, w_blend);
    }
}

// Transposed reduction of nine per-lane values over the wave.  Four exchange
// steps inside each 16-lane row, with partners lane^1, lane^2, lane^7 and
// lane^15 (quad permutes, half-row mirror, row mirror: one DPP add each), halve
// the number of values a lane carries at every step; afterwards lane i of every
// row holds the row sum of value number cls(i) = c0 + 2 c1 + 4 c2 + 8 c3, with
// c0 = b0^b2, c1 = b1^b2, c2 = b2^b3, c3 = b3 for the bits b of i (the dual
// basis of {1, 2, 7, 15}, so partners always agree on the bits fixed so far).
// Two cross-row exchanges then give every lane the wave total of its value.
// Numbers 9..15 only ever carry padding.  27 VALU operations for nine sums,
// where nine separate reductions would take about a hundred.
template <int CTRL>
__device__ __forceinline__ float xpair(float lo, float hi, bool c) {
    float keep = c ? hi : lo, send = c ? lo : hi;
    return keep + dpp_f<CTRL, 0xF>(send);
}

template <int CTRL>
__device__ __forceinline__ float xpad(float v) { return v + dpp_f<CTRL, 0xF>(v); }

__device__ __forceinline__ float reduce9(const float (&v)[9], bool c0, bool c1, bool c2, bool c3) {
    float a0 = xpair<0xB1>(v[0], v[1], c0), a1 = xpair<0xB1>(v[2], v[3], c0);
    float a2 = xpair<0xB1>(v[4], v[5], c0), a3 = xpair<0xB1>(v[6], v[7], c0);
    float a4 = xpad<0xB1>(v[8]);
    float b0 = xpair<0x4E>(a0, a1, c1), b1 = xpair<0x4E>(a2, a3, c1), b2 = xpad<0x4E>(a4);
    float d0 = xpair<0x141>(b0, b1, c2), d1 = xpad<0x141>(b2);
    float e = xpair<0x140>(d0, d1, c3);
    e += __shfl_xor(e, 16, kWave);
    e += __shfl_xor(e, 32, kWave);
    return e;
}

// Backward: each pixel walks from its last contributor towards the list start,
// recovering T_j = T_{j+1} / (1 - alpha_j), and forms
//   dL/dc_j     = alpha_j T_j dL/dC
//   dL/dalpha_j = dL/dC . (c_j T_j - S_j / (1 - alpha_j)),
// S_j = sum_{i>j} c_i alpha_i T_i + T_final bg being the colour behind j.  Only
// the scalar P_j = dL/dC . S_j is kept per pixel (P += w dL/dC . c_j).  Then
// dL/dpower = alpha dL/dalpha and dL/do = dL/dalpha alpha / o (unless alpha was
// clamped at alpha_max); dL/d(conic) and dL/d(mean) follow from the power.
// Lanes that do not blend a Gaussian run the same instructions with alpha = 0,
// which changes nothing (1 / (1 - 0) = 1 exactly).
// Six waves per SIMD: the register budget (80) then spills a few values to scratch, which
// measured about 2 % faster than five waves without spills.
template <int TW, int TH, bool STATS, int NB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6))) void render_bwd_kernel(RenderArgs a, const float *dimg, const float *Tin,
                                                       const int32_t *lastin, float *grad2d) {
    constexpr int NSB = TW * TH / 64, SBX = TW / 8;
    constexpr int R = NB >= 64 ? NB / 64 : 1;      // sub-batches of 64 staged at once
    __shared__ float4 sg[R * 64][3];  // the staged batch (see put_stage)
    const int lane = threadIdx.x;
    const int lx = lane & 7, ly = lane >> 3;
    const bool stager = NB >= 64 || lane < NB;
    const size_t HW = (size_t)a.W * a.H;
    const uint32_t nslots = a.counts[CNT_SLOTS];
    // reduction classes of this lane (see reduce9) and the lanes that write them
    const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
    const bool c0 = b0 ^ b2, c1 = b1 ^ b2, c2 = b2 ^ b3, c3 = b3;
    const int cls = (int)c0 | ((int)c1 << 1) | ((int)c2 << 2) | ((int)c3 << 3);
    const bool writer = lane < 16 && cls < 9;
    unsigned long long n_eval = 0, n_contrib = 0, n_atomic = 0, w_eval = 0;
    const int n_items = (int)min(a.counts[CNT_BITEMS], (uint32_t)a.n_items);
    int item;
    for (int iter = 0; next_item(a, iter, n_items, item); ++iter) {
        const uint4 it = a.bitems[item];
        int tid = (int)it.x;
        int v = tid / a.T, tile = tid - v * a.T;
        int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
        int x0 = tx * TW, y0 = ty * TH;
        int xb = x0 & ~31, yb = y0 & ~31;
        uint2 rg = a.ranges[tid];
        // the walk covers [cs, ce): the whole list, or chunk it.y of a split list; a chunk other
        // than the last starts from the checkpoint where the next chunk starts
        int cs = (int)rg.x, ce = (int)rg.y;
        bool from_chk = false;
        size_t qoff = 0, foff = 0;
        if (it.z != 0xFFFFFFFFu) {
            uint32_t nc = (rg.y - rg.x + a.lc - 1) / a.lc;
            cs = (int)(rg.x + it.y * a.lc);
            ce = min((int)rg.y, cs + (int)a.lc);
            from_chk = it.y + 1 < nc;
            if (it.z + it.y + 1 >= a.chk_cap || it.y >= nc) continue;  // cannot happen (capacity bound)
            qoff = (size_t)(it.z + it.y + 1) * (NSB * 64) + lane;
            foff = (size_t)it.z * (NSB * 64) + lane;
        }
        float T[NSB], P[NSB], gc0[NSB], gc1[NSB], gc2[NSB], px[NSB], py[NSB];
        int last[NSB], kmax[NSB];
        size_t vo = (size_t)v * HW;
        int wmax = -1;
#pragma unroll
        for (int k = 0; k < NSB; ++k) {
            int qx = 8 * (k % SBX) + lx, qy = 8 * (k / SBX) + ly;
            px[k] = (float)(x0 - xb + qx) + 0.5f;
            py[k] = (float)(y0 - yb + qy) + 0.5f;
            int gx = x0 + qx, gy = y0 + qy;
            last[k] = -1;
            T[k] = 1.f;
            gc0[k] = gc1[k] = gc2[k] = 0.f;
            if (gx < a.W && gy < a.H) {
                size_t o = (size_t)gy * a.W + gx;
                last[k] = lastin[vo + o];
                // a position outside this tile's list cannot come from render_fwd; ignore it
                if (last[k] < (int)rg.x || last[k] >= (int)rg.y) last[k] = -1;
                T[k] = Tin[vo + o];
                gc0[k] = dimg[3 * vo + o];
                gc1[k] = dimg[3 * vo + HW + o];
                gc2[k] = dimg[3 * vo + 2 * HW + o];
            }
            P[k] = T[k] * (gc0[k] * a.bg0 + gc1[k] * a.bg1 + gc2[k] * a.bg2);
            if (from_chk) {
                // colour behind the chunk: C_final - C(ce) plus the background
                const float4 q = a.chk[qoff + k * 64], f = a.chk[foff + k * 64];
                P[k] += __fmaf_rn(gc2[k], f.w - q.w, __fmaf_rn(gc1[k], f.z - q.z, gc0[k] * (f.y - q.y)));
                T[k] = q.x;
            }
            int mk = min(last[k], ce - 1);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) mk = max(mk, __shfl_xor(mk, o, kWave));
            kmax[k] = __builtin_amdgcn_readfirstlane(mk);  // per sub-block: walk no further than this
            wmax = max(wmax, kmax[k]);
        }
        int hi = wmax + 1;  // walk [cs, hi) backwards
        if (hi <= cs) continue;
        const float fxb = (float)xb, fyb = (float)yb, fox = (float)(x0 - xb), foy = (float)(y0 - yb);
        // batches [bs, e) of up to NB instances from the end of the walk; sub-batch r holds
        // instances bs + 64 r + lane
        uint32_t cmask[R], sl_next[R], bm_next[R];
        auto slot_at = [&](int base, int r, int end) {
            return stager ? load_slot(a, (uint32_t)(base + 64 * r + lane), (uint32_t)end) : 0xFFFFFFFFu;
        };
        auto bm_at = [&](int base, int r, int end) {
            return stager ? load_bm(a, (uint32_t)(base + 64 * r + lane), (uint32_t)end) : 0u;
        };
        int e = hi;
        int bs = max(cs, e - NB);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            Raw raw0 = load_raw(a, slot_at(bs, r, e), nslots);
            raw0.bm = bm_at(bs, r, e);
            Stage c = derive<TW, TH, true>(a, raw0, fxb, fyb, fox, foy);
            put_stage(sg + 64 * r, c, lane);
            cmask[r] = c.mask;
        }
        int bs2 = max(cs, bs - NB);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            sl_next[r] = slot_at(bs2, r, bs);
            bm_next[r] = bm_at(bs2, r, bs);
        }
        while (e > cs) {
            int e2 = bs;
            int bs3 = max(cs, bs2 - NB);
            Raw raw_next[R];
            uint32_t sl_after[R], bm_after[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                raw_next[r] = load_raw(a, sl_next[r], nslots);  // batch [bs2, bs)
                raw_next[r].bm = bm_next[r];
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                sl_after[r] = slot_at(bs3, r, bs2);  // batch [bs3, bs2)
                bm_after[r] = bm_at(bs3, r, bs2);
            }
#pragma unroll
            for (int rr = R - 1; rr >= 0; --rr) {
                const int sb = bs + 64 * rr;   // first instance of the sub-batch
                const int n = e - sb;          // instances of the batch at or after sb
                if (n <= 0) continue;          // wave-uniform: the sub-batch lies past the walk's end
                const float4(*sgr)[3] = sg + 64 * rr;
                // the sub-batch's Gaussians with a footprint in the tile, last first (lanes at or past
                // n carry an empty mask)
                uint64_t todo = __ballot(cmask[rr] != 0u && lane < n);
                while (todo) {
                    const int j = 63 - __builtin_clzll(todo);
                    todo &= ~(1ull << j);
                    const float4 q0 = sgr[j][0], q1 = sgr[j][1], q2 = sgr[j][2];
                    // with one sub-block every Gaussian of the ballot reaches it
                    const uint32_t m = NSB == 1 ? 1u : bcast_u(cmask[rr], j);
                    int idx = sb + j;
                    const float mx = q0.x, my = q0.y, A = q0.z, Bc = q0.w, Cc = q1.x, lo2 = q1.y;
                    const float cr = q1.z, cg = q1.w, cb = q2.x;
                    // per-lane sums of dp = dL/dpower and its moments in (dx, dy), and of the colour weights
                    float m0 = 0.f, mx1 = 0.f, my1 = 0.f, mxx = 0.f, mxy = 0.f, myy = 0.f, gr = 0.f, gg = 0.f,
                          gbl = 0.f;
                    bool hit_any = false;
#pragma unroll
                    for (int k = 0; k < NSB; ++k) {
                        if (!(m & (1u << k)) || idx > kmax[k]) continue;  // wave-uniform
                        float dx = px[k] - mx, dy = py[k] - my;
                        float al = alpha_of(power2(dx, dy, A, Bc, Cc, lo2), a.amax);
                        bool hit = (idx <= last[k]) && (al >= a.amin);
                        if (STATS) n_eval += idx <= last[k];
                        if (STATS) w_eval += lane == 0;
                        if (__ballot(hit) == 0) continue;  // wave-uniform
                        hit_any = true;
                        if (STATS) n_contrib += hit;
                        float ah = hit ? al : 0.f;
                        float iom = __builtin_amdgcn_rcpf(1.f - ah);
                        float Tj = T[k] * iom;
                        float w = ah * Tj;
                        float gdc = __fmaf_rn(gc2[k], cb, __fmaf_rn(gc1[k], cg, gc0[k] * cr));
                        gr = __fmaf_rn(w, gc0[k], gr);
                        gg = __fmaf_rn(w, gc1[k], gg);
                        gbl = __fmaf_rn(w, gc2[k], gbl);
                        float dal = __fmaf_rn(Tj, gdc, -(iom * P[k]));
                        P[k] = __fmaf_rn(w, gdc, P[k]);
                        T[k] = Tj;
                        float dp = al < a.amax ? dal * ah : 0.f;  // no gradient through the alpha_max clamp
                        float tx = dp * dx, tyv = dp * dy;
                        m0 += dp;
                        mx1 += tx;
                        my1 += tyv;
                        mxx = __fmaf_rn(tx, dx, mxx);
                        mxy = __fmaf_rn(tx, dy, mxy);
                        myy = __fmaf_rn(tyv, dy, myy);
                    }
                    if (!hit_any) continue;
                    // the slot's gradient is left as the moments of dL/dpower (the projection adjoint
                    // turns them into dL/dmu, dL/dconic and dL/do with its own conic and opacity:
                    // all linear in the moments, so the sum over tiles commutes with it)
                    uint32_t slot = __float_as_uint(q2.z);
                    float vals[9] = {mx1, my1, mxx, mxy, myy, m0, gr, gg, gbl};
                    float tot = reduce9(vals, c0, c1, c2, c3);
                    if (STATS && lane == 0) ++n_atomic;
                    if (writer) atomicAdd(grad2d + 9 * (size_t)slot + cls, tot);
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                Stage c = derive<TW, TH, true>(a, raw_next[r], fxb, fyb, fox, foy);
                put_stage(sg + 64 * r, c, lane);
                cmask[r] = c.mask;
                sl_next[r] = sl_after[r];
                bm_next[r] = bm_after[r];
            }
            e = e2;
            bs = bs2;
            bs2 = bs3;
        }
    }
    if (STATS) {
        stat_add(a.stats + 2, n_eval);
        stat_add(a.stats + 3, n_contrib);
        stat_add(a.stats + 4, n_atomic);
        stat_add(a.stats + 7, w_eval);
    }
}

__global__ void reset_work_kernel(uint32_t *w) { *w = 0u; }

// Fixed-order sum of the forward's L1 partials: workgroup g adds partials [g kL1Span, (g+1) kL1Span)
// (thread t those at t mod 256, then a tree over the threads) into out[g]; given loss, the one
// workgroup adds scale times the sum of all n into *loss instead.
__global__ __launch_bounds__(256) void l1_sum_kernel(const double *in, int n, double *out, double scale,
                                                     double *loss) {
    __shared__ double s[256];
    const int t = threadIdx.x;
    const int b = loss ? 0 : (int)blockIdx.x * kL1Span;
    const int e = loss ? n : min(n, b + kL1Span);
    double acc = 0.0;
    for (int i = b + t; i < e; i += 256) acc += in[i];
    s[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) s[t] += s[t + w];
        __syncthreads();
    }
    if (t == 0) {
        if (loss)
            atomicAdd(loss, s[0] * scale);
        else
            out[blockIdx.x] = s[0];
    }
}

RenderArgs make_args(const splat_plan &p, void *ws, unsigned long long *stats) {
    RenderArgs a;
    a.rec = ws_at<float4>(ws, p.off_rec);
    a.vals = ws_at<uint32_t>(ws, p.off_vals) + (p.sorted_buf ? p.inst_cap : 0);
    a.ranges = ws_at<uint2>(ws, p.off_ranges);
    a.queue = ws_at<uint32_t>(ws, p.off_queue);
    a.work = ws_at<uint32_t>(ws, p.off_counts) + CNT_WORK;
    a.counts = ws_at<uint32_t>(ws, p.off_counts);
    a.bitems = ws_at<uint4>(ws, p.off_bqueue);
    a.boff = ws_at<uint32_t>(ws, p.off_bqoff);
    a.chk = ws_at<float4>(ws, p.off_chk);
    a.chklast = ws_at<int32_t>(ws, p.off_chklast);
    a.bmask = ws_at<uint8_t>(ws, p.off_bmask);
    a.g2z = ws_at<float4>(ws, p.off_grad2d);
    a.l1 = L1Fuse{nullptr, nullptr, nullptr, nullptr, 0.0};
    a.l1part = ws_at<double>(ws, p.off_l1part);
    a.lc = (uint32_t)p.split_len;
    a.chk_cap = (uint32_t)p.chk_cap;
    a.stats = stats;
    a.n_items = p.n_views * p.tiles_per_view;
    a.T = p.tiles_per_view;
    a.tiles_x = p.tiles_x;
    a.W = p.width;
    a.H = p.height;
    a.persistent = p.s.persistent;
    a.roi_y0 = p.s.roi_y0;
    a.amin = (float)p.s.alpha_min;
    a.amax = (float)p.s.alpha_max;
    a.tmin = (float)p.s.t_min;
    a.lamin2 = (float)log2(p.s.alpha_min);
    a.bg0 = (float)p.s.bg[0];
    a.bg1 = (float)p.s.bg[1];
    a.bg2 = (float)p.s.bg[2];
    return a;
}

int persistent_grid(int n_items, int wg_per_cu) {
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        ncu = 256;
    int g = ncu * wg_per_cu;
    return g < n_items ? g : n_items;
}

template <int TW, int TH, int NB>
int fwd_impl(const splat_plan &p, void *ws, float *img, float *T, int32_t *last, unsigned long long *stats,
             hipStream_t st, const L1Fuse *l1) {
    RenderArgs a = make_args(p, ws, stats);
    if (l1) a.l1 = *l1;
    if (a.n_items == 0) return 0;
    int rc = 0;
    const bool joined = p.s.split_fwd && !stats;  // the instrumented variant walks every list in order
    if (joined) {
        // chunks 1.. of the split lists on their own (about equal work items: a static grid)
        int g1 = persistent_grid((int)(p.chk_cap < INT32_MAX ? p.chk_cap : INT32_MAX), 32);
        hipLaunchKernelGGL((render_fwd_kernel<TW, TH, false, 1, NB>), dim3(g1), dim3(64), 0, st, a, img, T, last);
        if ((rc = launch_status("render_fwd_chunks"))) return rc;
    }
    int grid = a.n_items;
    if (a.persistent) {
        hipLaunchKernelGGL(reset_work_kernel, dim3(1), dim3(1), 0, st, a.work);
        if ((rc = launch_status("reset_work"))) return rc;
        grid = persistent_grid(a.n_items, 32);
    }
    if (stats)
        hipLaunchKernelGGL((render_fwd_kernel<TW, TH, true, 0, NB>), dim3(grid), dim3(64), 0, st, a, img, T, last);
    else if (joined)
        hipLaunchKernelGGL((render_fwd_kernel<TW, TH, false, 2, NB>), dim3(grid), dim3(64), 0, st, a, img, T, last);
    else
        hipLaunchKernelGGL((render_fwd_kernel<TW, TH, false, 0, NB>), dim3(grid), dim3(64), 0, st, a, img, T, last);
    if ((rc = launch_status("render_fwd"))) return rc;
    if (a.l1.target && a.l1.loss) {
        const int ng = (a.n_items + kL1Span - 1) / kL1Span;
        double *gsum = a.l1part + a.n_items;
        hipLaunchKernelGGL(l1_sum_kernel, dim3(ng), dim3(256), 0, st, a.l1part, a.n_items, gsum, 0.0, nullptr);
        if ((rc = launch_status("render_fwd_l1_groups"))) return rc;
        hipLaunchKernelGGL(l1_sum_kernel, dim3(1), dim3(256), 0, st, gsum, ng, nullptr, a.l1.inv_n, a.l1.loss);
        rc = launch_status("render_fwd_l1_total");
    }
    return rc;
}

template <int TW, int TH, int NB>
int bwd_impl(const splat_plan &p, void *ws, const float *dimg, const float *T, const int32_t *last,
             unsigned long long *stats, hipStream_t st) {
    RenderArgs a = make_args(p, ws, stats);
    float *g2 = ws_at<float>(ws, p.off_grad2d);  // cleared by the forward
    int rc = 0;
    const int nT = a.n_items;
    if (nT == 0) return rc;
    a.n_items = (int)(p.bq_cap < INT32_MAX ? p.bq_cap : INT32_MAX);  // bound of the device item count
    int grid = nT;
    if (a.persistent) {
        hipLaunchKernelGGL(reset_work_kernel, dim3(1), dim3(1), 0, st, a.work);
        if ((rc = launch_status("reset_work"))) return rc;
        grid = persistent_grid(nT, 32);
    }
    if (stats)
        hipLaunchKernelGGL((render_bwd_kernel<TW, TH, true, NB>), dim3(grid), dim3(64), 0, st, a, dimg, T, last, g2);
    else
        hipLaunchKernelGGL((render_bwd_kernel<TW, TH, false, NB>), dim3(grid), dim3(64), 0, st, a, dimg, T, last, g2);
    return launch_status("render_bwd");
}

// Gaussians staged per LDS batch: the settings' value, at most the split length (chunk starts
// are batch starts); results do not depend on it
int batch_of(const splat_plan &p) { return p.s.batch < p.split_len ? p.s.batch : p.split_len; }

template <int TW, int TH>
int fwd_tile(const splat_plan &p, void *ws, float *img, float *T, int32_t *last, unsigned long long *s,
             hipStream_t st, const L1Fuse *l1) {
    switch (batch_of(p)) {
        case 32: return fwd_impl<TW, TH, 32>(p, ws, img, T, last, s, st, l1);
        case 64: return fwd_impl<TW, TH, 64>(p, ws, img, T, last, s, st, l1);
        case 128: return fwd_impl<TW, TH, 128>(p, ws, img, T, last, s, st, l1);
        case 256: return fwd_impl<TW, TH, 256>(p, ws, img, T, last, s, st, l1);
    }
    set_error("render_fwd: unsupported batch %d", p.s.batch);
    return SPLAT_EUNSUPPORTED;
}

template <int TW, int TH>
int bwd_tile(const splat_plan &p, void *ws, const float *dimg, const float *T, const int32_t *last,
             unsigned long long *s, hipStream_t st) {
    switch (batch_of(p)) {
        case 32: return bwd_impl<TW, TH, 32>(p, ws, dimg, T, last, s, st);
        case 64: return bwd_impl<TW, TH, 64>(p, ws, dimg, T, last, s, st);
        case 128: return bwd_impl<TW, TH, 128>(p, ws, dimg, T, last, s, st);
        case 256: return bwd_impl<TW, TH, 256>(p, ws, dimg, T, last, s, st);
    }
    set_error("render_bwd: unsupported batch %d", p.s.batch);
    return SPLAT_EUNSUPPORTED;
}

}  // namespace

int launch_render_fwd(const splat_plan &p, void *ws, float *img, float *T, int32_t *last, uint64_t *stats,
                      hipStream_t st, const L1Fuse *l1) {
    int tw = p.s.tile_w, th = p.s.tile_h;
    auto *s = reinterpret_cast<unsigned long long *>(stats);
    if (tw == 16 && th == 16) return fwd_tile<16, 16>(p, ws, img, T, last, s, st, l1);
    if (tw == 8 && th == 8) return fwd_tile<8, 8>(p, ws, img, T, last, s, st, l1);
    if (tw == 16 && th == 32) return fwd_tile<16, 32>(p, ws, img, T, last, s, st, l1);
    if (tw == 32 && th == 16) return fwd_tile<32, 16>(p, ws, img, T, last, s, st, l1);
    set_error("render_fwd: unsupported tile %dx%d", tw, th);
    return SPLAT_EUNSUPPORTED;
}

int launch_render_bwd(const splat_plan &p, void *ws, const float *dimg, const float *T, const int32_t *last,
                      uint64_t *stats, hipStream_t st) {
    int tw = p.s.tile_w, th = p.s.tile_h;
    auto *s = reinterpret_cast<unsigned long long *>(stats);
    if (tw == 16 && th == 16) return bwd_tile<16, 16>(p, ws, dimg, T, last, s, st);
    if (tw == 8 && th == 8) return bwd_tile<8, 8>(p, ws, dimg, T, last, s, st);
    if (tw == 16 && th == 32) return bwd_tile<16, 32>(p, ws, dimg, T, last, s, st);
    if (tw == 32 && th == 16) return bwd_tile<32, 16>(p, ws, dimg, T, last, s, st);
    set_error("render_bwd: unsupported tile %dx%d", tw, th);
    return SPLAT_EUNSUPPORTED;
}

}  // namespace splat
