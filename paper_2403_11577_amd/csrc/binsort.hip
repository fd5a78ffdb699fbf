// binsort.hip -- tile binning: scans, instance emission, stable LSD radix sorts,
// per-(view, tile) ranges and the cost-ordered work queue.
//
// Every (slot, covered tile) pair becomes one instance with value = slot, and every
// tile list ends up in (depth32, Gaussian id) order.  Two ways:
//  - slot-first (the default where a slot's payload fits 64 bits): the slots, which
//    the projection numbers in (view, Gaussian id) order, are sorted by
//    bits(depth32) - bits(near_z) carrying (slot, first tile, rect size); their
//    instances are emitted in that order with key view * T + tile and sorted on
//    the tile bits.  The depth passes then move one element per visible pair rather
//    than per (pair, tile), and the instance passes 32-bit keys.
//  - one 64-bit key per instance, ((view * T + tile) << depth_bits) | (bits(depth32)
//    - bits(near_z)), emitted in (view, Gaussian, tile row-major) order.
// All sorts are stable, so ties on depth are broken by the Gaussian index.
//
// Radix sort: reduce-then-scan per kRadixBits-bit digit with a fixed number of
// partitions (the key count lives on the device, so the grid never depends on
// it); the reduce counts digits with per-wave LDS histograms; inside a partition
// keys are ranked per wave with wave64 ballot peer matching, which keeps the
// order stable without any inter-workgroup waiting, and leave through an LDS
// reorder so that the scattered writes coalesce.
#include "common.hpp"

namespace splat {
namespace {

constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_T * SCAN_ITEMS;  // 2048

__device__ inline uint32_t load_n(const uint32_t *n_dev, int64_t n_cap) {
    if (!n_dev) return (uint32_t)n_cap;
    uint32_t n = *n_dev;
    return n < (uint64_t)n_cap ? n : (uint32_t)n_cap;
}

// inclusive wave scan
// inclusive scan over the wave with DPP (row shifts, then row broadcasts)
template <int CTRL, int ROWS, bool BC>
__device__ inline uint32_t dpp_add(uint32_t x) {
    return x + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xF, BC);
}

// inclusive prefix maximum over the wave, same pattern (lanes without a source see 0)
template <int CTRL, int ROWS, bool BC>
__device__ inline uint32_t dpp_max(uint32_t x) {
    return max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xF, BC));
}

__device__ inline uint32_t wave_incl_max(uint32_t x) {
    x = dpp_max<0x111, 0xF, true>(x);
    x = dpp_max<0x112, 0xF, true>(x);
    x = dpp_max<0x114, 0xF, true>(x);
    x = dpp_max<0x118, 0xF, true>(x);
    x = dpp_max<0x142, 0xA, false>(x);
    x = dpp_max<0x143, 0xC, false>(x);
    return x;
}

__device__ inline uint32_t wave_incl_scan(uint32_t x) {
    x = dpp_add<0x111, 0xF, true>(x);  // row_shr:1
    x = dpp_add<0x112, 0xF, true>(x);  // row_shr:2
    x = dpp_add<0x114, 0xF, true>(x);  // row_shr:4
    x = dpp_add<0x118, 0xF, true>(x);  // row_shr:8
    x = dpp_add<0x142, 0xA, false>(x);  // row_bcast:15 into rows 1, 3
    x = dpp_add<0x143, 0xC, false>(x);  // row_bcast:31 into rows 2, 3
    return x;
}

// exclusive block scan over 256 threads; returns the block total through *tot
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *lds, uint32_t *tot) {
    uint32_t inc = wave_incl_scan(v);
    int w = threadIdx.x >> 6;
    if (__lane_id() == 63) lds[w] = inc;
    __syncthreads();
    uint32_t base = 0, total = 0;
    int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) {
        uint32_t c = lds[i];
        if (i < w) base += c;
        total += c;
    }
    __syncthreads();
    *tot = total;
    return base + inc - v;
}

__global__ __launch_bounds__(SCAN_T) void scan_reduce_kernel(const uint32_t *in, const uint32_t *n_dev,
                                                            int64_t n_cap, uint32_t *partials) {
    __shared__ uint32_t lds[4];
    uint32_t n = load_n(n_dev, n_cap);
    uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    if (base >= n) {
        if (threadIdx.x == 0) partials[blockIdx.x] = 0;
        return;
    }
    uint32_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        uint64_t i = base + (uint64_t)k * SCAN_T + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_excl_scan(s, lds, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// single workgroup of 1024 threads: exclusive scan of the partials in place
__global__ __launch_bounds__(1024) void scan_partials_kernel(uint32_t *partials, int nparts, uint32_t *out,
                                                            const uint32_t *n_dev, int64_t n_cap,
                                                            uint32_t *total_dst) {
    __shared__ uint32_t lds[16];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nparts; base += 1024) {
        int i = base + threadIdx.x;
        uint32_t v = i < nparts ? partials[i] : 0u;
        uint32_t inc = wave_incl_scan(v);
        int w = threadIdx.x >> 6;
        if (__lane_id() == 63) lds[w] = inc;
        __syncthreads();
        uint32_t wb = 0, tot = 0;
        for (int k = 0; k < 16; ++k) {
            uint32_t c = lds[k];
            if (k < w) wb += c;
            tot += c;
        }
        uint32_t c0 = carry;
        if (i < nparts) partials[i] = c0 + wb + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) carry = c0 + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        uint32_t n = load_n(n_dev, n_cap);
        out[n] = carry;
        if (total_dst) *total_dst = carry;
    }
}

// SELF: the partials are the blocks' plain sums (no scan_partials_kernel): each workgroup adds
// up those before its own (at most 4 SCAN_T of them), and the one holding the last element
// writes the total to out[n] and *total_dst.  Otherwise partials[b] is already block b's
// exclusive prefix.
template <bool SELF>
__global__ __launch_bounds__(SCAN_T) void scan_down_kernel(const uint32_t *in, uint32_t *out, const uint32_t *n_dev,
                                                          int64_t n_cap, const uint32_t *partials,
                                                          uint32_t *total_dst) {
    __shared__ uint32_t lds[4], lds2[4];
    uint32_t n = load_n(n_dev, n_cap);
    uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    if (SELF && n == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            out[0] = 0u;
            if (total_dst) *total_dst = 0u;
        }
        return;
    }
    if (base >= n) return;
    uint32_t pre;
    if constexpr (SELF) {
        uint32_t acc = 0;
        for (int i = threadIdx.x; i < (int)blockIdx.x; i += SCAN_T) acc += partials[i];
        uint32_t inc = wave_incl_scan(acc);
        if (__lane_id() == 63) lds2[threadIdx.x >> 6] = inc;
        __syncthreads();
        pre = ((lds2[0] + lds2[1]) + lds2[2]) + lds2[3];
    } else {
        pre = partials[blockIdx.x];
    }
    // each thread owns SCAN_ITEMS consecutive elements
    uint64_t t0 = base + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        uint64_t i = t0 + k;
        v[k] = (i < n) ? in[i] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(s, lds, &tot) + pre;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        uint64_t i = t0 + k;
        if (i < n) out[i] = ex;
        ex += v[k];
    }
    if (SELF && threadIdx.x == 0 && (uint64_t)n <= base + SCAN_TILE) {  // the block holding element n - 1
        out[n] = pre + tot;
        if (total_dst) *total_dst = pre + tot;
    }
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// -------------------------------------------------------------------------------------
// emission
// -------------------------------------------------------------------------------------
// Instance count.  On overflow the count is the end of the longest prefix of
// slots whose instances all fit, so every key below the count is written.
__global__ void inst_finish_kernel(const uint32_t *offs, int64_t inst_cap, uint32_t *counts, uint32_t *status) {
    if (threadIdx.x != 0) return;
    uint32_t ns = counts[CNT_SLOTS];
    uint32_t tot = offs[ns];
    uint32_t cap = (uint32_t)inst_cap;
    if (tot <= cap) {
        counts[CNT_INST] = tot;
        return;
    }
    uint32_t lo = 0, hi = ns;  // largest k with offs[k] <= cap (offs[0] = 0)
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (offs[mid] <= cap) lo = mid; else hi = mid - 1;
    }
    counts[CNT_INST] = offs[lo];
    atomicOr(status, SPLAT_ST_CAPACITY);
}

__global__ __launch_bounds__(256) void emit_kernel(const uint32_t *__restrict__ counts,
                                                  const uint32_t *__restrict__ offs, const Rect16 *__restrict__ rect,
                                                  const uint32_t *__restrict__ dkeys, const int2 *__restrict__ meta,
                                                  int tiles_x, int T, int depth_bits, uint64_t *__restrict__ keys,
                                                  uint32_t *__restrict__ vals) {
    uint32_t ns = counts[CNT_SLOTS];
    uint32_t ni = counts[CNT_INST];  // <= capacity; only slots wholly below it emit
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < ns;
         s += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t o = offs[s];
        Rect16 r = rect[s];
        uint32_t nt = (uint32_t)(r.x1 - r.x0 + 1) * (uint32_t)(r.y1 - r.y0 + 1);
        if ((uint64_t)o + nt > (uint64_t)ni) continue;
        uint64_t dkey = (uint64_t)dkeys[s];  // bits(depth32) - bits(near_z), written by the projection
        uint64_t vbase = (uint64_t)meta[s].y * (uint64_t)T;
        for (int ty = r.y0; ty <= r.y1; ++ty)
            for (int tx = r.x0; tx <= r.x1; ++tx) {
                uint64_t tile = vbase + (uint64_t)(ty * tiles_x + tx);
                keys[o] = (tile << depth_bits) | dkey;
                vals[o] = (uint32_t)s;
                ++o;
            }
    }
}

// Slot-first binning.  A slot's payload (written by the projection) packs the slot id, its first
// tile (view * T + tile) and its rect's width and height in tiles minus one, at bit offsets 0,
// b0, b0 + tb, b0 + tb + b1; after the depth sort of the slots, pay[s] is the payload of the s-th
// nearest slot.
struct PayBits {
    int b0, tb, b1;
};

__device__ inline uint64_t field(uint64_t p, int at, int width) {
    if (width == 0 || at >= 64) return 0ull;
    const uint64_t v = p >> at;
    return width >= 64 ? v : v & ((1ull << width) - 1ull);
}

// tiles of every slot in depth order (scanned afterwards to the instance offsets)
__device__ inline uint32_t tiles_of(uint64_t p, PayBits pb) {
    return ((uint32_t)field(p, pb.b0 + pb.tb, pb.b1) + 1u) * ((uint32_t)field(p, pb.b0 + pb.tb + pb.b1, 64) + 1u);
}

// Instances of every run of 64 consecutive slots in depth order (the runs the emission's waves
// take), to be scanned to run offsets; counts[CNT_RUNS] = the number of runs.
__global__ __launch_bounds__(256) void run_tiles_kernel(uint32_t *__restrict__ counts,
                                                       const uint64_t *__restrict__ pay, PayBits pb,
                                                       uint32_t *__restrict__ rsum) {
    const uint32_t ns = counts[CNT_SLOTS];
    const uint32_t nr = (ns + 63u) / 64u;
    if (blockIdx.x == 0 && threadIdx.x == 0) counts[CNT_RUNS] = nr;
    const int lane = __lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * 4;
    // two runs per step, both payloads loaded before either is used
    for (uint64_t q = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); q < nr; q += 2 * stride) {
        const uint64_t q2 = q + stride;
        const uint64_t s = q * 64 + lane, s2 = q2 * 64 + lane;
        const uint64_t p = s < ns ? pay[s] : 0ull, p2 = s2 < ns ? pay[s2] : 0ull;
        const uint32_t tot = wave_incl_scan(s < ns ? tiles_of(p, pb) : 0u);
        const uint32_t tot2 = wave_incl_scan(s2 < ns ? tiles_of(p2, pb) : 0u);
        if (lane == 63) {
            rsum[q] = tot;
            if (q2 < nr) rsum[q2] = tot2;
        }
    }
}

// Instance count from the scanned run offsets (roff[nr] = the total).  On overflow the count is
// the end of the longest prefix of slots whose instances all fit: the run in which the capacity
// is crossed is found by bisection, then the one wave scans that run's tile counts.
__global__ __launch_bounds__(64) void run_finish_kernel(const uint32_t *roff, const uint64_t *pay, PayBits pb,
                                                       int64_t inst_cap, uint32_t *counts, uint32_t *status) {
    const uint32_t nr = counts[CNT_RUNS], ns = counts[CNT_SLOTS];
    const uint32_t tot = roff[nr];
    const uint32_t cap = (uint32_t)inst_cap;
    if (tot <= cap) {
        if (threadIdx.x == 0) counts[CNT_INST] = tot;
        return;
    }
    uint32_t lo = 0, hi = nr;  // largest run k with roff[k] <= cap (roff[0] = 0 and roff[nr] > cap)
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (roff[mid] <= cap) lo = mid; else hi = mid - 1;
    }
    const uint64_t s = (uint64_t)lo * 64 + threadIdx.x;
    // where each slot of the run ends: nondecreasing, so the slots that fit are a prefix
    const uint32_t end = roff[lo] + wave_incl_scan(s < ns ? tiles_of(pay[s], pb) : 0u);
    const int nfit = __popcll(__ballot(end <= cap));
    const uint32_t cnt = nfit ? (uint32_t)__shfl((int)end, nfit - 1, kWave) : roff[lo];
    if (threadIdx.x == 0) {
        counts[CNT_INST] = cnt;
        atomicOr(status, SPLAT_ST_CAPACITY);
    }
}

// one instance per (slot, covered tile) in depth order: key view * T + tile (u32), value slot.
// A wave takes a run of 64 consecutive slots; their instances form one run of the output from
// the run's offset, which the lanes write in turn, 64 positions at a time (coalesced stores,
// and no lane waits for a large slot of another): run position q belongs to the last slot with
// instances that starts at or before q.  Per window of 64 positions, each such slot that starts
// inside it marks its start, and a prefix maximum over the wave (carried from the window
// before) names every position's slot.
__global__ __launch_bounds__(256) void emit_sorted_kernel(const uint32_t *__restrict__ counts,
                                                         const uint32_t *__restrict__ roff,
                                                         const uint64_t *__restrict__ pay, PayBits pb, int tiles_x,
                                                         uint32_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    __shared__ uint32_t sbeg[4][64];  // per wave: run position of each slot's first instance
    __shared__ uint32_t smark[4][64];  // per wave and window: 1 + the slot starting at each position
    __shared__ uint4 sinf[4][64];     // per wave: the slots' first tile, rect width, 1 / width, slot id
    const uint32_t ns = counts[CNT_SLOTS];
    const uint32_t ni = counts[CNT_INST];  // <= capacity; only slots wholly below it emit
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    for (uint64_t s0 = ((uint64_t)blockIdx.x * 4 + w) * 64; s0 < ns; s0 += (uint64_t)gridDim.x * 256) {
        const uint64_t s = s0 + lane;
        const bool valid = s < ns;
        const uint64_t p = valid ? pay[s] : 0ull;
        const uint32_t run0 = roff[s0 / 64];
        uint32_t nt = valid ? tiles_of(p, pb) : 0u;
        const uint32_t incl = wave_incl_scan(nt);
        const uint32_t rel = valid ? incl - nt : 0xFFFFFFFFu;
        if ((uint64_t)run0 + incl > (uint64_t)ni) nt = 0u;  // and so does every later slot
        // the run ends where the last slot with instances ends
        uint32_t end = nt ? rel + nt : 0u;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) end = max(end, (uint32_t)__shfl_xor((int)end, d, kWave));
        sbeg[w][lane] = rel;
        const uint32_t wl = (uint32_t)field(p, pb.b0 + pb.tb, pb.b1) + 1u;
        sinf[w][lane] = make_uint4((uint32_t)field(p, pb.b0, pb.tb), wl, __float_as_uint(__builtin_amdgcn_rcpf((float)wl)),
                                   (uint32_t)field(p, 0, pb.b0));
        __builtin_amdgcn_wave_barrier();  // one wave: its LDS writes complete before its reads
        uint32_t carry = 0;  // 1 + the slot of the position before the window
        for (uint32_t q0 = 0; q0 < end; q0 += 64) {
            smark[w][lane] = 0u;
            __builtin_amdgcn_wave_barrier();
            if (nt && rel - q0 < 64u) smark[w][rel - q0] = (uint32_t)lane + 1u;  // unsigned: earlier starts fail
            __builtin_amdgcn_wave_barrier();
            const uint32_t own = max(wave_incl_max(smark[w][lane]), carry);
            carry = (uint32_t)__builtin_amdgcn_readlane((int)own, 63);
            __builtin_amdgcn_wave_barrier();  // every mark read before the next window clears them
            const uint32_t q = q0 + lane;
            if (q >= end) continue;
            const int j = (int)own - 1;
            const uint4 fj = sinf[w][j];
            const uint32_t wj = fj.y;
            const uint32_t r = q - sbeg[w][j];
            uint32_t dy = (uint32_t)((float)r * __uint_as_float(fj.z));
            if (dy * wj > r) --dy;           // the float estimate is within one of r / wj
            if ((dy + 1u) * wj <= r) ++dy;
            const uint32_t dx = r - dy * wj;
            keys[run0 + q] = fj.x + dy * (uint32_t)tiles_x + dx;
            vals[run0 + q] = fj.w;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// -------------------------------------------------------------------------------------
// radix sort
// -------------------------------------------------------------------------------------
constexpr int RS_T = 256;  // threads per partition workgroup = keys per round

__device__ inline void chunk_of(uint32_t n, int nparts, int part, uint32_t &b, uint32_t &e) {
    uint32_t per = (n + nparts - 1) / nparts;
    per = (per + RS_T - 1) / RS_T * RS_T;
    uint64_t bb = (uint64_t)part * per;
    uint64_t ee = bb + per;
    b = (uint32_t)(bb < n ? bb : n);
    e = (uint32_t)(ee < n ? ee : n);
}

// lanes of the wave holding the same digit as this lane
__device__ inline uint64_t match_digit(uint32_t d, bool act) {
    uint64_t peers = __ballot(act);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        uint64_t m = __ballot(act && ((d >> b) & 1u));
        peers &= ((d >> b) & 1u) ? m : ~m;
    }
    return act ? peers : 0ull;
}

constexpr uint32_t kDigitMask = (uint32_t)kRadixDigits - 1u;
constexpr int RS_DPT = kRadixDigits / RS_T;  // digits owned per thread
static_assert(kRadixDigits % RS_T == 0, "digits must be a multiple of the workgroup size");

constexpr int RS_UKPT = 16;  // keys per thread per upsweep round

template <typename K>
__global__ __launch_bounds__(RS_T) void radix_upsweep_kernel(const K *keys, const uint32_t *counts, int cnt_idx,
                                                            int shift, int nparts, uint32_t *hist) {
    // four LDS histograms per wave, lane l counting into copy l mod 4 (rows one bank apart): equal
    // digits within a wave, common in the high digits of coherent keys, serialise four times less
    constexpr int NH = 4 * (RS_T / 64);
    __shared__ uint32_t h[NH][kRadixDigits + 1];
    const int w = 4 * (threadIdx.x >> 6) + (threadIdx.x & 3);
    for (int q = 0; q < RS_DPT; ++q)
        for (int ww = 0; ww < NH; ++ww) h[ww][q * RS_T + threadIdx.x] = 0;
    __syncthreads();
    uint32_t n = counts[cnt_idx];
    uint32_t b, e;
    chunk_of(n, nparts, blockIdx.x, b, e);
    // RS_UKPT independent coalesced loads per thread are in flight before their counts
    for (uint32_t base = b; base < e; base += RS_T * RS_UKPT) {
        K kk[RS_UKPT];
#pragma unroll
        for (int k = 0; k < RS_UKPT; ++k) {
            const uint32_t i = base + k * RS_T + threadIdx.x;
            kk[k] = i < e ? keys[i] : (K)0;
        }
#pragma unroll
        for (int k = 0; k < RS_UKPT; ++k)
            if (base + k * RS_T + threadIdx.x < e) atomicAdd(&h[w][(uint32_t)(kk[k] >> shift) & kDigitMask], 1u);
    }
    __syncthreads();
    for (int q = 0; q < RS_DPT; ++q) {
        int d = q * RS_T + threadIdx.x;
        uint32_t c = 0;
        for (int ww = 0; ww < NH; ++ww) c += h[ww][d];
        hist[(size_t)d * nparts + blockIdx.x] = c;
    }
}

// exclusive scan over the workgroup (RS_T threads, in thread order); *total gets the sum
__device__ inline uint32_t block_exscan(uint32_t x, uint32_t *wsum, uint32_t *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = wave_incl_scan(x);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int q = 0; q < RS_T / 64; ++q) {
        uint32_t c = wsum[q];
        if (q < w) pre += c;
        tot += c;
    }
    *total = tot;
    return pre + incl - x;
}

// Downsweep of one pass.  A workgroup walks its chunk in tiles of RS_TILE keys;
// wave w takes the w-th quarter of the tile (RS_KPT loads of 64 consecutive keys,
// so position order inside the tile is (wave, round, lane)), and the next tile is
// loaded while this one is ranked.  Every wave ranks its keys stably on its own
// with per-wave digit counters in LDS (no workgroup barrier per round); one scan
// over (digit, wave) then places the tile in digit order in LDS, and the tile
// leaves in that order: the keys of one digit go out as one contiguous run, so
// the global stores coalesce.  Thread t owns digits [RS_DPT t, RS_DPT (t + 1)).
#ifndef SPLAT_RADIX_KPT
#define SPLAT_RADIX_KPT 16
#endif
constexpr int RS_KPT = SPLAT_RADIX_KPT;  // keys per thread per tile
constexpr int RS_WTILE = 64 * RS_KPT;
constexpr int RS_TILE = RS_T * RS_KPT;

template <typename K, typename V>
__device__ inline void rs_load(const K *kin, const V *vin, uint32_t base, uint32_t e, int w, int lane,
                               K (&key)[RS_KPT], V (&val)[RS_KPT]) {
#pragma unroll
    for (int k = 0; k < RS_KPT; ++k) {
        uint32_t i = base + w * RS_WTILE + k * 64 + lane;
        bool act = i < e;
        key[k] = act ? kin[i] : (K)0;
        val[k] = act ? vin[i] : (V)0;
    }
}

// KI keys in, KO keys out: a pass after which every remaining digit lies at or above bit
// out_shift can write the keys shifted down by out_shift as 32-bit words (the later passes
// then move 4 bytes less per key, read and written).  V: the values carried along; the key
// count is counts[cnt_idx].  A null kout moves the values only (a last pass whose keys nothing
// reads).
template <typename KI, typename KO, typename V>
__global__ __launch_bounds__(RS_T) void radix_downsweep_kernel(const KI *kin, const V *vin, KO *kout, V *vout,
                                                              const uint32_t *counts, int cnt_idx, int shift,
                                                              int out_shift, int nparts, const uint32_t *hoff) {
    __shared__ KI sk[RS_TILE];
    __shared__ V sv[RS_TILE];
    __shared__ uint32_t wc[RS_T / 64][kRadixDigits];  // per-wave running counts, then per-wave bases
    __shared__ uint32_t tstart[kRadixDigits];         // first LDS position of each digit in the tile
    __shared__ uint32_t gstart[kRadixDigits];         // global position of the tile's first key of each digit
    __shared__ uint32_t wsum[2][RS_T / 64];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    uint32_t gnext[RS_DPT];
    for (int q = 0; q < RS_DPT; ++q) {
        int d = RS_DPT * t + q;
        gnext[q] = hoff[(size_t)d * nparts + blockIdx.x];
        for (int ww = 0; ww < RS_T / 64; ++ww) wc[ww][d] = 0;
    }
    __syncthreads();
    uint32_t n = counts[cnt_idx];
    uint32_t b, e;
    chunk_of(n, nparts, blockIdx.x, b, e);
    KI key[RS_KPT];
    V val[RS_KPT];
    if (b < e) rs_load(kin, vin, b, e, w, lane, key, val);
    int parity = 0;
    for (uint32_t base = b; base < e; base += RS_TILE) {
        uint32_t tn = min((uint32_t)RS_TILE, e - base);
        KI nkey[RS_KPT];
        V nval[RS_KPT];
        uint32_t rank[RS_KPT];
        if (base + RS_TILE < e) rs_load(kin, vin, base + RS_TILE, e, w, lane, nkey, nval);
        // stable rank inside the wave: the peers' leader bumps the wave's counter after all
        // lanes read it (LDS operations of one wave complete in issue order)
#pragma unroll
        for (int k = 0; k < RS_KPT; ++k) {
            bool act = (uint32_t)(w * RS_WTILE + k * 64 + lane) < tn;
            uint32_t d = (uint32_t)(key[k] >> shift) & kDigitMask;
            uint64_t peers = match_digit(d, act);
            uint32_t r = rank_in(peers);
            uint32_t bse = act ? wc[w][d] : 0u;
            if (act && r == 0) wc[w][d] = bse + (uint32_t)__popcll(peers);
            rank[k] = bse + r;
        }
        __syncthreads();
        // digit-major, wave-minor exclusive scan of the counts
        uint32_t c[RS_DPT][RS_T / 64], seen[RS_DPT], mine = 0;
        for (int q = 0; q < RS_DPT; ++q) {
            seen[q] = 0;
            for (int ww = 0; ww < RS_T / 64; ++ww) {
                c[q][ww] = wc[ww][RS_DPT * t + q];
                seen[q] += c[q][ww];
            }
            mine += seen[q];
        }
        uint32_t tot;
        uint32_t start = block_exscan(mine, wsum[parity], &tot);
        for (int q = 0; q < RS_DPT; ++q) {
            int d = RS_DPT * t + q;
            tstart[d] = start;
            gstart[d] = gnext[q];
            gnext[q] += seen[q];
            uint32_t run = start;
            for (int ww = 0; ww < RS_T / 64; ++ww) {
                wc[ww][d] = run;
                run += c[q][ww];
            }
            start += seen[q];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RS_KPT; ++k) {
            if ((uint32_t)(w * RS_WTILE + k * 64 + lane) < tn) {
                uint32_t d = (uint32_t)(key[k] >> shift) & kDigitMask;
                uint32_t pos = wc[w][d] + rank[k];
                sk[pos] = key[k];
                sv[pos] = val[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RS_KPT; ++k) {
            uint32_t i = k * RS_T + t;
            if (i < tn) {
                KI kk = sk[i];
                uint32_t d = (uint32_t)(kk >> shift) & kDigitMask;
                uint32_t dst = gstart[d] + (i - tstart[d]);
                if (dst < n) {  // always true when both sweeps saw the same keys
                    if (kout) kout[dst] = (KO)(kk >> out_shift);
                    vout[dst] = sv[i];
                }
            }
        }
        for (int q = 0; q < RS_DPT; ++q)
            for (int ww = 0; ww < RS_T / 64; ++ww) wc[ww][RS_DPT * t + q] = 0;
#pragma unroll
        for (int k = 0; k < RS_KPT; ++k) {
            key[k] = nkey[k];
            val[k] = nval[k];
        }
        parity ^= 1;
        __syncthreads();
    }
}

// -------------------------------------------------------------------------------------
// tile ranges and the work queue
// -------------------------------------------------------------------------------------
// Tile t's instances are [ranges[t].x, ranges[t].y) of the sorted keys.  A thread takes 4
// consecutive keys and the one on each side (all six loads issued before any store), and
// writes the bounds of the runs that start or end among its four.
template <typename K>
__global__ __launch_bounds__(256) void ranges_kernel(const K *__restrict__ keys, const uint32_t *counts,
                                                    int depth_bits, uint64_t n_tiles, uint2 *__restrict__ ranges,
                                                    uint32_t *qh) {
    if (blockIdx.x == 0 && threadIdx.x < 66) qh[threadIdx.x] = 0u;  // the work queue's counters
    const uint32_t n = counts[CNT_INST];
    const uint64_t ng = ((uint64_t)n + 3) / 4;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t i0 = 4 * (int64_t)g;
        uint64_t t[6];  // tiles of keys i0 - 1 .. i0 + 4; all ones outside [0, n)
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int64_t i = i0 - 1 + k;
            t[k] = (i >= 0 && i < (int64_t)n) ? (uint64_t)(keys[i] >> depth_bits) : ~0ull;
        }
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            const uint64_t tk = t[k];
            if (tk >= n_tiles) continue;  // past the end; cannot happen for emitted keys
            const uint32_t i = (uint32_t)(i0 + k - 1);
            if (t[k - 1] != tk) ranges[tk].x = i;
            if (t[k + 1] != tk) ranges[tk].y = i + 1;
        }
    }
}

// The same for u32 keys on a 16-byte aligned buffer: lane l of a wave loads its four keys with
// one vector load; the key before them is lane l - 1's last and the key after them lane l + 1's
// first (lanes 0 and 63 load theirs).  The walk goes by whole waves, so every lane takes part
// in the exchanges.
__global__ __launch_bounds__(256) void ranges_vec_kernel(const uint32_t *__restrict__ keys, const uint32_t *counts,
                                                        int shift, uint32_t n_tiles, uint2 *__restrict__ ranges,
                                                        uint32_t *qh) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;  // past either end; never a tile (n_tiles < 2^31)
    if (blockIdx.x == 0 && threadIdx.x < 66) qh[threadIdx.x] = 0u;  // the work queue's counters
    const uint32_t n = counts[CNT_INST];
    const uint64_t ng = ((uint64_t)n + 3) / 4;
    const int lane = __lane_id();
    const uint4 *keys4 = reinterpret_cast<const uint4 *>(keys);
    auto tile_at = [&](int64_t i) { return (i >= 0 && i < (int64_t)n) ? keys[i] >> shift : kNone; };
    for (uint64_t g0 = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); g0 < ng;
         g0 += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t g = g0 + (uint64_t)lane;
        const int64_t i0 = 4 * (int64_t)g;
        uint32_t t[6];
        if (i0 + 3 < (int64_t)n) {
            const uint4 q = keys4[g];
            t[1] = q.x >> shift; t[2] = q.y >> shift; t[3] = q.z >> shift; t[4] = q.w >> shift;
        } else {
#pragma unroll
            for (int k = 1; k <= 4; ++k) t[k] = tile_at(i0 + k - 1);
        }
        t[0] = (uint32_t)__shfl_up((int)t[4], 1, kWave);
        t[5] = (uint32_t)__shfl_down((int)t[1], 1, kWave);
        if (lane == 0) t[0] = tile_at(i0 - 1);
        if (lane == 63) t[5] = tile_at(i0 + 4);
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            const uint32_t tk = t[k];
            if (tk >= n_tiles) continue;  // past the end; cannot happen for emitted keys
            const uint32_t i = (uint32_t)(i0 + k - 1);
            if (t[k - 1] != tk) ranges[tk].x = i;
            if (t[k + 1] != tk) ranges[tk].y = i + 1;
        }
    }
}

__device__ inline int cost_bucket(uint2 r) {
    uint32_t c = r.y - r.x;  // empty tiles have x = y = 0
    return c == 0 ? 0 : 32 - __clz(c);  // 1..32
}

// qh[66]: [0..32] bucket counts, [33..65] the running counts of the scatter (zeroed by the
// ranges kernel)
__global__ __launch_bounds__(256) void queue_hist_kernel(const uint2 *ranges, int n, uint32_t *qh) {
    __shared__ uint32_t h[33];
    if (threadIdx.x < 33) h[threadIdx.x] = 0;
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        atomicAdd(&h[cost_bucket(ranges[i])], 1u);
    __syncthreads();
    if (threadIdx.x < 33 && h[threadIdx.x]) atomicAdd(&qh[threadIdx.x], h[threadIdx.x]);
}

// Descending buckets: bucket b starts after the items of the buckets above it (each workgroup
// adds those counts up itself); each workgroup reserves one range per bucket with a single
// global atomic on the bucket's running count, then places its items with LDS atomics.
__global__ __launch_bounds__(256) void queue_scatter_kernel(const uint2 *ranges, int n, uint32_t *qh,
                                                           uint32_t *queue) {
    __shared__ uint32_t cnt[33], base[33], start[33];
    if (threadIdx.x < 33) {
        uint32_t acc = 0;
        for (int b = threadIdx.x + 1; b < 33; ++b) acc += qh[b];
        start[threadIdx.x] = acc;
    }
    for (int i0 = blockIdx.x * blockDim.x; i0 < n; i0 += gridDim.x * blockDim.x) {
        if (threadIdx.x < 33) cnt[threadIdx.x] = 0;
        __syncthreads();
        int i = i0 + threadIdx.x;
        int bk = i < n ? cost_bucket(ranges[i]) : 0;
        uint32_t local = i < n ? atomicAdd(&cnt[bk], 1u) : 0u;
        __syncthreads();
        if (threadIdx.x < 33 && cnt[threadIdx.x])
            base[threadIdx.x] = start[threadIdx.x] + atomicAdd(&qh[33 + threadIdx.x], cnt[threadIdx.x]);
        __syncthreads();
        if (i < n) queue[base[bk] + local] = (uint32_t)i;
        __syncthreads();
    }
}

// -------------------------------------------------------------------------------------
// render-adjoint work items
// -------------------------------------------------------------------------------------
// A list of at least Lc = 2^lc_log instances is split into ceil(L / Lc) chunks that the
// adjoint walks in parallel.  The queue is ordered by floor(log2 L), so the split lists are
// exactly its first nsplit positions.  Per split position the chunk count is written for a
// scan; nsplit is written by the one position where the split prefix ends.
__global__ __launch_bounds__(256) void split_count_kernel(const uint2 *ranges, const uint32_t *queue, int n,
                                                         int lc_log, uint32_t *cnt, uint32_t *counts) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        uint2 r = ranges[queue[q]];
        uint32_t L = r.y - r.x;
        bool sp = (L >> lc_log) != 0u;
        cnt[q] = sp ? (uint32_t)(((uint64_t)L + (1u << lc_log) - 1) >> lc_log) : 0u;
        bool sp_next = false;
        if (q + 1 < n) {
            uint2 r2 = ranges[queue[q + 1]];
            sp_next = ((r2.y - r2.x) >> lc_log) != 0u;
        }
        if (sp && !sp_next) counts[CNT_NSPLIT] = (uint32_t)(q + 1);
        if (q == 0 && !sp) counts[CNT_NSPLIT] = 0u;
    }
}

// items: the chunks of the split lists (at their scanned offsets; chunk c of a list whose
// checkpoints start at slot s is (tile, c, s)), then the unsplit tiles (tile, 0, ~0)
__global__ __launch_bounds__(256) void split_items_kernel(const uint2 *ranges, const uint32_t *queue, int n,
                                                         const uint32_t *off, uint32_t *counts, uint4 *items,
                                                         int64_t cap) {
    uint32_t ns = counts[CNT_NSPLIT], nch = counts[CNT_NCHUNK];
    if (blockIdx.x == 0 && threadIdx.x == 0) counts[CNT_BITEMS] = nch + ((uint32_t)n - ns);
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        uint32_t t = queue[q];
        if ((uint32_t)q < ns) {
            uint32_t o = off[q], c1 = off[q + 1];
            for (uint32_t c = 0; o + c < c1 && (int64_t)(o + c) < cap; ++c) items[o + c] = make_uint4(t, c, o, 0u);
        } else {
            uint64_t i = (uint64_t)nch + (uint32_t)q - ns;
            if ((int64_t)i < cap) items[i] = make_uint4(t, 0u, 0xFFFFFFFFu, 0u);
        }
    }
}

}  // namespace

size_t scan_partials(int64_t n_cap) { return (size_t)((n_cap + SCAN_TILE - 1) / SCAN_TILE) + 1; }

int launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return 0;
    int64_t nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)nb), dim3(256), 0, st, p, v, n);
    return launch_status("fill");
}

int launch_scan_u32(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, int64_t n_cap, uint32_t *partials,
                    uint32_t *total_dst, hipStream_t st) {
    int64_t nparts = (n_cap + SCAN_TILE - 1) / SCAN_TILE;
    if (nparts < 1) nparts = 1;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nparts), dim3(SCAN_T), 0, st, in, n_dev, n_cap, partials);
    int rc = launch_status("scan_reduce");
    if (rc) return rc;
    if (nparts <= 4 * SCAN_T) {  // the down-sweep adds up the block sums before each block itself
        hipLaunchKernelGGL(scan_down_kernel<true>, dim3((unsigned)nparts), dim3(SCAN_T), 0, st, in, out, n_dev, n_cap,
                           partials, total_dst);
        return launch_status("scan_down");
    }
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(1024), 0, st, partials, (int)nparts, out, n_dev, n_cap,
                       total_dst);
    rc = launch_status("scan_partials");
    if (rc) return rc;
    hipLaunchKernelGGL(scan_down_kernel<false>, dim3((unsigned)nparts), dim3(SCAN_T), 0, st, in, out, n_dev, n_cap,
                       partials, nullptr);
    return launch_status("scan_down");
}

int launch_radix_sort_keys(uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, const uint32_t *counts, int bit0,
                           int bits, int nparts, uint32_t *hist, uint32_t *partials, hipStream_t st, int *sorted_in_1,
                           int max_shift, int *key_shift) {
    int passes = (bits + kRadixBits - 1) / kRadixBits;
    const int top = bit0 + bits;
    // first pass after which the remaining digits fit a 32-bit word shifted down by S <= max_shift
    int sw = -1, S = 0;
    for (int p = 0; p + 1 < passes && max_shift >= 0; ++p) {
        int s1 = bit0 + kRadixBits * (p + 1);
        if (s1 <= max_shift && top - s1 <= 32) {
            sw = p;
            S = s1;
            break;
        }
    }
    uint64_t *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    int nh = kRadixDigits * nparts;
    int rc = 0;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = bit0 + kRadixBits * ps;
        auto *ki32 = reinterpret_cast<uint32_t *>(ki);
        auto *ko32 = reinterpret_cast<uint32_t *>(ko);
        if (sw >= 0 && ps > sw)
            hipLaunchKernelGGL(radix_upsweep_kernel<uint32_t>, dim3(nparts), dim3(RS_T), 0, st, ki32, counts,
                               (int)CNT_INST, shift - S, nparts, hist);
        else
            hipLaunchKernelGGL(radix_upsweep_kernel<uint64_t>, dim3(nparts), dim3(RS_T), 0, st, ki, counts,
                               (int)CNT_INST, shift, nparts, hist);
        if ((rc = launch_status("radix_upsweep"))) return rc;
        if ((rc = launch_scan_u32(hist, hist, nullptr, nh, partials, nullptr, st))) return rc;
        if (sw < 0 || ps < sw)
            hipLaunchKernelGGL((radix_downsweep_kernel<uint64_t, uint64_t, uint32_t>), dim3(nparts), dim3(RS_T), 0, st, ki,
                               vi, ko, vo, counts, (int)CNT_INST, shift, 0, nparts, hist);
        else if (ps == sw)
            hipLaunchKernelGGL((radix_downsweep_kernel<uint64_t, uint32_t, uint32_t>), dim3(nparts), dim3(RS_T), 0, st, ki,
                               vi, ko32, vo, counts, (int)CNT_INST, shift, S, nparts, hist);
        else
            hipLaunchKernelGGL((radix_downsweep_kernel<uint32_t, uint32_t, uint32_t>), dim3(nparts), dim3(RS_T), 0, st,
                               ki32, vi, ko32, vo, counts, (int)CNT_INST, shift - S, 0, nparts, hist);
        if ((rc = launch_status("radix_downsweep"))) return rc;
        uint64_t *tk = ki; ki = ko; ko = tk;
        uint32_t *tv = vi; vi = vo; vo = tv;
    }
    *sorted_in_1 = passes & 1;
    if (key_shift) *key_shift = sw >= 0 ? S : -1;
    return 0;
}

// Stable LSD sort of counts[cnt_idx] u32 keys on bits [0, bits), carrying V values; the result
// is in the second buffers when *sorted_in_1 (an odd number of passes).
// keys_out = false: the last pass writes the values only (the sorted keys are left unwritten)
template <typename V>
int launch_radix_sort_u32(uint32_t *k0, uint32_t *k1, V *v0, V *v1, const uint32_t *counts, int cnt_idx, int bits,
                          int nparts, uint32_t *hist, uint32_t *partials, hipStream_t st, int *sorted_in_1,
                          bool keys_out = true) {
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    const int nh = kRadixDigits * nparts;
    uint32_t *ki = k0, *ko = k1;
    V *vi = v0, *vo = v1;
    int rc = 0;
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = kRadixBits * ps;
        hipLaunchKernelGGL(radix_upsweep_kernel<uint32_t>, dim3(nparts), dim3(RS_T), 0, st, ki, counts, cnt_idx, shift,
                           nparts, hist);
        if ((rc = launch_status("radix_upsweep"))) return rc;
        if ((rc = launch_scan_u32(hist, hist, nullptr, nh, partials, nullptr, st))) return rc;
        hipLaunchKernelGGL((radix_downsweep_kernel<uint32_t, uint32_t, V>), dim3(nparts), dim3(RS_T), 0, st, ki, vi,
                           keys_out || ps + 1 < passes ? ko : nullptr, vo, counts, cnt_idx, shift, 0, nparts, hist);
        if ((rc = launch_status("radix_downsweep"))) return rc;
        uint32_t *tk = ki; ki = ko; ko = tk;
        V *tv = vi; vi = vo; vo = tv;
    }
    *sorted_in_1 = passes & 1;
    return 0;
}

int launch_radix_sort_u64(uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, const uint32_t *counts, int bit0,
                          int bits, int nparts, uint32_t *hist, uint32_t *partials, hipStream_t st, int *sorted_in_1) {
    return launch_radix_sort_keys(k0, k1, v0, v1, counts, bit0, bits, nparts, hist, partials, st, sorted_in_1, -1,
                                  nullptr);
}

// A projection writes the per-slot inputs of one bin sort only: binning for the other one finds
// no slots (and flags the status word) instead of reading buffers that projection left stale.
__global__ void prep_check_kernel(uint32_t *counts, uint32_t want, uint32_t *status) {
    if (counts[CNT_PREP] != want) {
        counts[CNT_SLOTS] = 0u;
        atomicOr(status, SPLAT_ST_SEQUENCE);
    }
}

int launch_bin_sort(const splat_plan &p, void *ws, hipStream_t st) {
    uint32_t *status = ws_at<uint32_t>(ws, p.off_status);
    uint32_t *counts = ws_at<uint32_t>(ws, p.off_counts);
    uint32_t *ntiles = ws_at<uint32_t>(ws, p.off_ntiles);
    uint32_t *partials = ws_at<uint32_t>(ws, p.off_scan);
    uint64_t *keys0 = ws_at<uint64_t>(ws, p.off_keys);
    uint64_t *keys1 = keys0 + p.inst_cap;
    uint32_t *vals0 = ws_at<uint32_t>(ws, p.off_vals);
    uint32_t *vals1 = vals0 + p.inst_cap;
    uint2 *ranges = ws_at<uint2>(ws, p.off_ranges);
    uint32_t *queue = ws_at<uint32_t>(ws, p.off_queue);
    uint32_t *hist = ws_at<uint32_t>(ws, p.off_hist);
    uint32_t *qh = hist + (size_t)kRadixDigits * p.n_sort_blocks + 1;
    int nT = p.n_views * p.tiles_per_view;

    int eb = (int)((p.slot_cap + 255) / 256);  // about one slot per thread
    if (eb > 65536) eb = 65536;
    int rc = 0, in1 = 0, kshift = -1;
    hipLaunchKernelGGL(prep_check_kernel, dim3(1), dim3(1), 0, st, counts, p.slot_sort ? kPrepSlotSort : kPrepInstSort,
                       status);
    if ((rc = launch_status("prep_check"))) return rc;
    if (p.slot_sort) {
        // slots by depth (the payload travels along), then the instances, emitted in that order,
        // by tile: stable sorts, so a tile's list is in (depth, slot) order as with the 64-bit keys
        uint64_t *pay0 = ws_at<uint64_t>(ws, p.off_spay), *pay1 = pay0 + p.slot_cap;
        uint32_t *soff = ws_at<uint32_t>(ws, p.off_soff);
        const PayBits pb{p.pack_bits[0], p.tile_bits, p.pack_bits[1]};
        int sin1 = 0;
        rc = launch_radix_sort_u32<uint64_t>(ws_at<uint32_t>(ws, p.off_dkey), ws_at<uint32_t>(ws, p.off_skeys), pay0,
                                             pay1, counts, CNT_SLOTS, p.depth_bits, p.n_sort_blocks, hist, partials, st,
                                             &sin1, false);  // only the payloads are read afterwards
        if (rc) return rc;
        const uint64_t *pay = sin1 ? pay1 : pay0;
        hipLaunchKernelGGL(run_tiles_kernel, dim3((eb + 3) / 4), dim3(256), 0, st, counts, pay, pb, soff);
        if ((rc = launch_status("run_tiles"))) return rc;
        if ((rc = launch_scan_u32(soff, soff, counts + CNT_RUNS, (p.slot_cap + 63) / 64, partials, nullptr, st)))
            return rc;
        hipLaunchKernelGGL(run_finish_kernel, dim3(1), dim3(64), 0, st, soff, pay, pb, p.inst_cap, counts, status);
        if ((rc = launch_status("run_finish"))) return rc;
        uint32_t *k32 = reinterpret_cast<uint32_t *>(keys0);
        hipLaunchKernelGGL(emit_sorted_kernel, dim3((eb + 3) / 4), dim3(256), 0, st, counts, soff, pay, pb, p.tiles_x,
                           k32, vals0);
        if ((rc = launch_status("emit_sorted"))) return rc;
        rc = launch_radix_sort_u32<uint32_t>(k32, reinterpret_cast<uint32_t *>(keys1), vals0, vals1, counts, CNT_INST,
                                             p.tile_bits, p.n_sort_blocks, hist, partials, st, &in1);
        if (rc) return rc;
        kshift = p.depth_bits;  // the instance keys are the tile field of the 64-bit key
    } else {
        // instance offsets: exclusive scan of the per-slot tile counts
        rc = launch_scan_u32(ntiles, ntiles, counts + CNT_SLOTS, p.slot_cap, partials, nullptr, st);
        if (rc) return rc;
        hipLaunchKernelGGL(inst_finish_kernel, dim3(1), dim3(64), 0, st, ntiles, p.inst_cap, counts, status);
        if ((rc = launch_status("inst_finish"))) return rc;
        hipLaunchKernelGGL(emit_kernel, dim3(eb), dim3(256), 0, st, counts, ntiles, ws_at<Rect16>(ws, p.off_rect),
                           ws_at<uint32_t>(ws, p.off_dkey), ws_at<int2>(ws, p.off_meta), p.tiles_x, p.tiles_per_view,
                           p.depth_bits, keys0, vals0);
        if ((rc = launch_status("emit"))) return rc;
        // LSD radix sort over the used key bits
        // the passes after the depth digits carry 32-bit keys (key >> key_shift, key_shift <= depth_bits)
        rc = launch_radix_sort_keys(keys0, keys1, vals0, vals1, counts, 0, p.depth_bits + p.tile_bits,
                                    p.n_sort_blocks, hist, partials, st, &in1, p.depth_bits, &kshift);
        if (rc) return rc;
    }
    if (kshift != p.key_shift || in1 != p.sorted_buf) {
        set_error("bin_sort: plan key shift %d / sorted buffer %d do not match the sort's %d / %d", p.key_shift,
                  p.sorted_buf, kshift, in1);
        return SPLAT_EINVAL;
    }
    const uint64_t *ki = in1 ? keys1 : keys0;
    // ranges of every (view, tile) and the cost-ordered queue
    if ((rc = launch_fill_u32(reinterpret_cast<uint32_t *>(ranges), 0u, (int64_t)2 * nT, st))) return rc;
    int rb = (int)((p.inst_cap / 4 + 256) / 256);
    if (rb > 8192) rb = 8192;
    if (kshift >= 0 && (reinterpret_cast<uintptr_t>(ki) & 15u) == 0)
        hipLaunchKernelGGL(ranges_vec_kernel, dim3(rb), dim3(256), 0, st, reinterpret_cast<const uint32_t *>(ki), counts,
                           p.depth_bits - kshift, (uint32_t)nT, ranges, qh);
    else if (kshift >= 0)
        hipLaunchKernelGGL(ranges_kernel<uint32_t>, dim3(rb), dim3(256), 0, st, reinterpret_cast<const uint32_t *>(ki),
                           counts, p.depth_bits - kshift, (uint64_t)nT, ranges, qh);
    else
        hipLaunchKernelGGL(ranges_kernel<uint64_t>, dim3(rb), dim3(256), 0, st, ki, counts, p.depth_bits, (uint64_t)nT,
                           ranges, qh);
    if ((rc = launch_status("ranges"))) return rc;
    int qb = (nT + 255) / 256;
    if (qb > 1024) qb = 1024;
    hipLaunchKernelGGL(queue_hist_kernel, dim3(qb), dim3(256), 0, st, ranges, nT, qh);
    if ((rc = launch_status("queue_hist"))) return rc;
    hipLaunchKernelGGL(queue_scatter_kernel, dim3(qb), dim3(256), 0, st, ranges, nT, qh, queue);
    if ((rc = launch_status("queue_scatter"))) return rc;

    // render-adjoint items: split lists first, each as its chunks, then the other tiles
    uint32_t *boff = ws_at<uint32_t>(ws, p.off_bqoff);
    int lc_log = 0;
    while ((1 << lc_log) < p.split_len) ++lc_log;
    hipLaunchKernelGGL(split_count_kernel, dim3(qb), dim3(256), 0, st, ranges, queue, nT, lc_log, boff, counts);
    if ((rc = launch_status("split_count"))) return rc;
    if ((rc = launch_scan_u32(boff, boff, counts + CNT_NSPLIT, nT, partials, counts + CNT_NCHUNK, st))) return rc;
    hipLaunchKernelGGL(split_items_kernel, dim3(qb), dim3(256), 0, st, ranges, queue, nT, boff, counts,
                       ws_at<uint4>(ws, p.off_bqueue), p.bq_cap);
    return launch_status("split_items");
}

}  // namespace splat
