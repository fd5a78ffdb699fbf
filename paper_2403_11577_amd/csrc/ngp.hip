// ngp.hip -- Gaussian parameters from a multiresolution hash grid and an MLP
// (F(X|Theta) of Sec. III-C: the model of Instant-NGP with four heads for colour,
// opacity, scale and rotation), forward and adjoint.
//
// Per Gaussian: the position is normalised into [0,1]^3 by the scene box; at every
// level l the cell of p = x_n N_l is found in float64 (so the cell and the trilinear
// weights are those of the definition), the 8 vertices are looked up -- dense index where
// the level's (N_l+1)^3 vertices fit in the table, spatial hash
// (v0 * 1) ^ (v1 * 2654435761) ^ (v2 * 805459861) mod T otherwise -- and blended; the 32
// features go through 32 -> 64 -> 64 -> 11 (ReLU); heads: colour and opacity sigmoid,
// scale scale_max * sigmoid, quaternion + (1, 0, 0, 0).  A wave takes a block of Gaussians at a
// time and runs the three layers on the matrix cores (see the MLP section below).
//
// Adjoint: the 11 output gradients are pushed back through the heads and the MLP (on the
// matrix cores, from the forward's values stored per Gaussian, or evaluated again), and
// the weight gradients -- sums over all Gaussians of outer products, a tall-skinny A^T B --
// are contracted on the matrix cores into per-workgroup partials (inside the adjoint that
// reads the stored values, by wgrad_kernel from the stored deltas otherwise), then reduced
// in a fixed float64 order.  The table gradient of a
// row is the sum, over every (Gaussian, vertex) that looked it up, of the
// trilinear weight times the Gaussian's encoding gradient.  Two ways to form it:
//  * scatter: hardware float atomics (16 levels x 8 vertices x 2 features), after
//    the lanes of a wave that share a row have been summed;
//  * indexed: the positions are fixed while the Gaussians are (a calibration stage
//    moves cameras, not Gaussians), so the lookups are inverted once -- every
//    (Gaussian, weight) pair sorted by (level, row) -- and each step reduces the
//    runs of that list: a workgroup sums 2048 consecutive pairs with a segmented
//    scan and writes every row whose run it holds whole, a second kernel adds up
//    the runs that cross workgroups.  No atomics, one writer per row, a fixed
//    summation order (float64), so the table gradient is reproducible bit for bit.
#include "common.hpp"

namespace splat {
namespace {

constexpr int NL = 16;       // max levels
constexpr int NF = 2;        // features per level
constexpr int ND = NL * NF;  // encoding width (levels * 2, padded to 32)
constexpr int NH = 64;       // hidden width
constexpr int NO = 11;       // outputs: colour 3, opacity 1, scale 3, quaternion 4
constexpr int NW = NH * ND + NH + NH * NH + NH + NO * NH + NO;  // weights in LDS

struct NgpArgs {
    int levels;
    uint32_t tmask;          // T - 1
    int64_t T;
    int res[NL];             // N_l
    int dense[NL];
    double lo[3], ext[3];
    float scale_max;
};

// both indexings are formed and one is selected: the dense flag may differ between the lanes
// of a wave, and a branch per vertex would keep the table reads from being issued together
__device__ __forceinline__ uint32_t vertex_row_n(int dense, uint32_t N, uint32_t tmask, uint32_t v0, uint32_t v1,
                                                 uint32_t v2) {
    const uint32_t m = N + 1u;
    const uint32_t rd = v0 + m * (v1 + m * v2);
    const uint32_t rh = ((v0 * 1u) ^ (v1 * 2654435761u) ^ (v2 * 805459861u)) & tmask;
    return dense ? rd : rh;
}

__device__ __forceinline__ uint32_t vertex_row(const NgpArgs &a, int l, uint32_t v0, uint32_t v1, uint32_t v2) {
    return vertex_row_n(a.dense[l], (uint32_t)a.res[l], a.tmask, v0, v1, v2);
}

// cell and fractions at resolution N
__device__ __forceinline__ void level_cell_n(int N, const double *xn, uint32_t *cell, double *fr) {
    for (int d = 0; d < 3; ++d) {
        double p = xn[d] * (double)N;
        double c = floor(p);
        if (c > (double)(N - 1)) c = (double)(N - 1);
        cell[d] = (uint32_t)c;
        fr[d] = p - c;
    }
}

__device__ __forceinline__ void level_cell(const NgpArgs &a, int l, const double *xn, uint32_t *cell, double *fr) {
    level_cell_n(a.res[l], xn, cell, fr);
}

__device__ __forceinline__ void normalise(const NgpArgs &a, const float *mean, int64_t n, int64_t i, double *xn) {
    for (int d = 0; d < 3; ++d) {
        double v = ((double)mean[d * n + i] - a.lo[d]) / a.ext[d];
        xn[d] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
    }
}

// the two features of level l (resolution N, dense indexing or not)
__device__ __forceinline__ void encode_at(const NgpArgs &a, const float2 *tables, int l, int N, int dense,
                                          const double *xn, float &e0, float &e1) {
    uint32_t cell[3];
    double fr[3];
    level_cell_n(N, xn, cell, fr);
    const float2 *tab = tables + (int64_t)l * a.T;
    e0 = 0.f;
    e1 = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
        double w = (cx ? fr[0] : 1.0 - fr[0]) * (cy ? fr[1] : 1.0 - fr[1]) * (cz ? fr[2] : 1.0 - fr[2]);
        float2 t = tab[vertex_row_n(dense, (uint32_t)N, a.tmask, cell[0] + cx, cell[1] + cy, cell[2] + cz)];
        e0 = __fmaf_rn((float)w, t.x, e0);
        e1 = __fmaf_rn((float)w, t.y, e1);
    }
}

// wave64 sum with DPP (quad swaps, half-row and row mirrors, row broadcasts); total in lane 63
template <int CTRL, int ROWS>
__device__ __forceinline__ float ngp_dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xF, false));
}

__device__ __forceinline__ float ngp_wave_total(float x) {
    x += ngp_dpp<0xB1, 0xF>(x);
    x += ngp_dpp<0x4E, 0xF>(x);
    x += ngp_dpp<0x141, 0xF>(x);
    x += ngp_dpp<0x140, 0xF>(x);
    x += ngp_dpp<0x142, 0xA>(x);
    x += ngp_dpp<0x143, 0xC>(x);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// tab[2e] += a0, tab[2e+1] += a1 for every lane with a non-zero pair (all 64 lanes active;
// e = level * T + row, so lanes of different levels never combine).  Lanes that share an
// entry are summed over the wave first, one entry at a time while an entry is shared by at
// least two lanes (the coarse levels, where many Gaussians sit in one cell); the rest go
// straight to the float atomics.
__device__ __forceinline__ void scatter2(float *tab, int64_t e, float a0, float a1) {
    const int lane = __lane_id();
    uint64_t todo = __ballot(a0 != 0.f || a1 != 0.f);  // Gaussians without a gradient add nothing
#pragma unroll 1
    for (int it = 0; it < 8 && todo; ++it) {
        int leader = __ffsll((long long)todo) - 1;
        const uint32_t klo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)e, leader);
        const uint32_t khi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)e >> 32), leader);
        const int64_t key = (int64_t)(((uint64_t)khi << 32) | klo);
        bool mine = ((todo >> lane) & 1ull) && e == key;
        uint64_t peers = __ballot(mine);
        if (__popcll(peers) < 2) break;
        float s0 = ngp_wave_total(mine ? a0 : 0.f), s1 = ngp_wave_total(mine ? a1 : 0.f);
        if (lane == leader) {
            atomicAdd(tab + 2 * key, s0);
            atomicAdd(tab + 2 * key + 1, s1);
        }
        todo &= ~peers;
    }
    if ((todo >> lane) & 1ull) {
        atomicAdd(tab + 2 * e, a0);
        atomicAdd(tab + 2 * e + 1, a1);
    }
}

// Stored activations and deltas, R_LEN values per Gaussian, kept feature-major: value f of
// Gaussian i at rows[f * ld + i] (ld = row_ld(n), a multiple of 64 above n, so the 64
// columns of every block of 64 or fewer Gaussians exist; columns past n are scratch), so that the
// 16 lanes of a lane group store 16 consecutive Gaussians.  R_O: the 11 outputs before the
// heads.  R_MASK: the ReLU decisions as bits, 16 per (layer, lane group) in the order the
// tile layout below holds them (R_MASK + 4 layer + q, bit 4 t + v for unit 16 t + 4 q + v), so
// that the adjoint reads 8 words per Gaussian instead of both hidden layers.
enum { R_DOUT = 0, R_H2 = 12, R_DH2 = R_H2 + NH, R_H1 = R_DH2 + NH, R_DH1 = R_H1 + NH, R_ENC = R_DH1 + NH,
       R_O = R_ENC + ND, R_MASK = R_O + 12, R_LEN = R_MASK + 8 };

__host__ __device__ inline int64_t row_ld(int64_t n) { return (n + 64) & ~(int64_t)63; }

// ---- the MLP on the matrix cores ----
//
// One wave evaluates the 16 FJ Gaussians g0 .. g0 + 16 FJ - 1 with v_mfma_f32_16x16x4f32
// (FP32 products and sums).  Lane l = 16 q + c (c = l % 16) holds every 16 x 16 block of a
// layer's features in "tile layout": register v of tile (t, j) is feature 16 t + 4 q + v of
// Gaussian g0 + 16 j + c (j < FJ).  That is the layout of an MFMA result (rows 4 q + v,
// column c), and it is also the layout in which the next layer takes the tile as its B
// operand when MFMA number v of an input tile uses, in lane group q, the input feature
// 16 t + 4 q + v as its k index: the layers chain in registers.  The A operand (weights)
// comes from LDS as one 16-byte read per lane for four consecutive MFMAs; weight rows are
// padded to 4 mod 32 floats, so the 16 rows a lane group reads fall into distinct banks.
// The encoding is computed in tile layout from the start: lane group q evaluates the levels
// 2 q, 2 q + 1, 8 + 2 q and 9 + 2 q of the lane's Gaussians g0 + 16 j + c.

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mma(float a, float b, f4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

constexpr int P32 = ND + 4, P64 = NH + 4, P16 = 16 + 4;  // padded row lengths (floats)

// forward weights: w3 and b3 padded to 16 outputs with zeros, w1 to 32 inputs
struct __align__(16) WFwd {
    float w1[NH][P32], w2[NH][P64], w3[16][P64], b1[NH], b2[NH], b3[16];
};

// adjoint weights, transposed: w3t[j][k] = w3[k][j] (k < 16), w2t[i][j] = w2[j][i], w1t[e][j] = w1[j][e]
struct __align__(16) WBwd {
    float w3t[NH][P16], w2t[NH][P64], w1t[ND][P64];
};

__device__ inline void load_fwd(WFwd &W, const float *w1, const float *b1, const float *w2, const float *b2,
                                const float *w3, const float *b3, int din) {
    for (int i = threadIdx.x; i < NH * ND; i += blockDim.x) {
        int r = i / ND, e = i - r * ND;
        W.w1[r][e] = e < din ? w1[r * din + e] : 0.f;
    }
    for (int i = threadIdx.x; i < NH * NH; i += blockDim.x) W.w2[i / NH][i % NH] = w2[i];
    for (int i = threadIdx.x; i < 16 * NH; i += blockDim.x) W.w3[i / NH][i % NH] = i < NO * NH ? w3[i] : 0.f;
    for (int i = threadIdx.x; i < NH; i += blockDim.x) {
        W.b1[i] = b1[i];
        W.b2[i] = b2[i];
    }
    for (int i = threadIdx.x; i < 16; i += blockDim.x) W.b3[i] = i < NO ? b3[i] : 0.f;
}

__device__ inline void load_bwd(WBwd &W, const float *w1, const float *w2, const float *w3, int din) {
    for (int i = threadIdx.x; i < NH * 16; i += blockDim.x) {
        int j = i / 16, k = i - j * 16;
        W.w3t[j][k] = k < NO ? w3[k * NH + j] : 0.f;
    }
    for (int i = threadIdx.x; i < NH * NH; i += blockDim.x) {
        int r = i / NH, cc = i - r * NH;
        W.w2t[cc][r] = w2[i];
    }
    for (int i = threadIdx.x; i < NH * ND; i += blockDim.x) {
        int j = i / ND, e = i - j * ND;
        W.w1t[e][j] = e < din ? w1[j * din + e] : 0.f;
    }
}

__device__ __forceinline__ f4 lds4(const float *p) { return *reinterpret_cast<const f4 *>(p); }

// levels evaluated by lane group q in slot s: 8 (s >> 1) + 2 q + (s & 1)
__device__ __forceinline__ int slot_level(int s, int q) { return 8 * (s >> 1) + 2 * q + (s & 1); }

// v[8 (s >> 1) + (s & 1) + 2 q] with the four candidates read as scalars
__device__ __forceinline__ int pick_level(const int *v, int s, int q) {
    const int b = 8 * (s >> 1) + (s & 1);
    int r = v[b];
    r = q == 1 ? v[b + 2] : r;
    r = q == 2 ? v[b + 4] : r;
    r = q == 3 ? v[b + 6] : r;
    return r;
}

__device__ __forceinline__ float sigm(float x) { return 1.f / (1.f + __expf(-x)); }

// The field for the 16 FJ Gaussians of block g0 (lanes past n evaluate the last Gaussian and
// write no parameters; PARAMS = false writes none at all).  SAVE: the encoding, both hidden layers (after the ReLU) and the
// outputs before the heads also go to the rows.
template <int FJ, bool SAVE, bool PARAMS = true>
__device__ __forceinline__ void field_block(const NgpArgs &a, const float2 *tables, const WFwd &W, const float *mean,
                                            int64_t n, int64_t g0, float *quat, float *scale, float *opac,
                                            float *color, float *rows) {
    const int lane = __lane_id(), c = lane & 15, q = lane >> 4;
    // the row stride, opaque to the compiler: the offsets of the stores below are then formed
    // where they are used, instead of all of them being hoisted out of the block loop
    int64_t ld = row_ld(n);
    asm volatile("" : "+s"(ld));
    // the lane's column of the rows at feature 4 q: feature F + 4 q + v of Gaussian g0 + 16 j + c
    // is lr[(F + v) ld + 16 j], a wave-uniform offset
    float *lr = SAVE ? rows + 4 * q * ld + g0 + c : nullptr;
    float *mr = SAVE ? rows + (int64_t)q * ld + g0 + c : nullptr;  // mask word R_MASK + 4 layer + q
    // opaque as well, so that every store adds a wave-uniform offset to them (otherwise the
    // compiler folds 4 q into a per-lane multiplier of ld for each store and keeps them all)
    asm volatile("" : "+v"(lr), "+v"(mr));
    f4 E[2][FJ];
    {
        double xn[FJ][3];
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
            const int64_t g = g0 + 16 * j + c;
            normalise(a, mean, n, g < n ? g : n - 1, xn[j]);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            // a level past the model's is evaluated at level 0 and contributes zero (no branch)
            const bool on = slot_level(s, q) < a.levels;
            const int l = on ? slot_level(s, q) : 0;
            const int N = on ? pick_level(a.res, s, q) : a.res[0];
            const int dense = on ? pick_level(a.dense, s, q) : a.dense[0];
#pragma unroll
            for (int j = 0; j < FJ; ++j) {
                float e0, e1;
                encode_at(a, tables, l, N, dense, xn[j], e0, e1);
                E[s >> 1][j][2 * (s & 1)] = on ? e0 : 0.f;
                E[s >> 1][j][2 * (s & 1) + 1] = on ? e1 : 0.f;
            }
            // one slot's 32 gathers in flight at a time (all of them at once would not fit the registers)
            asm volatile("" ::: "memory");
        }
    }
    if (SAVE)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int j = 0; j < FJ; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) lr[(int64_t)(R_ENC + 16 * t + v) * ld + 16 * j] = E[t][j][v];
    // hidden layer 1
    f4 H[4][FJ];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f4 b = lds4(&W.b1[16 * t + 4 * q]);
#pragma unroll
        for (int j = 0; j < FJ; ++j) H[t][j] = b;
    }
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const f4 w = lds4(&W.w1[16 * t + c][16 * kt + 4 * q]);
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int j = 0; j < FJ; ++j) H[t][j] = mma(w[v], E[kt][j][v], H[t][j]);
        }
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
        uint32_t m = 0u;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float h = H[t][j][v] > 0.f ? H[t][j][v] : 0.f;
                H[t][j][v] = h;
                m |= (h > 0.f ? 1u : 0u) << (4 * t + v);
                if (SAVE) lr[(int64_t)(R_H1 + 16 * t + v) * ld + 16 * j] = h;
            }
        if (SAVE) mr[(int64_t)R_MASK * ld + 16 * j] = __uint_as_float(m);
    }
    // hidden layer 2
    f4 G[4][FJ];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f4 b = lds4(&W.b2[16 * t + 4 * q]);
#pragma unroll
        for (int j = 0; j < FJ; ++j) G[t][j] = b;
    }
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const f4 w = lds4(&W.w2[16 * t + c][16 * kt + 4 * q]);
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int j = 0; j < FJ; ++j) G[t][j] = mma(w[v], H[kt][j][v], G[t][j]);
        }
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
        uint32_t m = 0u;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float h = G[t][j][v] > 0.f ? G[t][j][v] : 0.f;
                G[t][j][v] = h;
                m |= (h > 0.f ? 1u : 0u) << (4 * t + v);
                if (SAVE) lr[(int64_t)(R_H2 + 16 * t + v) * ld + 16 * j] = h;
            }
        if (SAVE) mr[(int64_t)(R_MASK + 4) * ld + 16 * j] = __uint_as_float(m);
    }
    // outputs (rows 11..15 of the padded w3 are zero)
    f4 O[FJ];
    {
        const f4 b = lds4(&W.b3[4 * q]);
#pragma unroll
        for (int j = 0; j < FJ; ++j) O[j] = b;
    }
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
        const f4 w = lds4(&W.w3[c][16 * kt + 4 * q]);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int j = 0; j < FJ; ++j) O[j] = mma(w[v], G[kt][j][v], O[j]);
    }
    // heads: output k = 4 q + v; colour 0..2 and opacity 3 sigmoid, scale 4..6
    // scale_max sigmoid, quaternion 7..10 + (1, 0, 0, 0)
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
        const int64_t g = g0 + 16 * j + c;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int k = 4 * q + v;
            const float o = O[j][v];
            if (SAVE && k < 12) lr[(int64_t)(R_O + v) * ld + 16 * j] = o;
            if (!PARAMS || g >= n || k >= NO) continue;
            const float s = sigm(o);
            if (k < 3) color[k * n + g] = s;
            else if (k == 3) opac[g] = s;
            else if (k < 7) scale[(k - 4) * n + g] = a.scale_max * s;
            else quat[(k - 7) * n + g] = k == 7 ? o + 1.f : o;
        }
    }
}

// The adjoint of block g0 from the stored rows: the output deltas D, dL/dh2 (G) and dL/dh1
// (H) are returned, and with STORE also written to the rows (for the weight-gradient kernel),
// the encoding gradients are returned too, all in tile layout (register v of tile (t, j):
// feature 16 t + 4 q + v of Gaussian g0 + 16 j + c; zero for lanes past n).
template <int FJ, bool STORE>
__device__ __forceinline__ void adjoint_block(const NgpArgs &a, const WBwd &W, int64_t n, int64_t g0,
                                              const float *dquat, const float *dscale, const float *dopac,
                                              const float *dcolor, float *rows, f4 (&dE)[2][FJ], f4 (&D)[FJ],
                                              f4 (&G)[4][FJ], f4 (&H)[4][FJ]) {
    const int lane = __lane_id(), c = lane & 15, q = lane >> 4;
    // the row stride, opaque to the compiler: the offsets of the stores below are then formed
    // where they are used, instead of all of them being hoisted out of the block loop
    int64_t ld = row_ld(n);
    asm volatile("" : "+s"(ld));
    float *lr = rows + 4 * q * ld + g0 + c;  // as in the forward
    asm volatile("" : "+v"(lr));
    // the ReLU decisions of the lane's units, loaded with the outputs before anything is stored
    uint32_t m1[FJ], m2[FJ];
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
        const float *mr = lr + (int64_t)(R_MASK - 3 * q) * ld + 16 * j;  // R_MASK + q
        m1[j] = __float_as_uint(mr[0]);
        m2[j] = __float_as_uint(mr[(int64_t)4 * ld]);
    }
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
        const int64_t g = g0 + 16 * j + c;
        const bool live = g < n;
        const int64_t gc = live ? g : n - 1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int k = 4 * q + v;
            float d = 0.f;
            if (k < NO) {
                const float o = lr[(int64_t)(R_O + v) * ld + 16 * j];
                const float s = sigm(o);
                if (k < 3) d = dcolor[k * n + gc] * s * (1.f - s);
                else if (k == 3) d = dopac[gc] * s * (1.f - s);
                else if (k < 7) d = dscale[(k - 4) * n + gc] * a.scale_max * s * (1.f - s);
                else d = dquat[(k - 7) * n + gc];
            }
            d = live ? d : 0.f;
            D[j][v] = d;
            if (STORE && k < 12) lr[(int64_t)(R_DOUT + v) * ld + 16 * j] = d;
        }
    }
    // dL/dh2 = w3^T dOut where h2 > 0
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int j = 0; j < FJ; ++j) G[t][j] = f4{0.f, 0.f, 0.f, 0.f};
        const f4 w = lds4(&W.w3t[16 * t + c][4 * q]);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int j = 0; j < FJ; ++j) G[t][j] = mma(w[v], D[j][v], G[t][j]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int j = 0; j < FJ; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float d = (m2[j] >> (4 * t + v)) & 1u ? G[t][j][v] : 0.f;
                G[t][j][v] = d;
                if (STORE) lr[(int64_t)(R_DH2 + 16 * t + v) * ld + 16 * j] = d;
            }
    // dL/dh1 = w2^T dL/dh2 where h1 > 0
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int j = 0; j < FJ; ++j) H[t][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const f4 w = lds4(&W.w2t[16 * t + c][16 * kt + 4 * q]);
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int j = 0; j < FJ; ++j) H[t][j] = mma(w[v], G[kt][j][v], H[t][j]);
        }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int j = 0; j < FJ; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float d = (m1[j] >> (4 * t + v)) & 1u ? H[t][j][v] : 0.f;
                H[t][j][v] = d;
                if (STORE) lr[(int64_t)(R_DH1 + 16 * t + v) * ld + 16 * j] = d;
            }
    // dL/denc = w1^T dL/dh1
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < FJ; ++j) dE[t][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const f4 w = lds4(&W.w1t[16 * t + c][16 * kt + 4 * q]);
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int j = 0; j < FJ; ++j) dE[t][j] = mma(w[v], H[kt][j][v], dE[t][j]);
        }
}

// SAVE: also store what the adjoint needs in the per-Gaussian rows.  Each wave takes blocks
// of FB = 16 FJ Gaussians; the weights are staged once per workgroup.  Measured at 2M
// Gaussians: the forward alone is fastest with 16 Gaussians per wave (fewer registers, five
// waves per SIMD to cover the table reads), the training forward with 64.
template <bool SAVE, int FJ = SAVE ? 4 : 1, int FB = 16 * FJ>
__global__ __launch_bounds__(256, 2) void ngp_fwd_kernel(NgpArgs a, const float *mean, int64_t n, const float2 *tables,
                                                      const float *w1, const float *b1, const float *w2,
                                                      const float *b2, const float *w3, const float *b3,
                                                      float *quat, float *scale, float *opac, float *color,
                                                      float *rows) {
    __shared__ WFwd W;
    load_fwd(W, w1, b1, w2, b2, w3, b3, 2 * a.levels);
    __syncthreads();
    const int64_t nblk = (n + FB - 1) / FB;
    for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < nblk; b += (int64_t)gridDim.x * 4)
        field_block<FJ, SAVE>(a, tables, W, mean, n, FB * b, quat, scale, opac, color, rows);
}

// ---- weight gradients on the matrix cores, contracted over the Gaussians ----
// dW3 = dOut^T h2 (dOut padded to 16 rows), dW2 = dh2^T h1, dW1 = dh1^T enc, and the bias
// gradients, the column sums of the deltas.  A wave adds 16 Gaussians g16 + 0..15 at a time.
// In an A tile lane (m, kq) (m = lane % 16, kq = lane / 16) holds in register s the delta of
// feature 16 t + m of Gaussian g16 + 4 kq + s; in a B tile, the activation of column 16 t + m
// of the same Gaussian; MFMA s then contracts the Gaussians {4 kq + s}.  The adjoint's deltas
// come in tile layout (Gaussian on the lane's low bits); transpose16 turns such a 16 x 16 tile
// into the A layout on the matrix cores: four MFMAs against selector matrices, each output
// element one product by 1.0 plus products by 0.0, so the values pass unchanged (the rows
// loaded by wgrad_kernel hold the same values, so all adjoint paths sum the same products in
// the same order).
constexpr int WG_NE3 = 12 * NH + 12, WG_NE2 = NH * NH + NH, WG_NE1 = NH * ND + NH;  // partial sizes
constexpr int WG_NE = WG_NE3 + WG_NE2 + WG_NE1;
constexpr int WG_FJ = 1;  // 16-Gaussian blocks per wave step of the saved adjoint (and of wgrad_kernel)

struct WAcc {
    f4 w3[4], w2[16], w1[8];  // C tiles (ti, tj): w3[tj], w2[4 ti + tj], w1[2 ti + tj]
    float b3, b2[4], b1[4];   // per lane: column sums of the deltas of features 16 t + lane % 16
};

__device__ __forceinline__ void wacc_zero(WAcc &acc) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc.w3[u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 16; ++u) acc.w2[u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 8; ++u) acc.w1[u] = f4{0.f, 0.f, 0.f, 0.f};
    acc.b3 = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) acc.b2[t] = acc.b1[t] = 0.f;
}

__device__ __forceinline__ f4 transpose16(const f4 x) {
    const int lane = __lane_id(), c = lane & 15, q = lane >> 4;
    f4 r = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 4; ++v) r = mma(x[v], c == 4 * q + v ? 1.f : 0.f, r);
    return r;
}

// four consecutive Gaussians g.. of feature row `row`; columns at or past n are scratch: zero
__device__ __forceinline__ f4 load_g4(const float *rows, int64_t ld, int row, int64_t g, int64_t n) {
    f4 v = *reinterpret_cast<const f4 *>(rows + (int64_t)row * ld + g);
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = g + s < n ? v[s] : 0.f;
    return v;
}

// adds the 16 Gaussians from g16 (g16 < n); D, G, H: the A tiles of dOut, dh2 and dh1.
// MASK selects the products (1: dW3, 2: dW2, 4: dW1); a tile's sum depends only on its own
// sequence of MFMAs, so any selection gives the same values for the products it forms.
template <int MASK>
__device__ __forceinline__ void wgrad_block(WAcc &acc, const f4 &D, const f4 (&G)[4], const f4 (&H)[4],
                                            const float *rows, int64_t ld, int64_t g16, int64_t n) {
    const int lane = __lane_id(), m = lane & 15, kq = lane >> 4;
    const int64_t g = g16 + 4 * kq;
    if constexpr ((MASK & 1) != 0) {
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
            const f4 h2 = load_g4(rows, ld, R_H2 + 16 * tj + m, g, n);
#pragma unroll
            for (int s = 0; s < 4; ++s) acc.w3[tj] = mma(D[s], h2[s], acc.w3[tj]);
        }
        acc.b3 += (D[0] + D[1]) + (D[2] + D[3]);
    }
    if constexpr ((MASK & 2) != 0) {
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
            const f4 h1 = load_g4(rows, ld, R_H1 + 16 * tj + m, g, n);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int ti = 0; ti < 4; ++ti) acc.w2[4 * ti + tj] = mma(G[ti][s], h1[s], acc.w2[4 * ti + tj]);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) acc.b2[t] += (G[t][0] + G[t][1]) + (G[t][2] + G[t][3]);
    }
    if constexpr ((MASK & 4) != 0) {
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
            const f4 en = load_g4(rows, ld, R_ENC + 16 * tj + m, g, n);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int ti = 0; ti < 4; ++ti) acc.w1[2 * ti + tj] = mma(H[ti][s], en[s], acc.w1[2 * ti + tj]);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) acc.b1[t] += (H[t][0] + H[t][1]) + (H[t][2] + H[t][3]);
    }
}

// The workgroup's sums, waves added in order in LDS (red: WG_NE floats), written to its slots
// of the three partial arrays ([group][WG_NE3], then [group][WG_NE2], then [group][WG_NE1]),
// each laid out as C[row][col] then the column sums of the deltas.  ngroups: the grid size.
template <int MASK>
__device__ __forceinline__ void wgrad_finish(WAcc &acc, float *red, float *partial, int ngroups) {
    const int w = threadIdx.x >> 6, lane = __lane_id(), m = lane & 15, kq = lane >> 4;
    // the bias sums of the four lane groups
    acc.b3 += __shfl_xor(acc.b3, 16, kWave);
    acc.b3 += __shfl_xor(acc.b3, 32, kWave);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        acc.b2[t] += __shfl_xor(acc.b2[t], 16, kWave);
        acc.b2[t] += __shfl_xor(acc.b2[t], 32, kWave);
        acc.b1[t] += __shfl_xor(acc.b1[t], 16, kWave);
        acc.b1[t] += __shfl_xor(acc.b1[t], 32, kWave);
    }
    float *r3 = red, *r2 = red + WG_NE3, *r1 = red + WG_NE3 + WG_NE2;
    for (int wv = 0; wv < 4; ++wv) {
        if (w == wv) {
            auto put = [&](float *d, int i, float v) { d[i] = wv == 0 ? v : d[i] + v; };
            if constexpr ((MASK & 1) != 0) {
#pragma unroll
                for (int tj = 0; tj < 4; ++tj)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int row = 4 * kq + i;
                        if (row < 12) put(r3, row * NH + 16 * tj + m, acc.w3[tj][i]);
                    }
                if (kq == 0 && m < 12) put(r3, 12 * NH + m, acc.b3);
            }
            if constexpr ((MASK & 2) != 0) {
#pragma unroll
                for (int ti = 0; ti < 4; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            put(r2, (16 * ti + 4 * kq + i) * NH + 16 * tj + m, acc.w2[4 * ti + tj][i]);
                if (kq == 0)
#pragma unroll
                    for (int t = 0; t < 4; ++t) put(r2, NH * NH + 16 * t + m, acc.b2[t]);
            }
            if constexpr ((MASK & 4) != 0) {
#pragma unroll
                for (int ti = 0; ti < 4; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            put(r1, (16 * ti + 4 * kq + i) * ND + 16 * tj + m, acc.w1[2 * ti + tj][i]);
                if (kq == 0)
#pragma unroll
                    for (int t = 0; t < 4; ++t) put(r1, NH * ND + 16 * t + m, acc.b1[t]);
            }
        }
        __syncthreads();
    }
    float *p3 = partial + (int64_t)blockIdx.x * WG_NE3;
    float *p2 = partial + (int64_t)ngroups * WG_NE3 + (int64_t)blockIdx.x * WG_NE2;
    float *p1 = partial + (int64_t)ngroups * (WG_NE3 + WG_NE2) + (int64_t)blockIdx.x * WG_NE1;
    if constexpr ((MASK & 1) != 0)
        for (int i = threadIdx.x; i < WG_NE3; i += blockDim.x) p3[i] = r3[i];
    if constexpr ((MASK & 2) != 0)
        for (int i = threadIdx.x; i < WG_NE2; i += blockDim.x) p2[i] = r2[i];
    if constexpr ((MASK & 4) != 0)
        for (int i = threadIdx.x; i < WG_NE1; i += blockDim.x) p1[i] = r1[i];
}

template <int MODE> struct __align__(16) BwdSmem { WFwd f; WBwd b; };
template <> struct __align__(16) BwdSmem<2> { WBwd b; };

// MODE 0: table gradients by atomics into dtables; MODE 1: the encoding gradients go to
// dEc[level][Gaussian] for the indexed reduction; MODE 2: as 1, with the forward's values
// read from the rows stored by the training forward instead of evaluated again (modes 0
// and 1 evaluate the field of the block and store the rows first).  Blocks of 32 Gaussians
// per wave in mode 2, 64 when the field is evaluated too.  Modes 0 and 1 store the deltas in
// the rows for wgrad_kernel; mode 2 adds the weight gradients itself from the registers, over
// the same blocks in the same order, into its workgroup's partial sums (partial).
template <int MODE, int FJ = MODE == 2 ? WG_FJ : 4, int FB = 16 * FJ>
__global__ __launch_bounds__(256, 2) void ngp_bwd_kernel(NgpArgs a, const float *mean, int64_t n, const float2 *tables,
                                                      const float *w1, const float *b1, const float *w2,
                                                      const float *b2, const float *w3, const float *b3,
                                                      const float *dquat, const float *dscale, const float *dopac,
                                                      const float *dcolor, float *dtables, float *rows, float2 *dEc,
                                                      float *partial) {
    __shared__ BwdSmem<MODE> S;
    if constexpr (MODE != 2) load_fwd(S.f, w1, b1, w2, b2, w3, b3, 2 * a.levels);
    load_bwd(S.b, w1, w2, w3, 2 * a.levels);
    __syncthreads();
    const int lane = __lane_id(), c = lane & 15, q = lane >> 4;
    const int64_t nblk = (n + FB - 1) / FB;
    WAcc acc;
    if constexpr (MODE == 2) wacc_zero(acc);
    for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < nblk; b += (int64_t)gridDim.x * 4) {
        const int64_t g0 = FB * b;
        if constexpr (MODE != 2)
            field_block<FJ, true, false>(a, tables, S.f, mean, n, g0, nullptr, nullptr, nullptr, nullptr, rows);
        f4 dE[2][FJ], D[FJ], G[4][FJ], H[4][FJ];
        adjoint_block<FJ, MODE != 2>(a, S.b, n, g0, dquat, dscale, dopac, dcolor, rows, dE, D, G, H);
        if constexpr (MODE == 2) {
            const int64_t ld = row_ld(n);
#pragma unroll
            for (int j = 0; j < FJ; ++j) {
                const int64_t g16 = g0 + 16 * j;
                if (g16 >= n) continue;  // wave-uniform
                f4 tg[4], th[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    tg[t] = transpose16(G[t][j]);
                    th[t] = transpose16(H[t][j]);
                }
                wgrad_block<7>(acc, transpose16(D[j]), tg, th, rows, ld, g16, n);
            }
        }
        if constexpr (MODE != 0) {
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int j = 0; j < FJ; ++j) {
                    const int64_t g = g0 + 16 * j + c;
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        const int l = 8 * t + 2 * q + p;
                        if (g < n && l < a.levels) dEc[(int64_t)l * n + g] = make_float2(dE[t][j][2 * p], dE[t][j][2 * p + 1]);
                    }
                }
        } else {
            // table adjoint: every (Gaussian, level, vertex) adds weight * dL/denc to its row
            double xn[FJ][3];
#pragma unroll
            for (int j = 0; j < FJ; ++j) {
                const int64_t g = g0 + 16 * j + c;
                normalise(a, mean, n, g < n ? g : n - 1, xn[j]);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int l = slot_level(s, q);
                const int N = pick_level(a.res, s, q), dense = pick_level(a.dense, s, q);
                const bool on = l < a.levels;
#pragma unroll
                for (int j = 0; j < FJ; ++j) {
                    const float de0 = dE[s >> 1][j][2 * (s & 1)], de1 = dE[s >> 1][j][2 * (s & 1) + 1];
                    uint32_t cell[3] = {0u, 0u, 0u};
                    double fr[3] = {0.0, 0.0, 0.0};
                    if (on) level_cell_n(N, xn[j], cell, fr);
#pragma unroll
                    for (int cc = 0; cc < 8; ++cc) {
                        int cx = cc & 1, cy = (cc >> 1) & 1, cz = (cc >> 2) & 1;
                        float w = (float)((cx ? fr[0] : 1.0 - fr[0]) * (cy ? fr[1] : 1.0 - fr[1]) * (cz ? fr[2] : 1.0 - fr[2]));
                        uint32_t r = vertex_row_n(dense, (uint32_t)N, a.tmask, cell[0] + cx, cell[1] + cy, cell[2] + cz);
                        // lanes past n carry zero deltas; levels past the model's add nothing
                        const bool add = on;
                        scatter2(dtables, add ? (int64_t)l * a.T + r : 0, add ? w * de0 : 0.f, add ? w * de1 : 0.f);
                    }
                }
            }
        }
    }
    if constexpr (MODE == 2) {
        __syncthreads();  // the weights in LDS are no longer read: their space takes the sums
        wgrad_finish<7>(acc, reinterpret_cast<float *>(&S), partial, (int)gridDim.x);
    }
}

// The weight gradients of modes 0 and 1 from the deltas they stored in the rows: the saved
// mode's blocks (16 WG_FJ Gaussians per wave step, the same grid), order and arithmetic, one
// product per launch (MASK 1, 2 or 4: fewer accumulators, more waves).
template <int MASK>
__global__ __launch_bounds__(256, 3) void wgrad_kernel(const float *rows, int64_t n, float *partial) {
    __shared__ float red[WG_NE];
    const int lane = __lane_id(), m = lane & 15, kq = lane >> 4;
    const int64_t ld = row_ld(n), nblk = (n + 16 * WG_FJ - 1) / (16 * WG_FJ);
    WAcc acc;
    wacc_zero(acc);
    for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < nblk; b += (int64_t)gridDim.x * 4) {
#pragma unroll
        for (int j = 0; j < WG_FJ; ++j) {
            const int64_t g16 = 16 * WG_FJ * b + 16 * j;
            if (g16 >= n) continue;  // wave-uniform
            const int64_t g = g16 + 4 * kq;
            f4 d = f4{0.f, 0.f, 0.f, 0.f}, tg[4], th[4];
            if ((MASK & 1) != 0 && m < 12) d = load_g4(rows, ld, R_DOUT + m, g, n);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                tg[t] = (MASK & 2) != 0 ? load_g4(rows, ld, R_DH2 + 16 * t + m, g, n) : f4{0.f, 0.f, 0.f, 0.f};
                th[t] = (MASK & 4) != 0 ? load_g4(rows, ld, R_DH1 + 16 * t + m, g, n) : f4{0.f, 0.f, 0.f, 0.f};
            }
            wgrad_block<MASK>(acc, d, tg, th, rows, ld, g16, n);
        }
    }
    __syncthreads();
    wgrad_finish<MASK>(acc, red, partial, (int)gridDim.x);
}

// out[e] += sum over workgroups of partial[g][e], in float64 and a fixed order (four
// interleaved sums of eight interleaved sums each, added in order); e < ma*nb is (i, j)
// of dw (i < mreal, j < din_w), the rest db[i] (i < mreal)
__global__ __launch_bounds__(256) void atb_reduce_kernel(const float *partial, int ngroups, int ma, int nb, int mreal,
                                                        int din_w, float *dw, float *db) {
    __shared__ double part[4][64];
    const int ne = ma * nb + ma;
    const int e = blockIdx.x * 64 + (threadIdx.x & 63), qg = threadIdx.x >> 6;
    double s = 0.0;
    if (e < ne) {
        // eight sums over every 32nd workgroup keep eight loads in flight; fixed order throughout
        double t[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int g = qg;
        for (; g + 28 < ngroups; g += 32)
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] += (double)partial[(int64_t)(g + 4 * u) * ne + e];
        for (; g < ngroups; g += 4) t[0] += (double)partial[(int64_t)g * ne + e];
        s = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    }
    part[qg][threadIdx.x & 63] = s;
    __syncthreads();
    if (qg != 0 || e >= ne) return;
    s = ((part[0][threadIdx.x] + part[1][threadIdx.x]) + part[2][threadIdx.x]) + part[3][threadIdx.x];
    if (e < ma * nb) {
        int i = e / nb, j = e - i * nb;
        if (i < mreal && j < din_w) dw[i * din_w + j] += (float)s;
    } else if (e - ma * nb < mreal) {
        db[e - ma * nb] += (float)s;
    }
}

constexpr int ATB_GROUPS = 1024;

// ---- the inverse index of the table lookups ----
constexpr int GT_T = 256;               // threads per reduction workgroup
constexpr int GT_EPT = 8;               // index entries per thread
constexpr int GT_TILE = GT_T * GT_EPT;  // entries per workgroup

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Index: per level, the 8 n (Gaussian, weight) pairs sorted by table row and padded with
// zero-weight pairs to whole tiles (so a tile never spans two levels); ent_g holds the
// Gaussian with bit 31 set on the first pair of a row's run; seg_row the row of every run;
// tile_seg the run of each tile's first pair, tile_nh the number of runs starting in it.
struct IndexLayout {
    int64_t E, P, tpl, ntiles, nseg_cap;
    size_t ent_g, ent_w, seg_row, tile_seg, tile_nh, end;
};

IndexLayout index_layout(int levels, int log2T, int64_t n) {
    IndexLayout L;
    L.E = 8 * n;
    L.P = (L.E + GT_TILE - 1) / GT_TILE * GT_TILE;
    L.tpl = L.P / GT_TILE;
    L.ntiles = (int64_t)levels * L.tpl;
    int64_t T = (int64_t)1 << log2T;
    L.nseg_cap = (int64_t)levels * (L.E < T ? L.E : T);
    int64_t tot = (int64_t)levels * L.P;
    size_t o = 0;
    L.ent_g = o; o = al256(o + (size_t)tot * 4);
    L.ent_w = o; o = al256(o + (size_t)tot * 4);
    L.seg_row = o; o = al256(o + (size_t)L.nseg_cap * 4);
    L.tile_seg = o; o = al256(o + (size_t)L.ntiles * 4);
    L.tile_nh = o; o = al256(o + (size_t)L.ntiles * 4);
    L.end = o;
    return L;
}

struct IndexBuildLayout {
    size_t counts, keys, vals, flags, hist, partials, end;
    int nparts;
};

IndexBuildLayout index_build_layout(int levels, int log2T, int64_t n) {
    IndexLayout I = index_layout(levels, log2T, n);
    int64_t te = (int64_t)levels * I.E, tp = (int64_t)levels * I.P;
    IndexBuildLayout B;
    int64_t np = (te + 8191) / 8192;
    B.nparts = (int)(np < 1 ? 1 : (np > 2048 ? 2048 : np));
    int64_t nh = (int64_t)kRadixDigits * B.nparts + 1;
    size_t o = 0;
    B.counts = o; o = al256(o + 8 * 4);
    B.keys = o; o = al256(o + (size_t)2 * te * 8);
    B.vals = o; o = al256(o + (size_t)2 * te * 4);
    B.flags = o; o = al256(o + (size_t)(tp + 1) * 4);
    B.hist = o; o = al256(o + (size_t)nh * 4);
    size_t p1 = scan_partials(tp + 1), p2 = scan_partials(nh);
    B.partials = o; o = al256(o + (p1 > p2 ? p1 : p2) * 4);
    B.end = o;
    return B;
}

// key = (level << log2T | row) << 32 | bits of the float weight, value = Gaussian; pair
// (l, i, c) at position (l n + i) 8 + c
__global__ void ngp_index_keys_kernel(NgpArgs a, int log2T, const float *mean, int64_t n, uint64_t *keys,
                                      uint32_t *vals, uint32_t *counts) {
    if (blockIdx.x == 0 && threadIdx.x == 0) counts[CNT_INST] = (uint32_t)((int64_t)a.levels * 8 * n);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double xn[3];
        normalise(a, mean, n, i, xn);
#pragma unroll 1
        for (int l = 0; l < a.levels; ++l) {
            uint32_t cell[3];
            double fr[3];
            level_cell(a, l, xn, cell, fr);
            uint64_t *kk = keys + ((int64_t)l * n + i) * 8;
            uint32_t *vv = vals + ((int64_t)l * n + i) * 8;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
                float w = (float)((cx ? fr[0] : 1.0 - fr[0]) * (cy ? fr[1] : 1.0 - fr[1]) * (cz ? fr[2] : 1.0 - fr[2]));
                uint32_t r = vertex_row(a, l, cell[0] + cx, cell[1] + cy, cell[2] + cz);
                kk[c] = ((uint64_t)(((uint32_t)l << log2T) | r) << 32) | (uint64_t)__float_as_uint(w);
                vv[c] = (uint32_t)i;
            }
        }
    }
}

// sorted pairs -> padded per-level layout, run-start flags
__global__ void ngp_index_place_kernel(const uint64_t *keys, const uint32_t *vals, int levels, int64_t E, int64_t P,
                                       uint32_t *ent_g, float *ent_w, uint32_t *flags) {
    const int64_t tot = (int64_t)levels * P;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t l = i / P, j = i - l * P;
        uint32_t g = 0u, head = 0u;
        float w = 0.f;
        if (j < E) {
            int64_t s = l * E + j;
            uint64_t k = keys[s];
            head = (j == 0 || (keys[s - 1] >> 32) != (k >> 32)) ? 1u : 0u;
            g = vals[s];
            w = __uint_as_float((uint32_t)k);
        }
        ent_g[i] = g | (head << 31);
        ent_w[i] = w;
        flags[i] = head;
    }
}

// after the exclusive scan of the flags: the row of every run and the tile metadata
__global__ void ngp_index_meta_kernel(const uint64_t *keys, const uint32_t *ent_g, const uint32_t *excl, int levels,
                                      int64_t E, int64_t P, uint32_t tmask, uint32_t *seg_row, uint32_t *tile_seg,
                                      uint32_t *tile_nh) {
    const int64_t tot = (int64_t)levels * P;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t head = ent_g[i] >> 31;
        uint32_t x = excl[i];
        if (head) {
            int64_t l = i / P, j = i - l * P;
            seg_row[x] = (uint32_t)(keys[l * E + j] >> 32) & tmask;
        }
        if (i % GT_TILE == 0) {
            int64_t t = i / GT_TILE;
            tile_seg[t] = x + head - 1u;
            tile_nh[t] = excl[i + GT_TILE] - x;
        }
    }
}

// running sum of a segmented sequence: c runs start in it, s = sum after the last start
// (of everything when c = 0)
struct SegAcc {
    uint32_t c;
    double s0, s1;
};

__device__ __forceinline__ SegAcc seg_join(const SegAcc &a, const SegAcc &b) {  // a, then b
    SegAcc r;
    r.c = a.c + b.c;
    r.s0 = b.c ? b.s0 : a.s0 + b.s0;
    r.s1 = b.c ? b.s1 : a.s1 + b.s1;
    return r;
}

// One workgroup per tile of GT_TILE pairs (thread t owns pairs [8t, 8t + 8)).  A run that
// starts and ends in the tile is written here (its only writer); the partial sum of a run
// that started in an earlier tile and ends here goes to carry_head, that of the run still
// open at the tile's end to carry_tail.
__global__ __launch_bounds__(GT_T) void ngp_gather_kernel(int64_t n, int64_t T, int64_t tpl, int64_t ntiles,
                                                         const uint32_t *ent_g, const float *ent_w,
                                                         const uint32_t *seg_row, const uint32_t *tile_seg,
                                                         const float2 *dEc, float *dtables, double2 *carry_head,
                                                         double2 *carry_tail) {
    __shared__ SegAcc wagg[GT_T / 64];
    __shared__ uint32_t first_head[GT_T];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t l = tile / tpl;
    const int64_t base = tile * GT_TILE + (int64_t)t * GT_EPT;
    const float2 *de = dEc + l * n;
    const uint4 ga = *reinterpret_cast<const uint4 *>(ent_g + base);
    const uint4 gb = *reinterpret_cast<const uint4 *>(ent_g + base + 4);
    const float4 wa = *reinterpret_cast<const float4 *>(ent_w + base);
    const float4 wb = *reinterpret_cast<const float4 *>(ent_w + base + 4);
    const uint32_t g[GT_EPT] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z, gb.w};
    const float wt[GT_EPT] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
    float v0[GT_EPT], v1[GT_EPT];
#pragma unroll
    for (int k = 0; k < GT_EPT; ++k) {
        float2 d = de[g[k] & 0x7FFFFFFFu];
        v0[k] = wt[k] * d.x;
        v1[k] = wt[k] * d.y;
    }
    SegAcc agg = {0u, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < GT_EPT; ++k) {
        if (g[k] >> 31) {
            agg.c += 1u;
            agg.s0 = v0[k];
            agg.s1 = v1[k];
        } else {
            agg.s0 += v0[k];
            agg.s1 += v1[k];
        }
    }
    // exclusive scan over the workgroup, in thread order
    SegAcc inc = agg;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        SegAcc o;
        o.c = __shfl_up(inc.c, off);
        o.s0 = __shfl_up(inc.s0, off);
        o.s1 = __shfl_up(inc.s1, off);
        if (lane >= off) inc = seg_join(o, inc);
    }
    SegAcc ex;
    ex.c = __shfl_up(inc.c, 1);
    ex.s0 = __shfl_up(inc.s0, 1);
    ex.s1 = __shfl_up(inc.s1, 1);
    if (lane == 0) ex = SegAcc{0u, 0.0, 0.0};
    if (lane == 63) wagg[w] = inc;
    first_head[t] = g[0] >> 31;
    __syncthreads();
    SegAcc pre = {0u, 0.0, 0.0};
    for (int q = 0; q < w; ++q) pre = seg_join(pre, wagg[q]);
    ex = seg_join(pre, ex);
    uint32_t next_head;
    if (t < GT_T - 1) next_head = first_head[t + 1];
    else next_head = tile + 1 < ntiles ? ent_g[(tile + 1) * GT_TILE] >> 31 : 1u;
    const uint32_t hf = first_head[0];
    const uint32_t seg0 = tile_seg[tile];
    uint32_t heads = ex.c;
    double r0 = ex.s0, r1 = ex.s1;
    float *tab = dtables + l * T * 2;
#pragma unroll
    for (int k = 0; k < GT_EPT; ++k) {
        if (g[k] >> 31) {
            heads += 1u;
            r0 = v0[k];
            r1 = v1[k];
        } else {
            r0 += v0[k];
            r1 += v1[k];
        }
        uint32_t last = k < GT_EPT - 1 ? g[k + 1] >> 31 : next_head;
        if (last) {
            if (heads > 0u) {
                float *dt = tab + 2 * (int64_t)seg_row[seg0 + heads - hf];
                dt[0] += (float)r0;
                dt[1] += (float)r1;
            } else {
                carry_head[tile] = make_double2(r0, r1);
            }
        } else if (t == GT_T - 1 && k == GT_EPT - 1) {
            carry_tail[tile] = make_double2(r0, r1);
        }
    }
}

// Runs that cross tiles: the tile where such a run starts adds the carries of the tiles it
// covers, in order, and writes the row.
__global__ void ngp_fixup_kernel(int64_t T, int64_t tpl, int64_t ntiles, const uint32_t *ent_g,
                                 const uint32_t *seg_row, const uint32_t *tile_seg, const uint32_t *tile_nh,
                                 const double2 *carry_head, const double2 *carry_tail, float *dtables) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (t + 1 >= ntiles || (ent_g[(t + 1) * GT_TILE] >> 31) || tile_nh[t] == 0u) continue;
        double s0 = carry_tail[t].x, s1 = carry_tail[t].y;
        for (int64_t u = t + 1;; ++u) {
            bool ends = tile_nh[u] > 0u || u + 1 >= ntiles || (ent_g[(u + 1) * GT_TILE] >> 31);
            const double2 c = ends ? carry_head[u] : carry_tail[u];
            s0 += c.x;
            s1 += c.y;
            if (ends) break;
        }
        uint32_t seg = tile_seg[t] + tile_nh[t] - (ent_g[t * GT_TILE] >> 31);
        float *dt = dtables + ((t / tpl) * T + seg_row[seg]) * 2;
        dt[0] += (float)s0;
        dt[1] += (float)s1;
    }
}

// workgroups of the field kernels: four waves of fb Gaussians each per pass, at most 1024
// workgroups (the weights are staged once per workgroup)
int64_t field_groups(int64_t n, int fb) {
    int64_t g = (n + 4 * fb - 1) / (4 * fb);
    return g < 1 ? 1 : (g > 1024 ? 1024 : g);
}

int ngp_args(const splat_ngp &m, NgpArgs &a) {
    a.levels = m.levels;
    a.T = (int64_t)1 << m.log2_table;
    a.tmask = (uint32_t)(a.T - 1);
    double b = m.levels > 1 ? exp(log((double)m.n_max / (double)m.n_min) / (double)(m.levels - 1)) : 1.0;
    for (int l = 0; l < NL; ++l) {
        a.res[l] = 0;
        a.dense[l] = 0;
        if (l >= m.levels) continue;
        a.res[l] = (int)floor((double)m.n_min * pow(b, (double)l));
        double v = (double)a.res[l] + 1.0;
        a.dense[l] = v * v * v <= (double)a.T;
    }
    for (int d = 0; d < 3; ++d) {
        a.lo[d] = m.lo[d];
        a.ext[d] = m.hi[d] - m.lo[d];
    }
    a.scale_max = (float)m.scale_max;
    return 0;
}

// adjoint scratch: per-Gaussian rows, A^T B partials, encoding gradients per level (indexed
// path) and the run carries of the indexed reduction
struct WsLayout {
    size_t rows, partial, dec, carry_head, carry_tail, end;
};

WsLayout ws_layout(int64_t n) {
    WsLayout W;
    int64_t ntiles = (int64_t)NL * ((8 * n + GT_TILE - 1) / GT_TILE);
    size_t o = 0;
    W.rows = o; o = al256(o + (size_t)row_ld(n) * R_LEN * sizeof(float));
    W.partial = o; o = al256(o + (size_t)ATB_GROUPS * WG_NE * sizeof(float));
    W.dec = o; o = al256(o + (size_t)NL * n * sizeof(float2));
    W.carry_head = o; o = al256(o + (size_t)ntiles * sizeof(double2));
    W.carry_tail = o; o = al256(o + (size_t)ntiles * sizeof(double2));
    W.end = o;
    return W;
}

}  // namespace

size_t ngp_ws_bytes(int64_t n) { return ws_layout(n).end; }

size_t ngp_index_bytes(const splat_ngp &m, int64_t n) { return index_layout(m.levels, m.log2_table, n).end; }

size_t ngp_index_ws_bytes(const splat_ngp &m, int64_t n) {
    return index_build_layout(m.levels, m.log2_table, n).end;
}

int launch_ngp_index_build(const splat_ngp &m, const float *mean, int64_t n, void *index, void *ws, hipStream_t st) {
    NgpArgs a;
    ngp_args(m, a);
    const IndexLayout I = index_layout(m.levels, m.log2_table, n);
    const IndexBuildLayout Bl = index_build_layout(m.levels, m.log2_table, n);
    const int64_t te = (int64_t)m.levels * I.E, tp = (int64_t)m.levels * I.P;
    uint32_t *counts = ws_at<uint32_t>(ws, Bl.counts);
    uint64_t *k0 = ws_at<uint64_t>(ws, Bl.keys), *k1 = k0 + te;
    uint32_t *v0 = ws_at<uint32_t>(ws, Bl.vals), *v1 = v0 + te;
    uint32_t *flags = ws_at<uint32_t>(ws, Bl.flags);
    int64_t nb = (n + 255) / 256;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(ngp_index_keys_kernel, dim3((unsigned)nb), dim3(256), 0, st, a, m.log2_table, mean, n, k0, v0,
                       counts);
    int rc = launch_status("ngp_index_keys");
    if (rc) return rc;
    int lb = 0;
    while ((1 << lb) < m.levels) ++lb;
    int in1 = 0;
    rc = launch_radix_sort_u64(k0, k1, v0, v1, counts, 32, m.log2_table + lb, Bl.nparts, ws_at<uint32_t>(ws, Bl.hist),
                               ws_at<uint32_t>(ws, Bl.partials), st, &in1);
    if (rc) return rc;
    const uint64_t *ks = in1 ? k1 : k0;
    const uint32_t *vs = in1 ? v1 : v0;
    uint32_t *ent_g = ws_at<uint32_t>(index, I.ent_g);
    int64_t gb = (tp + 255) / 256;
    if (gb > 16384) gb = 16384;
    hipLaunchKernelGGL(ngp_index_place_kernel, dim3((unsigned)gb), dim3(256), 0, st, ks, vs, m.levels, I.E, I.P,
                       ent_g, ws_at<float>(index, I.ent_w), flags);
    if ((rc = launch_status("ngp_index_place"))) return rc;
    if ((rc = launch_scan_u32(flags, flags, nullptr, tp, ws_at<uint32_t>(ws, Bl.partials), nullptr, st))) return rc;
    hipLaunchKernelGGL(ngp_index_meta_kernel, dim3((unsigned)gb), dim3(256), 0, st, ks, ent_g, flags, m.levels, I.E,
                       I.P, a.tmask, ws_at<uint32_t>(index, I.seg_row), ws_at<uint32_t>(index, I.tile_seg),
                       ws_at<uint32_t>(index, I.tile_nh));
    return launch_status("ngp_index_meta");
}

namespace {
// weight gradients: dW3 = sum dOut^T h2 (11 x 64, dOut padded to 12), dW2 = sum dh2^T h1,
// dW1 = sum dh1^T enc (enc padded to 32 columns); biases are the column sums of the deltas
// the weight gradients from the partials of the ng workgroups of the saved adjoint or of
// wgrad_kernel: dW3 (11 x 64), dW2 (64 x 64), dW1 (64 x 2 levels) and the biases
int launch_wgrad_reduce(const splat_ngp &m, int ng, float *partial, float *dw1, float *db1, float *dw2, float *db2,
                        float *dw3, float *db3, hipStream_t st) {
    auto reduce = [&](const float *part, int ma, int nb, int mreal, int dinw, float *dw, float *db) {
        int ne = ma * nb + ma;
        hipLaunchKernelGGL(atb_reduce_kernel, dim3((unsigned)((ne + 63) / 64)), dim3(256), 0, st, part, ng, ma, nb,
                           mreal, dinw, dw, db);
        return launch_status("ngp_wgrad_reduce");
    };
    int rc;
    if ((rc = reduce(partial, 12, NH, NO, NH, dw3, db3))) return rc;
    if ((rc = reduce(partial + (int64_t)ng * WG_NE3, NH, NH, NH, NH, dw2, db2))) return rc;
    return reduce(partial + (int64_t)ng * (WG_NE3 + WG_NE2), NH, ND, NH, 2 * m.levels, dw1, db1);
}

int launch_wgrad(const splat_ngp &m, int64_t n, float *rows, float *partial, float *dw1, float *db1, float *dw2,
                 float *db2, float *dw3, float *db3, hipStream_t st) {
    const int ng = (int)field_groups(n, 16 * WG_FJ);  // the saved adjoint's grid
    hipLaunchKernelGGL(wgrad_kernel<1>, dim3((unsigned)ng), dim3(256), 0, st, rows, n, partial);
    hipLaunchKernelGGL(wgrad_kernel<2>, dim3((unsigned)ng), dim3(256), 0, st, rows, n, partial);
    hipLaunchKernelGGL(wgrad_kernel<4>, dim3((unsigned)ng), dim3(256), 0, st, rows, n, partial);
    int rc = launch_status("ngp_wgrad");
    if (rc) return rc;
    return launch_wgrad_reduce(m, ng, partial, dw1, db1, dw2, db2, dw3, db3, st);
}
}  // namespace

namespace {
// adjoint with the table gradients through the index; saved: the forward's values come from
// the rows of the training forward (mean and the tables are not read)
int ngp_bwd_via_index(const splat_ngp &m, const float *mean, int64_t n, const void *index, const float *dquat,
                      const float *dscale, const float *dopac, const float *dcolor, void *ws, float *dtables,
                      float *dw1, float *db1, float *dw2, float *db2, float *dw3, float *db3, bool saved,
                      hipStream_t st) {
    NgpArgs a;
    ngp_args(m, a);
    const WsLayout W = ws_layout(n);
    const IndexLayout I = index_layout(m.levels, m.log2_table, n);
    float *rows = ws_at<float>(ws, W.rows);
    float2 *dEc = ws_at<float2>(ws, W.dec);
    const int64_t nb = field_groups(n, saved ? 16 * WG_FJ : 64);
    const float2 *tab = reinterpret_cast<const float2 *>(m.tables);
    float *partial = ws_at<float>(ws, W.partial);
    if (saved)
        hipLaunchKernelGGL(ngp_bwd_kernel<2>, dim3((unsigned)nb), dim3(256), 0, st, a, mean, n, tab, m.w1, m.b1,
                           m.w2, m.b2, m.w3, m.b3, dquat, dscale, dopac, dcolor, dtables, rows, dEc, partial);
    else
        hipLaunchKernelGGL(ngp_bwd_kernel<1>, dim3((unsigned)nb), dim3(256), 0, st, a, mean, n, tab, m.w1, m.b1,
                           m.w2, m.b2, m.w3, m.b3, dquat, dscale, dopac, dcolor, dtables, rows, dEc, nullptr);
    int rc = launch_status("ngp_bwd");
    if (rc) return rc;
    void *ix = const_cast<void *>(index);
    const uint32_t *ent_g = ws_at<uint32_t>(ix, I.ent_g);
    const uint32_t *seg_row = ws_at<uint32_t>(ix, I.seg_row), *tile_seg = ws_at<uint32_t>(ix, I.tile_seg);
    double2 *ch = ws_at<double2>(ws, W.carry_head), *ct = ws_at<double2>(ws, W.carry_tail);
    hipLaunchKernelGGL(ngp_gather_kernel, dim3((unsigned)I.ntiles), dim3(GT_T), 0, st, n, a.T, I.tpl, I.ntiles, ent_g,
                       ws_at<float>(ix, I.ent_w), seg_row, tile_seg, dEc, dtables, ch, ct);
    if ((rc = launch_status("ngp_gather"))) return rc;
    int64_t fb = (I.ntiles + 255) / 256;
    hipLaunchKernelGGL(ngp_fixup_kernel, dim3((unsigned)fb), dim3(256), 0, st, a.T, I.tpl, I.ntiles, ent_g, seg_row,
                       tile_seg, ws_at<uint32_t>(ix, I.tile_nh), ch, ct, dtables);
    if ((rc = launch_status("ngp_fixup"))) return rc;
    if (saved) return launch_wgrad_reduce(m, (int)nb, partial, dw1, db1, dw2, db2, dw3, db3, st);
    return launch_wgrad(m, n, rows, partial, dw1, db1, dw2, db2, dw3, db3, st);
}

int ngp_fwd(const splat_ngp &m, const float *mean, int64_t n, float *quat, float *scale, float *opac, float *color,
            float *rows, hipStream_t st) {
    NgpArgs a;
    ngp_args(m, a);
    const int64_t nb = field_groups(n, rows ? 64 : 16);
    const float2 *tab = reinterpret_cast<const float2 *>(m.tables);
    if (rows)
        hipLaunchKernelGGL(ngp_fwd_kernel<true>, dim3((unsigned)nb), dim3(256), 0, st, a, mean, n, tab, m.w1, m.b1,
                           m.w2, m.b2, m.w3, m.b3, quat, scale, opac, color, rows);
    else
        hipLaunchKernelGGL(ngp_fwd_kernel<false>, dim3((unsigned)nb), dim3(256), 0, st, a, mean, n, tab, m.w1, m.b1,
                           m.w2, m.b2, m.w3, m.b3, quat, scale, opac, color, rows);
    return launch_status("ngp_fwd");
}
}  // namespace

int launch_ngp_bwd_indexed(const splat_ngp &m, const float *mean, int64_t n, const void *index, const float *dquat,
                           const float *dscale, const float *dopac, const float *dcolor, void *ws, float *dtables,
                           float *dw1, float *db1, float *dw2, float *db2, float *dw3, float *db3, hipStream_t st) {
    return ngp_bwd_via_index(m, mean, n, index, dquat, dscale, dopac, dcolor, ws, dtables, dw1, db1, dw2, db2, dw3,
                             db3, false, st);
}

int launch_ngp_bwd_saved(const splat_ngp &m, int64_t n, const void *index, const float *dquat, const float *dscale,
                         const float *dopac, const float *dcolor, void *ws, float *dtables, float *dw1, float *db1,
                         float *dw2, float *db2, float *dw3, float *db3, hipStream_t st) {
    return ngp_bwd_via_index(m, nullptr, n, index, dquat, dscale, dopac, dcolor, ws, dtables, dw1, db1, dw2, db2, dw3,
                             db3, true, st);
}

int launch_ngp_fwd(const splat_ngp &m, const float *mean, int64_t n, float *quat, float *scale, float *opac,
                   float *color, hipStream_t st) {
    return ngp_fwd(m, mean, n, quat, scale, opac, color, nullptr, st);
}

int launch_ngp_fwd_train(const splat_ngp &m, const float *mean, int64_t n, float *quat, float *scale, float *opac,
                         float *color, void *ws, hipStream_t st) {
    return ngp_fwd(m, mean, n, quat, scale, opac, color, ws_at<float>(ws, ws_layout(n).rows), st);
}

int launch_ngp_bwd(const splat_ngp &m, const float *mean, int64_t n, const float *dquat, const float *dscale,
                   const float *dopac, const float *dcolor, void *ws, float *dtables, float *dw1, float *db1,
                   float *dw2, float *db2, float *dw3, float *db3, hipStream_t st) {
    NgpArgs a;
    ngp_args(m, a);
    const WsLayout W = ws_layout(n);
    float *rows = ws_at<float>(ws, W.rows);
    const int64_t nb = field_groups(n, 64);
    hipLaunchKernelGGL(ngp_bwd_kernel<0>, dim3((unsigned)nb), dim3(256), 0, st, a, mean, n,
                       reinterpret_cast<const float2 *>(m.tables), m.w1, m.b1, m.w2, m.b2, m.w3, m.b3, dquat, dscale,
                       dopac, dcolor, dtables, rows, nullptr, nullptr);
    int rc = launch_status("ngp_bwd");
    if (rc) return rc;
    return launch_wgrad(m, n, rows, ws_at<float>(ws, W.partial), dw1, db1, dw2, db2, dw3, db3, st);
}

}  // namespace splat
