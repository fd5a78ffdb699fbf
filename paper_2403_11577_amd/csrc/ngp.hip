// ngp.hip -- Gaussian parameters from a multiresolution hash grid and an MLP
// (F(X|Theta) of Sec. III-C: the model of Instant-NGP with four heads for colour,
// opacity, scale and rotation), forward and adjoint.
//
// Per Gaussian (one thread): the position is normalised into [0,1]^3 by the scene
// box; at every level l the cell of p = x_n N_l is found in float64 (so the cell
// and the trilinear weights are those of the definition), the 8 vertices are
// looked up -- dense index where the level's (N_l+1)^3 vertices fit in the table,
// spatial hash (v0 * 1) ^ (v1 * 2654435761) ^ (v2 * 805459861) mod T otherwise --
// and blended; the 32 features go through 32 -> 64 -> 64 -> 11 (ReLU) with the
// weights broadcast from LDS; heads: colour and opacity sigmoid, scale
// scale_max * sigmoid, quaternion + (1, 0, 0, 0).
//
// Adjoint: the forward is recomputed, the 11 output gradients are pushed back
// through the heads and the MLP, table gradients are scattered with hardware
// float atomics (16 levels x 8 vertices x 2 features) after the lanes of a wave
// that share a table row have been summed (coarse levels), and the per-Gaussian
// activations and deltas are stored so that the weight gradients -- sums over all
// Gaussians of outer products, a tall-skinny A^T B -- are formed by atb_kernel
// (per-workgroup partials in registers, then a fixed-order reduction).
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

__device__ __forceinline__ uint32_t vertex_row(const NgpArgs &a, int l, uint32_t v0, uint32_t v1, uint32_t v2) {
    if (a.dense[l]) {
        uint32_t n = (uint32_t)a.res[l] + 1u;
        return v0 + n * (v1 + n * v2);
    }
    return ((v0 * 1u) ^ (v1 * 2654435761u) ^ (v2 * 805459861u)) & a.tmask;
}

// cell and fractions of level l
__device__ __forceinline__ void level_cell(const NgpArgs &a, int l, const double *xn, uint32_t *cell, double *fr) {
    int N = a.res[l];
    for (int d = 0; d < 3; ++d) {
        double p = xn[d] * (double)N;
        double c = floor(p);
        if (c > (double)(N - 1)) c = (double)(N - 1);
        cell[d] = (uint32_t)c;
        fr[d] = p - c;
    }
}

__device__ __forceinline__ void normalise(const NgpArgs &a, const float *mean, int64_t n, int64_t i, double *xn) {
    for (int d = 0; d < 3; ++d) {
        double v = ((double)mean[d * n + i] - a.lo[d]) / a.ext[d];
        xn[d] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
    }
}

// the two features of level l
__device__ __forceinline__ void encode_level(const NgpArgs &a, const float2 *tables, const double *xn, int l,
                                             float &e0, float &e1) {
    uint32_t cell[3];
    double fr[3];
    level_cell(a, l, xn, cell, fr);
    const float2 *tab = tables + (int64_t)l * a.T;
    e0 = 0.f;
    e1 = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
        double w = (cx ? fr[0] : 1.0 - fr[0]) * (cy ? fr[1] : 1.0 - fr[1]) * (cz ? fr[2] : 1.0 - fr[2]);
        float2 t = tab[vertex_row(a, l, cell[0] + cx, cell[1] + cy, cell[2] + cz)];
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

// tab[2r] += a0, tab[2r+1] += a1 for every lane with a non-zero pair (all 64 lanes active,
// e.g. Gaussians outside every view of the batch carry no gradient).  Lanes that share a
// row are summed over the wave first, one row at a time while a row is shared by at least two
// lanes (the coarse levels, where the whole wave often sits in one cell); the rest go
// straight to the float atomics.
__device__ __forceinline__ void scatter2(float *tab, uint32_t r, float a0, float a1) {
    const int lane = __lane_id();
    uint64_t todo = __ballot(a0 != 0.f || a1 != 0.f);  // Gaussians without a gradient add nothing
#pragma unroll 1
    for (int it = 0; it < 8 && todo; ++it) {
        int leader = __ffsll((long long)todo) - 1;
        uint32_t key = (uint32_t)__builtin_amdgcn_readlane((int)r, leader);
        bool mine = ((todo >> lane) & 1ull) && r == key;
        uint64_t peers = __ballot(mine);
        if (__popcll(peers) < 2) break;
        float s0 = ngp_wave_total(mine ? a0 : 0.f), s1 = ngp_wave_total(mine ? a1 : 0.f);
        if (lane == leader) {
            atomicAdd(tab + 2 * (int64_t)key, s0);
            atomicAdd(tab + 2 * (int64_t)key + 1, s1);
        }
        todo &= ~peers;
    }
    if ((todo >> lane) & 1ull) {
        atomicAdd(tab + 2 * (int64_t)r, a0);
        atomicAdd(tab + 2 * (int64_t)r + 1, a1);
    }
}

// Row layout of the stored activations and deltas (floats per Gaussian).
enum { R_DOUT = 0, R_H2 = 12, R_DH2 = R_H2 + NH, R_H1 = R_DH2 + NH, R_DH1 = R_H1 + NH, R_ENC = R_DH1 + NH,
       R_DE = R_ENC + ND, R_LEN = R_DE + ND };

struct Weights {
    float w1[NH][ND], b1[NH], w2[NH][NH], b2[NH], w3[NO][NH], b3[NO];
};

__device__ inline void load_weights(Weights &W, const float *w1, const float *b1, const float *w2, const float *b2,
                                    const float *w3, const float *b3, int din) {
    for (int i = threadIdx.x; i < NH * ND; i += blockDim.x) {
        int r = i / ND, c = i - r * ND;
        W.w1[r][c] = c < din ? w1[r * din + c] : 0.f;
    }
    for (int i = threadIdx.x; i < NH * NH; i += blockDim.x) W.w2[i / NH][i % NH] = w2[i];
    for (int i = threadIdx.x; i < NO * NH; i += blockDim.x) W.w3[i / NH][i % NH] = w3[i];
    for (int i = threadIdx.x; i < NH; i += blockDim.x) {
        W.b1[i] = b1[i];
        W.b2[i] = b2[i];
    }
    for (int i = threadIdx.x; i < NO; i += blockDim.x) W.b3[i] = b3[i];
}

// Encoding and MLP 2L -> 64 -> 64 -> 11.  Every level's two features go straight into the 64
// first-layer sums (the level loop stays rolled: its gathers are not all in flight at once),
// and every second-layer unit straight into the 11 outputs, so one 64-wide vector is live at a
// time.  With ROW, the encoding, h1 and h2 are also stored to the per-Gaussian row, with the
// ReLU masks.
template <bool ROW>
__device__ __forceinline__ void field(const NgpArgs &a, const float2 *tables, const Weights &W, const double *xn,
                                      float *o, float *row, uint64_t &m1, uint64_t &m2) {
    float h1[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) h1[j] = W.b1[j];
#pragma unroll 1
    for (int l = 0; l < a.levels; ++l) {
        float e0, e1;
        encode_level(a, tables, xn, l, e0, e1);
        if (ROW) {
            row[R_ENC + 2 * l] = e0;
            row[R_ENC + 2 * l + 1] = e1;
        }
#pragma unroll
        for (int j = 0; j < NH; ++j) h1[j] = __fmaf_rn(W.w1[j][2 * l + 1], e1, __fmaf_rn(W.w1[j][2 * l], e0, h1[j]));
    }
    if (ROW)
        for (int l = a.levels; l < NL; ++l) row[R_ENC + 2 * l] = row[R_ENC + 2 * l + 1] = 0.f;
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        float s = h1[j];
        h1[j] = s > 0.f ? s : 0.f;
        if (ROW) {
            row[R_H1 + j] = h1[j];
            m1 |= (s > 0.f ? 1ull : 0ull) << j;
        }
    }
#pragma unroll
    for (int k = 0; k < NO; ++k) o[k] = W.b3[k];
#pragma unroll 2
    for (int j = 0; j < NH; ++j) {
        float s = W.b2[j];
#pragma unroll
        for (int i = 0; i < NH; ++i) s = __fmaf_rn(W.w2[j][i], h1[i], s);
        float h = s > 0.f ? s : 0.f;
        if (ROW) {
            row[R_H2 + j] = h;
            m2 |= (s > 0.f ? 1ull : 0ull) << j;
        }
#pragma unroll
        for (int k = 0; k < NO; ++k) o[k] = __fmaf_rn(W.w3[k][j], h, o[k]);
    }
}

__device__ __forceinline__ float sigm(float x) { return 1.f / (1.f + __expf(-x)); }

__global__ __launch_bounds__(256, 2) void ngp_fwd_kernel(NgpArgs a, const float *mean, int64_t n, const float2 *tables,
                                                     const float *w1, const float *b1, const float *w2,
                                                     const float *b2, const float *w3, const float *b3,
                                                     float *quat, float *scale, float *opac, float *color) {
    __shared__ Weights W;
    load_weights(W, w1, b1, w2, b2, w3, b3, 2 * a.levels);
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double xn[3];
        normalise(a, mean, n, i, xn);
        float o[NO];
        uint64_t m1 = 0, m2 = 0;
        field<false>(a, tables, W, xn, o, nullptr, m1, m2);
#pragma unroll
        for (int c = 0; c < 3; ++c) color[c * n + i] = sigm(o[c]);
        opac[i] = sigm(o[3]);
#pragma unroll
        for (int c = 0; c < 3; ++c) scale[c * n + i] = a.scale_max * sigm(o[4 + c]);
        quat[i] = o[7] + 1.f;
#pragma unroll
        for (int c = 1; c < 4; ++c) quat[c * n + i] = o[7 + c];
    }
}

__global__ __launch_bounds__(256, 2) void ngp_bwd_kernel(NgpArgs a, const float *mean, int64_t n,
                                                        const float2 *tables, const float *w1, const float *b1,
                                                        const float *w2, const float *b2, const float *w3,
                                                        const float *b3, const float *dquat, const float *dscale,
                                                        const float *dopac, const float *dcolor, float *dtables,
                                                        float *rows) {
    __shared__ Weights W;
    load_weights(W, w1, b1, w2, b2, w3, b3, 2 * a.levels);
    __syncthreads();
    // every lane runs every iteration (the wave-level combining below needs all 64 lanes);
    // lanes past the end redo the last Gaussian and add nothing
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i0 = base + threadIdx.x;
        const bool live = i0 < n;
        const int64_t i = live ? i0 : n - 1;
        double xn[3];
        normalise(a, mean, n, i, xn);
        float *row = rows + (live ? i : n) * R_LEN;  // row n: scratch of the lanes past the end
        // forward again; activations go to the row store at once
        float o[NO];
        uint64_t m1 = 0, m2 = 0;  // ReLU masks of the two hidden layers
        field<true>(a, tables, W, xn, o, row, m1, m2);
        // heads
        float d[NO];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float s = sigm(o[c]);
            d[c] = dcolor[c * n + i] * s * (1.f - s);
        }
        {
            float s = sigm(o[3]);
            d[3] = dopac[i] * s * (1.f - s);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float s = sigm(o[4 + c]);
            d[4 + c] = dscale[c * n + i] * a.scale_max * s * (1.f - s);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) d[7 + c] = dquat[c * n + i];
        if (!live)
#pragma unroll
            for (int k = 0; k < NO; ++k) d[k] = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) row[R_DOUT + k] = k < NO ? d[k] : 0.f;
        // second hidden layer: each delta stored as soon as it is formed
#pragma unroll 4
        for (int j = 0; j < NH; ++j) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < NO; ++k) s = __fmaf_rn(W.w3[k][j], d[k], s);
            row[R_DH2 + j] = (m2 >> j) & 1ull ? s : 0.f;
        }
        // first hidden layer from the stored deltas (this thread's own row, cache resident); each
        // dh1[j] goes straight into the 2L encoding gradients
        float de[ND];
#pragma unroll
        for (int e = 0; e < ND; ++e) de[e] = 0.f;
        {
            float dh2[NH];
#pragma unroll
            for (int k = 0; k < NH; ++k) dh2[k] = row[R_DH2 + k];
#pragma unroll 2
            for (int j = 0; j < NH; ++j) {
                float s = 0.f;
#pragma unroll
                for (int k = 0; k < NH; ++k) s = __fmaf_rn(W.w2[k][j], dh2[k], s);
                float dh = (m1 >> j) & 1ull ? s : 0.f;
                row[R_DH1 + j] = dh;
#pragma unroll
                for (int e = 0; e < ND; ++e) de[e] = __fmaf_rn(W.w1[j][e], dh, de[e]);
            }
        }
#pragma unroll
        for (int e = 0; e < ND; ++e) row[R_DE + e] = de[e];
        // table adjoint, level by level
#pragma unroll 1
        for (int l = 0; l < a.levels; ++l) {
            float de0 = row[R_DE + 2 * l], de1 = row[R_DE + 2 * l + 1];
            uint32_t cell[3];
            double fr[3];
            level_cell(a, l, xn, cell, fr);
            float *tab = dtables + (int64_t)l * a.T * 2;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
                float w = (float)((cx ? fr[0] : 1.0 - fr[0]) * (cy ? fr[1] : 1.0 - fr[1]) * (cz ? fr[2] : 1.0 - fr[2]));
                uint32_t r = vertex_row(a, l, cell[0] + cx, cell[1] + cy, cell[2] + cz);
                scatter2(tab, r, w * de0, w * de1);
            }
        }
    }
}

// C[ma][nb] = sum_r A_r[i] B_r[j] and s[ma] = sum_r A_r[i] over the rows r of a chunk
// range, A_r = rows[r*R_LEN + aoff .. + ma), B_r = rows[r*R_LEN + boff .. + nb).
// Each workgroup sums its own range in registers and writes its partial.
constexpr int ATB_ROWS = 64;

__global__ __launch_bounds__(256) void atb_kernel(const float *rows, int64_t n, int aoff, int ma, int boff, int nb,
                                                 float *partial) {
    __shared__ float sa[ATB_ROWS][NH + 1], sb[ATB_ROWS][NH + 1];
    const int t = threadIdx.x;
    const int ne = ma * nb + ma;
    constexpr int KE = (NH * NH + NH + 255) / 256;
    float acc[KE];
#pragma unroll
    for (int k = 0; k < KE; ++k) acc[k] = 0.f;
    int64_t per = (n + gridDim.x - 1) / gridDim.x;
    int64_t r0 = (int64_t)blockIdx.x * per, r1 = r0 + per < n ? r0 + per : n;
    for (int64_t base = r0; base < r1; base += ATB_ROWS) {
        int cnt = (int)(r1 - base < ATB_ROWS ? r1 - base : ATB_ROWS);
        for (int i = t; i < ATB_ROWS * NH; i += 256) {
            int r = i / NH, c = i - r * NH;
            bool ok = r < cnt;
            sa[r][c] = ok && c < ma ? rows[(base + r) * R_LEN + aoff + c] : 0.f;
            sb[r][c] = ok && c < nb ? rows[(base + r) * R_LEN + boff + c] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KE; ++k) {
            int e = t + 256 * k;
            if (e >= ne) break;
            float s = acc[k];
            if (e < ma * nb) {
                int i = e / nb, j = e - i * nb;
#pragma unroll 8
                for (int r = 0; r < ATB_ROWS; ++r) s = __fmaf_rn(sa[r][i], sb[r][j], s);
            } else {
                int i = e - ma * nb;
#pragma unroll 8
                for (int r = 0; r < ATB_ROWS; ++r) s += sa[r][i];
            }
            acc[k] = s;
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < KE; ++k) {
        int e = t + 256 * k;
        if (e < ne) partial[(int64_t)blockIdx.x * ne + e] = acc[k];
    }
}

// out[e] += sum over workgroups of partial[g][e] (fixed order); e < ma*nb goes to dw, the rest to db
__global__ void atb_reduce_kernel(const float *partial, int ngroups, int ma, int nb, int din_w, float *dw,
                                  float *db) {
    int ne = ma * nb + ma;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int g = 0; g < ngroups; ++g) s += (double)partial[(int64_t)g * ne + e];
        if (e < ma * nb) {
            int i = e / nb, j = e - i * nb;
            if (j < din_w) dw[i * din_w + j] += (float)s;
        } else {
            db[e - ma * nb] += (float)s;
        }
    }
}

constexpr int ATB_GROUPS = 512;

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

}  // namespace

size_t ngp_ws_bytes(int64_t n) {
    return (size_t)(n + 1) * R_LEN * sizeof(float) + (size_t)ATB_GROUPS * (NH * NH + NH) * sizeof(float);  // rows + partials
}

int launch_ngp_fwd(const splat_ngp &m, const float *mean, int64_t n, float *quat, float *scale, float *opac,
                   float *color, hipStream_t st) {
    NgpArgs a;
    ngp_args(m, a);
    int64_t nb = (n + 255) / 256;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(ngp_fwd_kernel, dim3((unsigned)nb), dim3(256), 0, st, a, mean, n,
                       reinterpret_cast<const float2 *>(m.tables), m.w1, m.b1, m.w2, m.b2, m.w3, m.b3, quat, scale,
                       opac, color);
    return launch_status("ngp_fwd");
}

int launch_ngp_bwd(const splat_ngp &m, const float *mean, int64_t n, const float *dquat, const float *dscale,
                   const float *dopac, const float *dcolor, void *ws, float *dtables, float *dw1, float *db1,
                   float *dw2, float *db2, float *dw3, float *db3, hipStream_t st) {
    NgpArgs a;
    ngp_args(m, a);
    float *rows = static_cast<float *>(ws);
    float *partial = rows + (size_t)(n + 1) * R_LEN;
    int64_t nb = (n + 255) / 256;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(ngp_bwd_kernel, dim3((unsigned)nb), dim3(256), 0, st, a, mean, n,
                       reinterpret_cast<const float2 *>(m.tables), m.w1, m.b1, m.w2, m.b2, m.w3, m.b3, dquat, dscale,
                       dopac, dcolor, dtables, rows);
    int rc = launch_status("ngp_bwd");
    if (rc) return rc;
    int din = 2 * m.levels;
    struct Job { int aoff, ma, boff, nb, dinw; float *dw, *db; };
    Job jobs[3] = {{R_DOUT, NO, R_H2, NH, NH, dw3, db3}, {R_DH2, NH, R_H1, NH, NH, dw2, db2},
                   {R_DH1, NH, R_ENC, din, din, dw1, db1}};
    for (const Job &j : jobs) {
        hipLaunchKernelGGL(atb_kernel, dim3(ATB_GROUPS), dim3(256), 0, st, rows, n, j.aoff, j.ma, j.boff, j.nb,
                           partial);
        if ((rc = launch_status("ngp_atb"))) return rc;
        hipLaunchKernelGGL(atb_reduce_kernel, dim3(16), dim3(256), 0, st, partial, ATB_GROUPS, j.ma, j.nb, j.dinw,
                           j.dw, j.db);
        if ((rc = launch_status("ngp_atb_reduce"))) return rc;
    }
    return 0;
}

}  // namespace splat
