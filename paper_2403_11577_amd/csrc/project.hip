// project.hip -- EWA projection of the Gaussians into every view, and its adjoint.
//
// Paper Eq. (2) moves the means into the camera frame, Eq. (3) rotates the
// Gaussians (folded here into the covariance: with A = W R(q) diag(s) the
// camera-frame covariance is A A^T), and the splatting function Phi of Eq. (5)
// is EWA splatting: 2-D covariance J A A^T J^T + eps2d I under the perspective
// Jacobian J, its inverse (conic) and the screen-space mean.
//
// Layout: one thread per (view, Gaussian) candidate; SoA float32 parameter
// planes are read coalesced; the arithmetic is float64 (the projection is
// bandwidth bound, so the float64 rate costs nothing and removes the float32
// cancellation of thin, elongated footprints).  Visible pairs are compacted per
// view in Gaussian order by a count pass, a scan and a write pass that both
// call the same projection function.
#include "common.hpp"

namespace splat {
namespace {

enum { PC_OK = 0, PC_NEAR = 1, PC_FAR = 2, PC_OPAC = 4, PC_QUAT = 8, PC_OFF = 16, PC_NONFINITE = 32 };

struct Proj {
    float depth32;
    double t[3];
    double R[9];    // rotation of the unit quaternion
    double qh[4], qn;
    double A[9];    // W R diag(s)
    double J[6];
    bool clx, cly;
    double xh, yh;
    double T[6];    // J A
    double S2[3];   // xx, xy, yy (with eps2d)
    double Q[3];    // conic a, b, c
    double mu[2];
    int px0, px1, py0, py1;  // pixel rect (inclusive)
};

__device__ inline bool finite_f(float v) { return isfinite(v); }

// The geometric part of the projection of one Gaussian into one view (no
// culling): camera-frame mean, A = W R(q) diag(s), Jacobian with the guard
// clamp, 2-D covariance, conic and screen mean.
__device__ inline void project_core(const splat_settings &S, const double *M, const double *K4, int W, int H,
                                    const float *x, const float *q, const float *s, Proj &P) {
    double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
    double n2 = qw * qw + qx * qx + qy * qy + qz * qz;
    P.qn = sqrt(n2);
    qw /= P.qn; qx /= P.qn; qy /= P.qn; qz /= P.qn;
    P.qh[0] = qw; P.qh[1] = qx; P.qh[2] = qy; P.qh[3] = qz;
    double *R = P.R;
    R[0] = 1.0 - 2.0 * (qy * qy + qz * qz); R[1] = 2.0 * (qx * qy - qw * qz); R[2] = 2.0 * (qx * qz + qw * qy);
    R[3] = 2.0 * (qx * qy + qw * qz); R[4] = 1.0 - 2.0 * (qx * qx + qz * qz); R[5] = 2.0 * (qy * qz - qw * qx);
    R[6] = 2.0 * (qx * qz - qw * qy); R[7] = 2.0 * (qy * qz + qw * qx); R[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
    double xd[3] = {x[0], x[1], x[2]};
    for (int i = 0; i < 3; ++i) P.t[i] = M[4 * i] * xd[0] + M[4 * i + 1] * xd[1] + M[4 * i + 2] * xd[2] + M[4 * i + 3];
    // A = W R diag(s)
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            P.A[3 * i + j] = (M[4 * i] * R[j] + M[4 * i + 1] * R[3 + j] + M[4 * i + 2] * R[6 + j]) * (double)s[j];
    double fx = K4[0], fy = K4[1], cx = K4[2], cy = K4[3];
    double tz = P.t[2];
    double ux = P.t[0] / tz, uy = P.t[1] / tz;
    double gx0 = (-cx - S.guard * W) / fx, gx1 = (W - cx + S.guard * W) / fx;
    double gy0 = (-cy - S.guard * H) / fy, gy1 = (H - cy + S.guard * H) / fy;
    P.clx = (ux < gx0) || (ux > gx1);
    P.cly = (uy < gy0) || (uy > gy1);
    P.xh = fmin(fmax(ux, gx0), gx1);
    P.yh = fmin(fmax(uy, gy0), gy1);
    double *J = P.J;
    J[0] = fx / tz; J[1] = 0.0; J[2] = -fx * P.xh / tz;
    J[3] = 0.0; J[4] = fy / tz; J[5] = -fy * P.yh / tz;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            P.T[3 * i + j] = J[3 * i] * P.A[j] + J[3 * i + 1] * P.A[3 + j] + J[3 * i + 2] * P.A[6 + j];
    double sxx = P.T[0] * P.T[0] + P.T[1] * P.T[1] + P.T[2] * P.T[2] + S.eps2d;
    double sxy = P.T[0] * P.T[3] + P.T[1] * P.T[4] + P.T[2] * P.T[5];
    double syy = P.T[3] * P.T[3] + P.T[4] * P.T[4] + P.T[5] * P.T[5] + S.eps2d;
    P.S2[0] = sxx; P.S2[1] = sxy; P.S2[2] = syy;
    double idet = 1.0 / (sxx * syy - sxy * sxy);
    P.Q[0] = syy * idet; P.Q[1] = -sxy * idet; P.Q[2] = sxx * idet;
    P.mu[0] = fx * ux + cx;
    P.mu[1] = fy * uy + cy;
}

// The projection of one Gaussian into one view.  Returns a cull code (0 = visible).
__device__ int project_gauss(const splat_settings &S, const double *M, const double *K4, int W, int H,
                             const float *x, const float *q, const float *s, float o, Proj &P) {
    if (!(finite_f(x[0]) && finite_f(x[1]) && finite_f(x[2]) && finite_f(q[0]) && finite_f(q[1]) &&
          finite_f(q[2]) && finite_f(q[3]) && finite_f(s[0]) && finite_f(s[1]) && finite_f(s[2]) &&
          finite_f(o)))
        return PC_NONFINITE;
    // float32 depth key: fma chain on float32-rounded row 2 of W2C
    P.depth32 = __fmaf_rn((float)M[8], x[0], __fmaf_rn((float)M[9], x[1], __fmaf_rn((float)M[10], x[2], (float)M[11])));
    if (!(P.depth32 > (float)S.near_z)) return PC_NEAR;
    if (P.depth32 > (float)S.far_z) return PC_FAR;
    if ((double)o < S.alpha_min) return PC_OPAC;
    {
        double n2 = (double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3];
        if (!(n2 >= 1e-24)) return PC_QUAT;
    }
    project_core(S, M, K4, W, H, x, q, s, P);
    double sxx = P.S2[0], syy = P.S2[2];
    double k2 = fmax(2.0 * log((double)o / S.alpha_min), 0.0);
    double ex = sqrt(k2 * sxx) * (1.0 + S.pad_rel) + S.pad_px;
    double ey = sqrt(k2 * syy) * (1.0 + S.pad_rel) + S.pad_px;
    double a0 = ceil(P.mu[0] - 0.5 - ex), a1 = floor(P.mu[0] - 0.5 + ex);
    double b0 = ceil(P.mu[1] - 0.5 - ey), b1 = floor(P.mu[1] - 0.5 + ey);
    a0 = fmax(a0, 0.0); b0 = fmax(b0, 0.0);
    a1 = fmin(a1, (double)(W - 1)); b1 = fmin(b1, (double)(H - 1));
    if (!(a0 <= a1) || !(b0 <= b1)) return PC_OFF;
    P.px0 = (int)a0; P.px1 = (int)a1; P.py0 = (int)b0; P.py1 = (int)b1;
    return PC_OK;
}

__device__ inline void load_gauss(const splat_gaussians &g, int64_t i, float *x, float *q, float *s, float &o) {
    int64_t n = g.n;
    x[0] = g.mean[i]; x[1] = g.mean[n + i]; x[2] = g.mean[2 * n + i];
    q[0] = g.quat[i]; q[1] = g.quat[n + i]; q[2] = g.quat[2 * n + i]; q[3] = g.quat[3 * n + i];
    s[0] = g.scale[i]; s[1] = g.scale[n + i]; s[2] = g.scale[2 * n + i];
    o = g.opacity[i];
}

__device__ inline void flag_status(uint32_t *status, int code) {
    uint32_t bits = (code == PC_NONFINITE ? SPLAT_ST_NONFINITE : 0u) | (code == PC_QUAT ? SPLAT_ST_DEGENERATE : 0u);
    uint64_t any = __ballot(bits != 0);
    if (any) {
        // reduce the bits over the wave, then one atomic
        uint32_t b = bits;
        for (int o = 32; o > 0; o >>= 1) b |= __shfl_xor(b, o, kWave);
        if (__lane_id() == (int)(__ffsll((long long)any) - 1)) atomicOr(status, b);
    }
}

// block-level exclusive rank of `vis` (256 threads = 4 waves); returns the block total via *tot
__device__ inline uint32_t block_rank(bool vis, uint32_t *lds4, uint32_t *tot) {
    uint64_t m = __ballot(vis);
    int w = threadIdx.x >> 6;
    if (__lane_id() == 0) lds4[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t base = 0, total = 0;
    for (int i = 0; i < 4; ++i) {
        uint32_t c = lds4[i];
        if (i < w) base += c;
        total += c;
    }
    *tot = total;
    return base + rank_in(m);
}

__global__ __launch_bounds__(256) void project_count_kernel(splat_settings S, splat_gaussians g, const double *w2c,
                                                           const double *intr, int W, int H, int nb,
                                                           uint32_t *blockcnt, uint64_t *visbits, uint32_t *status) {
    __shared__ uint32_t lds4[4];
    int v = blockIdx.y;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int code = PC_OFF;
    if (i < g.n) {
        float x[3], q[4], s[3], o;
        load_gauss(g, i, x, q, s, o);
        Proj P;
        code = project_gauss(S, w2c + 12 * v, intr + 4 * v, W, H, x, q, s, o, P);
    }
    flag_status(status, code);
    uint64_t m = __ballot(code == PC_OK);
    if (__lane_id() == 0) visbits[((size_t)v * nb + blockIdx.x) * 4 + (threadIdx.x >> 6)] = m;
    uint32_t tot;
    block_rank(code == PC_OK, lds4, &tot);
    if (threadIdx.x == 0) blockcnt[(size_t)v * nb + blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void project_write_kernel(splat_settings S, splat_gaussians g, const double *w2c,
                                                           const double *intr, int W, int H, int nb,
                                                           const uint32_t *blockoff, int64_t slot_cap,
                                                           float4 *rec, int2 *meta, Rect16 *rect,
                                                           uint32_t *ntiles) {
    __shared__ uint32_t lds4[4];
    int v = blockIdx.y;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int code = PC_OFF;
    Proj P;
    float x[3], q[4], s[3], o = 0.f;
    if (i < g.n) {
        load_gauss(g, i, x, q, s, o);
        code = project_gauss(S, w2c + 12 * v, intr + 4 * v, W, H, x, q, s, o, P);
    }
    uint32_t tot;
    uint32_t r = block_rank(code == PC_OK, lds4, &tot);
    if (code != PC_OK) return;
    uint64_t slot = (uint64_t)blockoff[(size_t)v * nb + blockIdx.x] + r;
    if (slot >= (uint64_t)slot_cap) return;  // capacity flagged by the scan finisher
    float mxh = (float)P.mu[0], myh = (float)P.mu[1];
    float mxl = (float)(P.mu[0] - (double)mxh), myl = (float)(P.mu[1] - (double)myh);
    int64_t n = g.n;
    rec[3 * slot + 0] = make_float4(mxh, myh, mxl, myl);
    rec[3 * slot + 1] = make_float4((float)P.Q[0], (float)P.Q[1], (float)P.Q[2], o);
    rec[3 * slot + 2] = make_float4(g.color[i], g.color[n + i], g.color[2 * n + i], P.depth32);
    meta[slot] = make_int2((int)i, v);
    int tw = S.tile_w, th = S.tile_h;
    Rect16 rc;
    rc.x0 = (uint16_t)(P.px0 / tw); rc.x1 = (uint16_t)(P.px1 / tw);
    rc.y0 = (uint16_t)(P.py0 / th); rc.y1 = (uint16_t)(P.py1 / th);
    rect[slot] = rc;
    ntiles[slot] = (uint32_t)(rc.x1 - rc.x0 + 1) * (uint32_t)(rc.y1 - rc.y0 + 1);
}

// totals after the block-count scan: slot count (clamped), view offsets, capacity flag
__global__ void project_finish_kernel(const uint32_t *blockoff, int V, int nb, int64_t slot_cap,
                                      uint32_t *counts, uint32_t *view_off, uint32_t *status) {
    int v = threadIdx.x;
    uint32_t total = blockoff[(size_t)V * nb];
    uint32_t cap = (uint32_t)slot_cap;
    if (v <= V) {
        uint32_t off = (v < V) ? blockoff[(size_t)v * nb] : total;
        view_off[v] = off < cap ? off : cap;
    }
    if (v == 0) {
        counts[CNT_SLOTS] = total < cap ? total : cap;
        if (total > cap) atomicOr(status, SPLAT_ST_CAPACITY);
    }
}

// ----------------------------------------------------------------------------------
// adjoint
// ----------------------------------------------------------------------------------
// Chain rule of one visible (view, Gaussian) pair from its slot gradient gd[9]
// = d(mu x, mu y; conic a, b, c; opacity; r, g, b).  Adds the quaternion, scale
// and mean gradients to gq, gs, gm and returns the W2C gradient in gw[12].
__device__ void slot_adjoint(const Proj &P, const double *M, const double *K4, const float *x, const float *s,
                             const float *gd, double *gq, double *gs, double *gm, double *gw) {
    double gmx = gd[0], gmy = gd[1], ga = gd[2], gb = gd[3], gc = gd[4];
    // conic -> Sigma2: G2 = -Q GQ Q with GQ = [[ga, gb/2], [gb/2, gc]]
    double a = P.Q[0], b = P.Q[1], c = P.Q[2];
    double hb = 0.5 * gb;
    double m00 = a * ga + b * hb, m01 = a * hb + b * gc;
    double m10 = b * ga + c * hb, m11 = b * hb + c * gc;
    double g2xx = -(m00 * a + m01 * b);
    double g2xy = -(m00 * b + m01 * c);
    double g2yy = -(m10 * b + m11 * c);
    // Sigma2 = T T^T + eps I -> dT = 2 G2 T
    double gT[6];
    for (int j = 0; j < 3; ++j) {
        gT[j] = 2.0 * (g2xx * P.T[j] + g2xy * P.T[3 + j]);
        gT[3 + j] = 2.0 * (g2xy * P.T[j] + g2yy * P.T[3 + j]);
    }
    // T = J A -> dJ = gT A^T, dA = J^T gT
    double gJ[6], gA[9];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k)
            gJ[3 * r + k] = gT[3 * r] * P.A[3 * k] + gT[3 * r + 1] * P.A[3 * k + 1] + gT[3 * r + 2] * P.A[3 * k + 2];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) gA[3 * r + k] = P.J[r] * gT[k] + P.J[3 + r] * gT[3 + k];
    // J(t), mu(t)
    double fx = K4[0], fy = K4[1];
    double tx = P.t[0], ty = P.t[1], tz = P.t[2];
    double iz = 1.0 / tz, iz2 = iz * iz;
    double gt0 = gmx * fx * iz, gt1 = gmy * fy * iz;
    double gt2 = -(gmx * fx * tx + gmy * fy * ty) * iz2 - (gJ[0] * fx + gJ[4] * fy) * iz2;
    if (!P.clx) {
        gt0 += -gJ[2] * fx * iz2;
        gt2 += 2.0 * gJ[2] * fx * tx * iz2 * iz;
    } else {
        gt2 += gJ[2] * fx * P.xh * iz2;
    }
    if (!P.cly) {
        gt1 += -gJ[5] * fy * iz2;
        gt2 += 2.0 * gJ[5] * fy * ty * iz2 * iz;
    } else {
        gt2 += gJ[5] * fy * P.yh * iz2;
    }
    double gt[3] = {gt0, gt1, gt2};
    // A = W R D: dW += gA (R D)^T ; dR = W^T gA D ; ds_k = ((W R)^T gA)_kk
    double gR[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int m = 0; m < 3; ++m) acc += M[4 * m + r] * gA[3 * m + k];  // (W^T gA)[r][k]
            gR[3 * r + k] = acc * (double)s[k];
            gs[k] += P.R[3 * r + k] * acc;  // ((W R)^T gA)_kk = sum_r R[r][k] (W^T gA)[r][k]
        }
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int m = 0; m < 3; ++m) acc += gA[3 * r + m] * P.R[3 * k + m] * (double)s[m];
            gw[4 * r + k] = acc + gt[r] * (double)x[k];
        }
    for (int r = 0; r < 3; ++r) gw[4 * r + 3] = gt[r];
    for (int k = 0; k < 3; ++k) gm[k] += M[k] * gt[0] + M[4 + k] * gt[1] + M[8 + k] * gt[2];
    // R(q_hat) -> q_hat -> q
    double w = P.qh[0], qx = P.qh[1], qy = P.qh[2], qz = P.qh[3];
    double gq0 = 2.0 * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
    double gq1 = 2.0 * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2.0 * qx * gR[4] - w * gR[5] + qz * gR[6] + w * gR[7] - 2.0 * qx * gR[8]);
    double gq2 = 2.0 * (-2.0 * qy * gR[0] + qx * gR[1] + w * gR[2] + qx * gR[3] + qz * gR[5] - w * gR[6] + qz * gR[7] - 2.0 * qy * gR[8]);
    double gq3 = 2.0 * (-2.0 * qz * gR[0] - w * gR[1] + qx * gR[2] + w * gR[3] - 2.0 * qz * gR[4] + qy * gR[5] + qx * gR[6] + qy * gR[7]);
    double dot = w * gq0 + qx * gq1 + qy * gq2 + qz * gq3;
    double iq = 1.0 / P.qn;
    gq[0] += (gq0 - w * dot) * iq;
    gq[1] += (gq1 - qx * dot) * iq;
    gq[2] += (gq2 - qy * dot) * iq;
    gq[3] += (gq3 - qz * dot) * iq;
}

// Transposed FP64 reduction of twelve per-lane values over the wave: four
// exchange steps inside each 16-lane row with partners lane^1, lane^2, lane^7 and
// lane^15 (DPP moves of both halves), then two cross-row exchanges.  Lane i ends
// with the wave total of value number cls(i) = c0 + 2 c1 + 4 c2 + 8 c3, where
// c0 = b0^b2, c1 = b1^b2, c2 = b2^b3, c3 = b3 for the bits b of i & 15 (numbers
// 12..15 carry padding).  About 80 VALU operations instead of twelve separate
// shuffle reductions.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ double xpair_d(double lo, double hi, bool c) {
    double keep = c ? hi : lo, send = c ? lo : hi;
    return keep + dpp_d<CTRL>(send);
}

template <int CTRL>
__device__ __forceinline__ double xpad_d(double v) { return v + dpp_d<CTRL>(v); }

__device__ inline double reduce12(const double (&v)[12], bool c0, bool c1, bool c2, bool c3) {
    double a0 = xpair_d<0xB1>(v[0], v[1], c0), a1 = xpair_d<0xB1>(v[2], v[3], c0);
    double a2 = xpair_d<0xB1>(v[4], v[5], c0), a3 = xpair_d<0xB1>(v[6], v[7], c0);
    double a4 = xpair_d<0xB1>(v[8], v[9], c0), a5 = xpair_d<0xB1>(v[10], v[11], c0);
    double b0 = xpair_d<0x4E>(a0, a1, c1), b1 = xpair_d<0x4E>(a2, a3, c1), b2 = xpair_d<0x4E>(a4, a5, c1);
    double d0 = xpair_d<0x141>(b0, b1, c2), d1 = xpad_d<0x141>(b2);
    double e = xpair_d<0x140>(d0, d1, c3);
    e += __shfl_xor(e, 16, kWave);
    e += __shfl_xor(e, 32, kWave);
    return e;
}

struct LaneClass {
    bool c0, c1, c2, c3;
    int cls;
    __device__ explicit LaneClass(int lane) {
        int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
        c0 = b0 ^ b2; c1 = b1 ^ b2; c2 = b2 ^ b3; c3 = b3;
        cls = (int)c0 | ((int)c1 << 1) | ((int)c2 << 2) | ((int)c3 << 3);
    }
};

// One thread per Gaussian walks every view; the visibility mask written by the
// count pass and the per-block slot offsets give the slot of each visible pair
// (slots are compacted per view in Gaussian order), so the per-Gaussian
// gradients are summed in float64 registers and written once, without atomics.
// The W2C gradient of each view is reduced over the workgroup in float64 and
// stored as the workgroup's partial; dw2c_reduce_kernel sums the partials of a
// view in a fixed order (deterministic, no contended float64 atomics).
__global__ __launch_bounds__(256) void project_bwd_kernel(splat_settings S, splat_gaussians g, const double *w2c,
                                                         const double *intr, int W, int H, int V, int nb,
                                                         const uint32_t *blockoff, const uint64_t *visbits,
                                                         int64_t slot_cap, const float *grad2d, float *dquat,
                                                         float *dscale, float *dopac, float *dcolor, float *dmean,
                                                         double *dwpart) {
    __shared__ double red[4][12];
    const int b = blockIdx.x, wv = threadIdx.x >> 6, lane = __lane_id();
    const LaneClass lc(lane);
    const bool writer = lane < 16 && lc.cls < 12;
    const int64_t i = (int64_t)b * 256 + threadIdx.x;
    const int64_t n = g.n;
    const bool live = i < n;
    float x[3] = {0.f, 0.f, 0.f}, q[4] = {1.f, 0.f, 0.f, 0.f}, s[3] = {1.f, 1.f, 1.f}, o = 1.f;
    if (live) load_gauss(g, i, x, q, s, o);
    double gq[4] = {0, 0, 0, 0}, gs[3] = {0, 0, 0}, gm[3] = {0, 0, 0}, go = 0.0, gc[3] = {0, 0, 0};
    for (int v = 0; v < V; ++v) {
        const uint64_t *vb = visbits + ((size_t)v * nb + b) * 4;
        double *part = dwpart + ((size_t)v * nb + b) * 12;
        uint64_t mask = vb[wv];
        bool vis = live && ((mask >> lane) & 1ull);
        if (!__syncthreads_or(vis)) {  // nothing of this workgroup visible in view v
            if (threadIdx.x < 12) part[threadIdx.x] = 0.0;
            continue;
        }
        double gw[12];
        for (int k = 0; k < 12; ++k) gw[k] = 0.0;
        if (vis) {
            uint32_t before = 0;
            for (int w2 = 0; w2 < wv; ++w2) before += (uint32_t)__popcll(vb[w2]);
            uint64_t slot = (uint64_t)blockoff[(size_t)v * nb + b] + before + rank_in(mask);
            if (slot < (uint64_t)slot_cap) {
                const double *M = w2c + 12 * v;
                const double *K4 = intr + 4 * v;
                Proj P;
                project_core(S, M, K4, W, H, x, q, s, P);
                const float *gd = grad2d + 9 * slot;
                go += gd[5];
                gc[0] += gd[6];
                gc[1] += gd[7];
                gc[2] += gd[8];
                slot_adjoint(P, M, K4, x, s, gd, gq, gs, gm, gw);
            }
        }
        double tot = 0.0;
        if (mask != 0ull) tot = reduce12(gw, lc.c0, lc.c1, lc.c2, lc.c3);  // wave-uniform
        if (writer) red[wv][lc.cls] = tot;
        __syncthreads();
        if (threadIdx.x < 12) {
            int k = threadIdx.x;
            part[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
        }
        __syncthreads();
    }
    if (!live) return;
    for (int k = 0; k < 4; ++k) dquat[k * n + i] += (float)gq[k];
    for (int k = 0; k < 3; ++k) dscale[k * n + i] += (float)gs[k];
    dopac[i] += (float)go;
    for (int k = 0; k < 3; ++k) dcolor[k * n + i] += (float)gc[k];
    if (dmean)
        for (int k = 0; k < 3; ++k) dmean[k * n + i] += (float)gm[k];
}

// dw2c[v] += sum over the workgroups of their partials, in a fixed order.
__global__ __launch_bounds__(256) void dw2c_reduce_kernel(const double *dwpart, int nb, double *dw2c) {
    __shared__ double red[4][12];
    const int v = blockIdx.x, wv = threadIdx.x >> 6, lane = __lane_id();
    const LaneClass lc(lane);
    double acc[12];
    for (int k = 0; k < 12; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        const double *p = dwpart + ((size_t)v * nb + b) * 12;
        for (int k = 0; k < 12; ++k) acc[k] += p[k];
    }
    double tot = reduce12(acc, lc.c0, lc.c1, lc.c2, lc.c3);
    if (lane < 16 && lc.cls < 12) red[wv][lc.cls] = tot;
    __syncthreads();
    if (threadIdx.x < 12) {
        int k = threadIdx.x;
        dw2c[12 * v + k] += ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

}  // namespace

int launch_project(const splat_plan &p, void *ws, const splat_gaussians &g, const double *w2c,
                   const double *intr, hipStream_t st) {
    int V = p.n_views, nb = p.n_blocks_proj;
    uint32_t *status = ws_at<uint32_t>(ws, p.off_status);
    uint32_t *counts = ws_at<uint32_t>(ws, p.off_counts);
    uint32_t *blockcnt = ws_at<uint32_t>(ws, p.off_blockcnt);
    if (g.n == 0) {
        int rc = launch_fill_u32(blockcnt, 0u, (int64_t)V * nb + 1, st);
        if (rc) return rc;
    } else {
        hipLaunchKernelGGL(project_count_kernel, dim3(nb, V), dim3(256), 0, st, p.s, g, w2c, intr, p.width,
                           p.height, nb, blockcnt, ws_at<uint64_t>(ws, p.off_visbits), status);
        int rc = launch_status("project_count");
        if (rc) return rc;
        rc = launch_scan_u32(blockcnt, blockcnt, nullptr, (int64_t)V * nb, ws_at<uint32_t>(ws, p.off_scan),
                             nullptr, st);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(project_finish_kernel, dim3(1), dim3(((V + 1 + 63) / 64) * 64), 0, st, blockcnt, V, nb,
                       p.slot_cap, counts, ws_at<uint32_t>(ws, p.off_view_off), status);
    int rc = launch_status("project_finish");
    if (rc || g.n == 0) return rc;
    hipLaunchKernelGGL(project_write_kernel, dim3(nb, V), dim3(256), 0, st, p.s, g, w2c, intr, p.width, p.height,
                       nb, blockcnt, p.slot_cap, ws_at<float4>(ws, p.off_rec), ws_at<int2>(ws, p.off_meta),
                       ws_at<Rect16>(ws, p.off_rect), ws_at<uint32_t>(ws, p.off_ntiles));
    return launch_status("project_write");
}

int launch_project_bwd(const splat_plan &p, void *ws, const splat_gaussians &g, const double *w2c,
                       const double *intr, float *dquat, float *dscale, float *dopac, float *dcolor,
                       float *dmean, double *dw2c, hipStream_t st) {
    if (g.n == 0) return 0;
    int nb = p.n_blocks_proj;
    double *part = ws_at<double>(ws, p.off_dwpart);
    hipLaunchKernelGGL(project_bwd_kernel, dim3(nb), dim3(256), 0, st, p.s, g, w2c, intr, p.width, p.height,
                       p.n_views, nb, ws_at<uint32_t>(ws, p.off_blockcnt), ws_at<uint64_t>(ws, p.off_visbits),
                       p.slot_cap, ws_at<float>(ws, p.off_grad2d), dquat, dscale, dopac, dcolor, dmean, part);
    int rc = launch_status("project_bwd");
    if (rc) return rc;
    hipLaunchKernelGGL(dw2c_reduce_kernel, dim3(p.n_views), dim3(256), 0, st, part, nb, dw2c);
    return launch_status("dw2c_reduce");
}

}  // namespace splat
