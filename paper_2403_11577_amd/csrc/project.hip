// project.hip -- EWA projection of the Gaussians into every view, and its adjoint.
//
// Paper Eq. (2) moves the means into the camera frame, Eq. (3) rotates the
// Gaussians (folded here into the covariance: with A = W R(q) diag(s) the
// camera-frame covariance is A A^T), and the splatting function Phi of Eq. (5)
// is EWA splatting: 2-D covariance J A A^T J^T + eps2d I under the perspective
// Jacobian J, its inverse (conic) and the screen-space mean.
//
// Layout: one thread per Gaussian, walking every view, so its view-independent
// part (rotation, footprint radius) is formed once; SoA float32 parameter planes
// are read coalesced.  The arithmetic is float64: on this chip the float64 vector
// rate equals the unpacked float32 rate, and float64 removes the float32
// cancellation of thin, elongated footprints (a float32 pre-cull rejects most
// invisible pairs first).  Visible pairs are compacted per view in Gaussian order
// by a count pass, a scan and a write pass that both call the same projection
// function.
#include "common.hpp"

namespace splat {
namespace {

enum { PC_OK = 0, PC_NEAR = 1, PC_FAR = 2, PC_OPAC = 4, PC_QUAT = 8, PC_OFF = 16, PC_NONFINITE = 32 };

// View-independent part of a Gaussian: unit quaternion, its rotation and the
// squared footprint radius k^2 = 2 ln(o / alpha_min) (clamped at 0).
struct GaussPre {
    double qh[4], qn, R[9], k2;
};

// Per-view camera constants: focal lengths, principal point and the clamp bounds
// of the Jacobian's x/z, y/z ratios; then float32 copies of the world-to-camera matrix and
// of those constants for the cull bounds and the depth key (converted once per view instead
// of once per (Gaussian, view) pair).
struct CamC {
    double fx, fy, cx, cy, gx0, gx1, gy0, gy1;
    float m[12];
    float fxf, fyf, cxf, cyf, gx0f, gx1f, gy0f, gy1f;
};
static_assert(sizeof(CamC) == kCamBytes, "camera constants");

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

__device__ inline void gauss_pre(const splat_settings &S, const float *q, float o, GaussPre &G) {
    double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
    double n2 = qw * qw + qx * qx + qy * qy + qz * qz;
    G.qn = sqrt(n2);
    qw /= G.qn; qx /= G.qn; qy /= G.qn; qz /= G.qn;
    G.qh[0] = qw; G.qh[1] = qx; G.qh[2] = qy; G.qh[3] = qz;
    double *R = G.R;
    R[0] = 1.0 - 2.0 * (qy * qy + qz * qz); R[1] = 2.0 * (qx * qy - qw * qz); R[2] = 2.0 * (qx * qz + qw * qy);
    R[3] = 2.0 * (qx * qy + qw * qz); R[4] = 1.0 - 2.0 * (qx * qx + qz * qz); R[5] = 2.0 * (qy * qz - qw * qx);
    R[6] = 2.0 * (qx * qz - qw * qy); R[7] = 2.0 * (qy * qz + qw * qx); R[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
    G.k2 = fmax(2.0 * log((double)o / S.alpha_min), 0.0);
}

__global__ void camconst_kernel(splat_settings S, const double *intr, const double *w2c, int V, int W, int H,
                                CamC *cam) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const double *K4 = intr + 4 * v;
    CamC c;
    c.fx = K4[0]; c.fy = K4[1]; c.cx = K4[2]; c.cy = K4[3];
    c.gx0 = (-c.cx - S.guard * W) / c.fx; c.gx1 = (W - c.cx + S.guard * W) / c.fx;
    c.gy0 = (-c.cy - S.guard * H) / c.fy; c.gy1 = (H - c.cy + S.guard * H) / c.fy;
    for (int k = 0; k < 12; ++k) c.m[k] = (float)w2c[12 * v + k];
    c.fxf = (float)c.fx; c.fyf = (float)c.fy; c.cxf = (float)c.cx; c.cyf = (float)c.cy;
    c.gx0f = (float)c.gx0; c.gx1f = (float)c.gx1; c.gy0f = (float)c.gy0; c.gy1f = (float)c.gy1;
    cam[v] = c;
}

// The geometric part of the projection of one Gaussian into one view (no
// culling): camera-frame mean, A = W R(q) diag(s), Jacobian with the guard
// clamp, 2-D covariance, conic (if asked) and screen mean.
__device__ inline void project_view(const splat_settings &S, const double *M, const CamC &C, const float *x,
                                    const float *s, const GaussPre &G, bool conic, Proj &P) {
    for (int k = 0; k < 9; ++k) P.R[k] = G.R[k];
    for (int k = 0; k < 4; ++k) P.qh[k] = G.qh[k];
    P.qn = G.qn;
    const double *R = G.R;
    double xd[3] = {x[0], x[1], x[2]};
    for (int i = 0; i < 3; ++i) P.t[i] = M[4 * i] * xd[0] + M[4 * i + 1] * xd[1] + M[4 * i + 2] * xd[2] + M[4 * i + 3];
    // A = W R diag(s)
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            P.A[3 * i + j] = (M[4 * i] * R[j] + M[4 * i + 1] * R[3 + j] + M[4 * i + 2] * R[6 + j]) * (double)s[j];
    double tz = P.t[2];
    double ux = P.t[0] / tz, uy = P.t[1] / tz;
    P.clx = (ux < C.gx0) || (ux > C.gx1);
    P.cly = (uy < C.gy0) || (uy > C.gy1);
    P.xh = fmin(fmax(ux, C.gx0), C.gx1);
    P.yh = fmin(fmax(uy, C.gy0), C.gy1);
    double *J = P.J;
    J[0] = C.fx / tz; J[1] = 0.0; J[2] = -C.fx * P.xh / tz;
    J[3] = 0.0; J[4] = C.fy / tz; J[5] = -C.fy * P.yh / tz;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            P.T[3 * i + j] = J[3 * i] * P.A[j] + J[3 * i + 1] * P.A[3 + j] + J[3 * i + 2] * P.A[6 + j];
    double sxx = P.T[0] * P.T[0] + P.T[1] * P.T[1] + P.T[2] * P.T[2] + S.eps2d;
    double sxy = P.T[0] * P.T[3] + P.T[1] * P.T[4] + P.T[2] * P.T[5];
    double syy = P.T[3] * P.T[3] + P.T[4] * P.T[4] + P.T[5] * P.T[5] + S.eps2d;
    P.S2[0] = sxx; P.S2[1] = sxy; P.S2[2] = syy;
    if (conic) {
        double idet = 1.0 / (sxx * syy - sxy * sxy);
        P.Q[0] = syy * idet; P.Q[1] = -sxy * idet; P.Q[2] = sxx * idet;
    }
    P.mu[0] = C.fx * ux + C.cx;
    P.mu[1] = C.fy * uy + C.cy;
}

// project_view with the conic, as the adjoint needs it: the clamp decisions are taken as the
// forward takes them (x/z and y/z by division), the Jacobian's entries by one reciprocal of the
// depth (returned in iz); R, qh and the screen mean are not copied or formed.
__device__ inline void project_view_adj(const splat_settings &S, const double *M, const CamC &C, const float *x,
                                        const float *s, const GaussPre &G, Proj &P, double &iz) {
    const double *R = G.R;
    double xd[3] = {x[0], x[1], x[2]};
    for (int i = 0; i < 3; ++i) P.t[i] = M[4 * i] * xd[0] + M[4 * i + 1] * xd[1] + M[4 * i + 2] * xd[2] + M[4 * i + 3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            P.A[3 * i + j] = (M[4 * i] * R[j] + M[4 * i + 1] * R[3 + j] + M[4 * i + 2] * R[6 + j]) * (double)s[j];
    const double tz = P.t[2];
    const double ux = P.t[0] / tz, uy = P.t[1] / tz;
    P.clx = (ux < C.gx0) || (ux > C.gx1);
    P.cly = (uy < C.gy0) || (uy > C.gy1);
    P.xh = fmin(fmax(ux, C.gx0), C.gx1);
    P.yh = fmin(fmax(uy, C.gy0), C.gy1);
    iz = 1.0 / tz;
    double *J = P.J;
    J[0] = C.fx * iz; J[1] = 0.0; J[2] = -C.fx * P.xh * iz;
    J[3] = 0.0; J[4] = C.fy * iz; J[5] = -C.fy * P.yh * iz;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            P.T[3 * i + j] = J[3 * i] * P.A[j] + J[3 * i + 1] * P.A[3 + j] + J[3 * i + 2] * P.A[6 + j];
    const double sxx = P.T[0] * P.T[0] + P.T[1] * P.T[1] + P.T[2] * P.T[2] + S.eps2d;
    const double sxy = P.T[0] * P.T[3] + P.T[1] * P.T[4] + P.T[2] * P.T[5];
    const double syy = P.T[3] * P.T[3] + P.T[4] * P.T[4] + P.T[5] * P.T[5] + S.eps2d;
    const double idet = 1.0 / (sxx * syy - sxy * sxy);
    P.Q[0] = syy * idet; P.Q[1] = -sxy * idet; P.Q[2] = sxx * idet;
}

// Pixel rectangle of the alpha >= alpha_min footprint (exact AABB of the ellipse,
// padded) inside the rendered rows; PC_OFF if it misses them.
__device__ inline int footprint(const splat_settings &S, double k2, int W, int H, Proj &P) {
    double ex = sqrt(k2 * P.S2[0]) * (1.0 + S.pad_rel) + S.pad_px;
    double ey = sqrt(k2 * P.S2[2]) * (1.0 + S.pad_rel) + S.pad_px;
    double a0 = ceil(P.mu[0] - 0.5 - ex), a1 = floor(P.mu[0] - 0.5 + ex);
    double b0 = ceil(P.mu[1] - 0.5 - ey), b1 = floor(P.mu[1] - 0.5 + ey);
    a0 = fmax(a0, 0.0); b0 = fmax(b0, (double)S.roi_y0);  // rows above the region of interest are not rendered
    a1 = fmin(a1, (double)(W - 1)); b1 = fmin(b1, (double)(H - 1));
    if (!(a0 <= a1) || !(b0 <= b1)) return PC_OFF;
    P.px0 = (int)a0; P.px1 = (int)a1; P.py0 = (int)b0; P.py1 = (int)b1;
    return PC_OK;
}

// float32 depth key: fma chain on float32-rounded row 2 of W2C
// m: the float32 copy of the view's world-to-camera matrix (CamC::m)
__device__ inline float depth_key(const float *m, const float *x) {
    return __fmaf_rn(m[8], x[0], __fmaf_rn(m[9], x[1], __fmaf_rn(m[10], x[2], m[11])));
}

// Conservative float32 frustum test, run before the float64 projection: true
// only if the exact footprint rectangle is certainly empty.  The exact
// half-width is k sqrt(Sigma2_xx) (1 + pad_rel) + pad_px with Sigma2_xx =
// |J_x A|^2 + eps2d <= |J_x|^2 max(s)^2 + eps2d (W and R are rotations), where
// J_x = (fx / z, 0, -fx xh / z) with the clamped ratio xh; likewise for y.  The
// bound is widened by 0.1% + 1 px + 1e-5 |mu| to cover float32 rounding (and the one-ulp
// hardware reciprocal and square root).  sm2 = max(s)^2, k2f = k^2 in float32.
__device__ inline bool offscreen_bound(const splat_settings &S, const CamC &C, int W, int H, const float *x,
                                       float sm2, float k2f, float z) {
    const float *m = C.m;
    float t0 = __fmaf_rn(m[0], x[0], __fmaf_rn(m[1], x[1], __fmaf_rn(m[2], x[2], m[3])));
    float t1 = __fmaf_rn(m[4], x[0], __fmaf_rn(m[5], x[1], __fmaf_rn(m[6], x[2], m[7])));
    float iz = __builtin_amdgcn_rcpf(z);
    float ux = t0 * iz, uy = t1 * iz;
    float xh = fminf(fmaxf(ux, C.gx0f), C.gx1f);
    float yh = fminf(fmaxf(uy, C.gy0f), C.gy1f);
    float e2 = (float)S.eps2d;
    float jx = C.fxf * iz, jy = C.fyf * iz;
    float sx = jx * jx * (1.f + xh * xh) * sm2 + e2;
    float sy = jy * jy * (1.f + yh * yh) * sm2 + e2;
    float pr = 1.f + (float)S.pad_rel, pp = (float)S.pad_px;
    float mx = C.fxf * ux + C.cxf, my = C.fyf * uy + C.cyf;
    float ex = (__builtin_amdgcn_sqrtf(k2f * sx) * pr + pp) * 1.001f + 1.f + 1e-5f * fabsf(mx);
    float ey = (__builtin_amdgcn_sqrtf(k2f * sy) * pr + pp) * 1.001f + 1.f + 1e-5f * fabsf(my);
    // NaN anywhere makes every comparison false: not culled here, decided exactly afterwards
    return (mx - 0.5f + ex < 0.f) || (mx - 0.5f - ex > (float)(W - 1)) || (my - 0.5f + ey < (float)S.roi_y0) ||
           (my - 0.5f - ey > (float)(H - 1));
}

// Conservative float32 test of the opposite kind: true only if the exact footprint rectangle
// is certainly non-empty.  The exact half-width is at least h = k sqrt(eps2d) + pad_px
// (Sigma2_xx >= eps2d); with h >= 1/2 the interval [u - h, u + h] around u = mu_x - 1/2
// contains the integer nearest to u, which lies in [0, W - 1] whenever u does (likewise for
// y and the rows [roi_y0, H - 1]).  u is bounded through the float32 mean: its error in u_x
// is at most 1e-6 (a0 + |u_x| a2) / z, a0 and a2 being the sums of the magnitudes of the terms
// of t0 and z (four roundings of 2^-24 each, and one ulp of the reciprocal, widened 4x), and
// 1e-5 |mu| + 1 px are added.  h_ok: h >= 1/2 with h = sqrt(k2 eps2d) 0.9999 + pad_px (per
// Gaussian).
__device__ inline bool onscreen_bound(const splat_settings &S, const CamC &C, int W, int H, const float *x,
                                      bool h_ok, float z) {
    if (!h_ok) return false;
    const float *m = C.m;
    float t0 = __fmaf_rn(m[0], x[0], __fmaf_rn(m[1], x[1], __fmaf_rn(m[2], x[2], m[3])));
    float t1 = __fmaf_rn(m[4], x[0], __fmaf_rn(m[5], x[1], __fmaf_rn(m[6], x[2], m[7])));
    float a0 = fabsf(m[0] * x[0]) + fabsf(m[1] * x[1]) + fabsf(m[2] * x[2]) + fabsf(m[3]);
    float a1 = fabsf(m[4] * x[0]) + fabsf(m[5] * x[1]) + fabsf(m[6] * x[2]) + fabsf(m[7]);
    float a2 = fabsf(m[8] * x[0]) + fabsf(m[9] * x[1]) + fabsf(m[10] * x[2]) + fabsf(m[11]);
    float iz = __builtin_amdgcn_rcpf(z);
    float ux = t0 * iz, uy = t1 * iz;
    float fx = C.fxf, fy = C.fyf;
    float mx = fx * ux + C.cxf, my = fy * uy + C.cyf;
    float dx = 1.f + 1e-5f * fabsf(mx) + 1e-6f * fabsf(fx) * (a0 + fabsf(ux) * a2) * iz;
    float dy = 1.f + 1e-5f * fabsf(my) + 1e-6f * fabsf(fy) * (a1 + fabsf(uy) * a2) * iz;
    float u = mx - 0.5f, v = my - 0.5f;
    // NaN anywhere makes every comparison false: decided exactly afterwards
    return (u - dx >= 0.f) && (u + dx <= (float)(W - 1)) && (v - dy >= (float)S.roi_y0) && (v + dy <= (float)(H - 1));
}

// What a view makes of one Gaussian, in the order of the cull tests: non-finite
// input, depth at or before the near plane, beyond the far plane, opacity below
// alpha_min, degenerate quaternion, footprint off the image; 0 = visible.
struct GaussIn {
    float x[3], q[4], s[3], o;
    bool fin, opac_ok, quat_ok;
    GaussPre G;
    float k2f, sm2;  // the cull bounds' per-Gaussian terms: k^2 and max(s)^2 in float32
    bool h_ok;       // the smallest footprint half-width reaches half a pixel
};

__device__ inline void gauss_in(const splat_settings &S, const splat_gaussians &g, int64_t i, GaussIn &gi) {
    int64_t n = g.n;
    gi.x[0] = g.mean[i]; gi.x[1] = g.mean[n + i]; gi.x[2] = g.mean[2 * n + i];
    gi.q[0] = g.quat[i]; gi.q[1] = g.quat[n + i]; gi.q[2] = g.quat[2 * n + i]; gi.q[3] = g.quat[3 * n + i];
    gi.s[0] = g.scale[i]; gi.s[1] = g.scale[n + i]; gi.s[2] = g.scale[2 * n + i];
    gi.o = g.opacity[i];
    gi.fin = finite_f(gi.x[0]) && finite_f(gi.x[1]) && finite_f(gi.x[2]) && finite_f(gi.q[0]) && finite_f(gi.q[1]) &&
             finite_f(gi.q[2]) && finite_f(gi.q[3]) && finite_f(gi.s[0]) && finite_f(gi.s[1]) && finite_f(gi.s[2]) &&
             finite_f(gi.o);
    gi.opac_ok = (double)gi.o >= S.alpha_min;
    double n2 = (double)gi.q[0] * gi.q[0] + (double)gi.q[1] * gi.q[1] + (double)gi.q[2] * gi.q[2] +
                (double)gi.q[3] * gi.q[3];
    gi.quat_ok = n2 >= 1e-24;
    const bool pre = gi.fin && gi.opac_ok && gi.quat_ok;
    if (pre) gauss_pre(S, gi.q, gi.o, gi.G);
    gi.k2f = pre ? (float)gi.G.k2 : 0.f;  // read by the bounds only after those three checks
    const float sm = fmaxf(fmaxf(gi.s[0], gi.s[1]), gi.s[2]);
    gi.sm2 = sm * sm;
    gi.h_ok = sqrtf(gi.k2f * (float)S.eps2d) * 0.9999f + (float)S.pad_px >= 0.5001f;
}

__device__ inline int classify(const splat_settings &S, const double *M, const CamC &C, int W, int H,
                               const GaussIn &gi, Proj &P) {
    if (!gi.fin) return PC_NONFINITE;
    P.depth32 = depth_key(C.m, gi.x);
    if (!(P.depth32 > (float)S.near_z)) return PC_NEAR;
    if (P.depth32 > (float)S.far_z) return PC_FAR;
    if (!gi.opac_ok) return PC_OPAC;
    if (!gi.quat_ok) return PC_QUAT;
    if (offscreen_bound(S, C, W, H, gi.x, gi.sm2, gi.k2f, P.depth32)) return PC_OFF;
    // most visible pairs are decided here; the float64 projection is for the ones near an edge
    if (onscreen_bound(S, C, W, H, gi.x, gi.h_ok, P.depth32)) return PC_OK;
    project_view(S, M, C, gi.x, gi.s, gi.G, false, P);
    return footprint(S, gi.G.k2, W, H, P);
}

__device__ inline void flag_status(uint32_t *status, uint32_t bits) {
    uint64_t any = __ballot(bits != 0);
    if (any) {
        // reduce the bits over the wave, then one atomic
        uint32_t b = bits;
        for (int o = 32; o > 0; o >>= 1) b |= __shfl_xor(b, o, kWave);
        if (__lane_id() == (int)(__ffsll((long long)any) - 1)) atomicOr(status, b);
    }
}

// Count pass: one thread per Gaussian walks every view (the parameters are read
// once); per (view, wave) it stores the visibility mask and the visible count.
// Slots are later numbered by an exclusive scan over (view, wave), so they are
// compacted per view in Gaussian order.
__global__ __launch_bounds__(256) void project_count_kernel(splat_settings S, splat_gaussians g, const double *w2c,
                                                           const CamC *cam, int W, int H, int V, int nb,
                                                           uint32_t *wavecnt, uint64_t *visbits, uint32_t *status) {
    const int b = blockIdx.x, w = threadIdx.x >> 6, lane = __lane_id();
    const int64_t i = (int64_t)b * 256 + threadIdx.x;
    const bool live = i < g.n;
    GaussIn gi;
    if (live) gauss_in(S, g, i, gi);
    uint32_t bits = 0;
    for (int v = 0; v < V; ++v) {
        int code = PC_OFF;
        if (live) {
            Proj P;
            code = classify(S, w2c + 12 * v, cam[v], W, H, gi, P);
        }
        bits |= (code == PC_NONFINITE ? SPLAT_ST_NONFINITE : 0u) | (code == PC_QUAT ? SPLAT_ST_DEGENERATE : 0u);
        uint64_t m = __ballot(code == PC_OK);
        if (lane == 0) {
            size_t k = ((size_t)v * nb + b) * 4 + w;
            visbits[k] = m;
            wavecnt[k] = (uint32_t)__popcll(m);
        }
    }
    flag_status(status, bits);
}

// Packing of a slot's payload for the slot-first bin sort (null spay: not used): slot id, first
// tile (view * T + tile), rect width - 1 and height - 1 in tiles, at bit offsets 0, b0, b0 + tb,
// b0 + tb + b1.
struct SlotPack {
    uint64_t *spay;
    int b0, tb, b1, tiles_x, T;
};

// Write pass: the same walk, projecting only the pairs the count pass marked
// visible, into their slots.
__global__ __launch_bounds__(256) void project_write_kernel(splat_settings S, splat_gaussians g, const double *w2c,
                                                           const CamC *cam, int W, int H, int V, int nb,
                                                           const uint32_t *waveoff, const uint64_t *visbits,
                                                           int64_t slot_cap, float4 *rec, int2 *meta, Rect16 *rect,
                                                           uint32_t *ntiles, uint32_t *dkey, SlotPack sp) {
    const int b = blockIdx.x, w = threadIdx.x >> 6, lane = __lane_id();
    const int64_t i = (int64_t)b * 256 + threadIdx.x;
    if (i >= g.n) return;
    GaussIn gi;
    gauss_in(S, g, i, gi);
    const int64_t n = g.n;
    const float cr = g.color[i], cg = g.color[n + i], cb = g.color[2 * n + i];
    // tile sizes are powers of two and the footprint bounds are non-negative: shifts divide
    const int tws = __builtin_ctz((unsigned)S.tile_w), ths = __builtin_ctz((unsigned)S.tile_h);
    for (int v = 0; v < V; ++v) {
        size_t k = ((size_t)v * nb + b) * 4 + w;
        uint64_t m = visbits[k];
        if (!((m >> lane) & 1ull)) continue;
        uint64_t slot = (uint64_t)waveoff[k] + rank_in(m);
        if (slot >= (uint64_t)slot_cap) continue;  // capacity flagged by the scan finisher
        const double *M = w2c + 12 * v;
        Proj P;
        P.depth32 = depth_key(cam[v].m, gi.x);
        project_view(S, M, cam[v], gi.x, gi.s, gi.G, true, P);
        footprint(S, gi.G.k2, W, H, P);  // visible: the count pass found this rectangle non-empty
        float mxh = (float)P.mu[0], myh = (float)P.mu[1];
        float mxl = (float)(P.mu[0] - (double)mxh), myl = (float)(P.mu[1] - (double)myh);
        rec[3 * slot + 0] = make_float4(mxh, myh, mxl, myl);
        rec[3 * slot + 1] = make_float4((float)P.Q[0], (float)P.Q[1], (float)P.Q[2], gi.o);
        rec[3 * slot + 2] = make_float4(cr, cg, cb, P.depth32);
        dkey[slot] = __float_as_uint(P.depth32) - __float_as_uint((float)S.near_z);
        Rect16 rc;
        rc.x0 = (uint16_t)(P.px0 >> tws); rc.x1 = (uint16_t)(P.px1 >> tws);
        rc.y0 = (uint16_t)(P.py0 >> ths); rc.y1 = (uint16_t)(P.py1 >> ths);
        if (!sp.spay) {  // the 64-bit instance sort reads the rect, tile count and view of every slot
            meta[slot] = make_int2((int)i, v);
            rect[slot] = rc;
            ntiles[slot] = (uint32_t)(rc.x1 - rc.x0 + 1) * (uint32_t)(rc.y1 - rc.y0 + 1);
        } else {
            const uint64_t first = (uint64_t)v * (uint64_t)sp.T + (uint64_t)rc.y0 * (uint64_t)sp.tiles_x + rc.x0;
            // a field of width 0 holds 0 and may sit at bit 64: no shift by 64
            const int s1 = sp.b0 + sp.tb, s2 = s1 + sp.b1;
            sp.spay[slot] = slot | (first << sp.b0) | (s1 < 64 ? (uint64_t)(rc.x1 - rc.x0) << s1 : 0ull) |
                            (s2 < 64 ? (uint64_t)(rc.y1 - rc.y0) << s2 : 0ull);
        }
    }
}


// (Gaussian id, view) of every slot, from the visibility words and slot offsets the last
// projection left (its write pass stores them only for the 64-bit instance sort)
__global__ __launch_bounds__(256) void slot_meta_kernel(int64_t n, int V, int nb, const uint32_t *waveoff,
                                                        const uint64_t *visbits, const uint32_t *counts, int2 *meta) {
    const int b = blockIdx.x, w = threadIdx.x >> 6, lane = __lane_id();
    const int64_t i = (int64_t)b * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t ns = counts[CNT_SLOTS];
    for (int v = 0; v < V; ++v) {
        const size_t k = ((size_t)v * nb + b) * 4 + w;
        const uint64_t m = visbits[k];
        if (!((m >> lane) & 1ull)) continue;
        const uint64_t slot = (uint64_t)waveoff[k] + rank_in(m);
        if (slot < ns) meta[slot] = make_int2((int)i, v);
    }
}

// totals after the (view, wave) count scan: slot count (clamped), view offsets, capacity flag
__global__ void project_finish_kernel(const uint32_t *waveoff, int V, int nw, int64_t slot_cap, uint32_t *counts,
                                      uint32_t *view_off, uint32_t *status, uint32_t prep) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t total = waveoff[(size_t)V * nw];
    uint32_t cap = (uint32_t)slot_cap;
    if (v <= V) {
        uint32_t off = (v < V) ? waveoff[(size_t)v * nw] : total;
        view_off[v] = off < cap ? off : cap;
    }
    if (v == 0) {
        counts[CNT_SLOTS] = total < cap ? total : cap;
        counts[CNT_PREP] = prep;
        if (total > cap) atomicOr(status, SPLAT_ST_CAPACITY);
    }
}

// ----------------------------------------------------------------------------------
// adjoint
// ----------------------------------------------------------------------------------
// Chain rule of one visible (view, Gaussian) pair from its slot gradient: the
// render adjoint leaves in gd[0..4] the moments (Mx, My, Mxx, Mxy, Myy) of
// dL/dpower over the pixel offsets d = pixel - mu (M. = sum dL/dpower * d. over
// the pixels), with power = -(a dx^2 + 2 b dx dy + c dy^2)/2 for the conic
// (a, b, c), so that dL/dmu = (a Mx + b My, b Mx + c My) and
// dL/d(a, b, c) = (-Mxx/2, -Mxy, -Myy/2).  Adds the quaternion, scale and mean
// gradients to gR (dL/dR of the Gaussian's rotation, turned into the quaternion's gradient once
// per Gaussian after the views: the map from dR to dq depends on the quaternion only), gs, gm
// and returns the W2C gradient in gw[12].  iz = 1 / t_z (from project_view_adj).
__device__ void slot_adjoint(const Proj &P, const double *R, const double *M, const CamC &C, const float *x,
                             const float *s, const float *gd, double iz, double *gRs, double *gs, double *gm,
                             double *gw) {
    double a = P.Q[0], b = P.Q[1], c = P.Q[2];
    const double Mx = gd[0], My = gd[1];
    double gmx = a * Mx + b * My, gmy = b * Mx + c * My;
    double ga = -0.5 * (double)gd[2], gb = -(double)gd[3], gc = -0.5 * (double)gd[4];
    // conic -> Sigma2: G2 = -Q GQ Q with GQ = [[ga, gb/2], [gb/2, gc]]
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
    double fx = C.fx, fy = C.fy;
    double tx = P.t[0], ty = P.t[1], tz = P.t[2];
    double iz2 = iz * iz;
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
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int m = 0; m < 3; ++m) acc += M[4 * m + r] * gA[3 * m + k];  // (W^T gA)[r][k]
            gRs[3 * r + k] += acc * (double)s[k];
            gs[k] += R[3 * r + k] * acc;  // ((W R)^T gA)_kk = sum_r R[r][k] (W^T gA)[r][k]
        }
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int m = 0; m < 3; ++m) acc += gA[3 * r + m] * R[3 * k + m] * (double)s[m];
            gw[4 * r + k] = acc + gt[r] * (double)x[k];
        }
    for (int r = 0; r < 3; ++r) gw[4 * r + 3] = gt[r];
    for (int k = 0; k < 3; ++k) gm[k] += M[k] * gt[0] + M[4 + k] * gt[1] + M[8 + k] * gt[2];
}

// R(q_hat) -> q_hat -> q: the quaternion gradient of a Gaussian from its summed dL/dR
__device__ inline void quat_adjoint(const GaussPre &G, const double *gR, double *gq) {
    double w = G.qh[0], qx = G.qh[1], qy = G.qh[2], qz = G.qh[3];
    double gq0 = 2.0 * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
    double gq1 = 2.0 * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2.0 * qx * gR[4] - w * gR[5] + qz * gR[6] + w * gR[7] - 2.0 * qx * gR[8]);
    double gq2 = 2.0 * (-2.0 * qy * gR[0] + qx * gR[1] + w * gR[2] + qx * gR[3] + qz * gR[5] - w * gR[6] + qz * gR[7] - 2.0 * qy * gR[8]);
    double gq3 = 2.0 * (-2.0 * qz * gR[0] - w * gR[1] + qx * gR[2] + w * gR[3] - 2.0 * qz * gR[4] + qy * gR[5] + qx * gR[6] + qy * gR[7]);
    double dot = w * gq0 + qx * gq1 + qy * gq2 + qz * gq3;
    double iq = 1.0 / G.qn;
    gq[0] = (gq0 - w * dot) * iq;
    gq[1] = (gq1 - qx * dot) * iq;
    gq[2] = (gq2 - qy * dot) * iq;
    gq[3] = (gq3 - qz * dot) * iq;
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
                                                         const CamC *cam, int V, int nb, const uint32_t *waveoff,
                                                         const uint64_t *visbits, int64_t slot_cap,
                                                         const float *grad2d, float *dquat, float *dscale,
                                                         float *dopac, float *dcolor, float *dmean, double *dwpart) {
    // Every wave walks the views on its own (no workgroup barrier in the loop), writing its
    // FP64 W2C partial per view; the next view's visibility word and slot base are loaded
    // while the current view is processed.
    const int b = blockIdx.x, wv = threadIdx.x >> 6, lane = __lane_id();
    const LaneClass lc(lane);
    const bool writer = lane < 16 && lc.cls < 12;
    const int64_t i = (int64_t)b * 256 + threadIdx.x;
    const int64_t n = g.n;
    const bool live = i < n;
    GaussIn gi;
    if (live) gauss_in(S, g, i, gi);
    double gR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gs[3] = {0, 0, 0}, gm[3] = {0, 0, 0}, go = 0.0, gc[3] = {0, 0, 0};
    size_t k0 = (size_t)b * 4 + wv;  // (view, block, wave) index of view 0
    const size_t kstep = (size_t)nb * 4;
    uint64_t mask = visbits[k0];
    uint32_t base = waveoff[k0];
    for (int v = 0; v < V; ++v, k0 += kstep) {
        uint64_t mask_n = 0;
        uint32_t base_n = 0;
        if (v + 1 < V) {
            mask_n = visbits[k0 + kstep];
            base_n = waveoff[k0 + kstep];
        }
        double *part = dwpart + k0 * 12;
        const bool vis = live && ((mask >> lane) & 1ull);
        if (mask != 0ull) {  // otherwise nothing of this wave is visible in view v: no partial (the
                             // reduction skips it by the same visibility word)
            double gw[12];
            for (int k = 0; k < 12; ++k) gw[k] = 0.0;
            if (vis) {
                uint64_t slot = (uint64_t)base + rank_in(mask);
                if (slot < (uint64_t)slot_cap) {
                    const double *M = w2c + 12 * v;
                    const CamC C = cam[v];
                    Proj P;
                    double iz;
                    project_view_adj(S, M, C, gi.x, gi.s, gi.G, P, iz);
                    const float *gd = grad2d + 9 * slot;
                    go += (double)gd[5] / (double)gi.o;   // gd[5] = sum of dL/dpower = o dL/do
                    gc[0] += gd[6];
                    gc[1] += gd[7];
                    gc[2] += gd[8];
                    slot_adjoint(P, gi.G.R, M, C, gi.x, gi.s, gd, iz, gR, gs, gm, gw);
                }
            }
            double tot = reduce12(gw, lc.c0, lc.c1, lc.c2, lc.c3);
            if (writer) part[lc.cls] = tot;
        }
        mask = mask_n;
        base = base_n;
    }
    if (!live) return;
    double gq[4] = {0, 0, 0, 0};
    if (gi.fin && gi.opac_ok && gi.quat_ok) quat_adjoint(gi.G, gR, gq);  // G is set for these only
    for (int k = 0; k < 4; ++k) dquat[k * n + i] += (float)gq[k];
    for (int k = 0; k < 3; ++k) dscale[k * n + i] += (float)gs[k];
    dopac[i] += (float)go;
    for (int k = 0; k < 3; ++k) dcolor[k * n + i] += (float)gc[k];
    if (dmean)
        for (int k = 0; k < 3; ++k) dmean[k * n + i] += (float)gm[k];
}

// dw2c[v] += sum over the (block, wave) partials of view v, in a fixed order, in two
// stages: workgroup (s, v) sums the partials q = t + 256 (s + DW_S j) of view v (thread t,
// j = 0, 1, ...) into stage[v][s], then dw2c_finish_kernel adds the DW_S stage sums of a
// view in order.  DW_S workgroups per view keep the whole chip reading.
constexpr int DW_S = kDw2cStages;

__global__ __launch_bounds__(256) void dw2c_reduce_kernel(const double *dwpart, const uint64_t *visbits, int nparts,
                                                          double *stage) {
    __shared__ double red[4][12];
    const int s = blockIdx.x, v = blockIdx.y, wv = threadIdx.x >> 6, lane = __lane_id();
    const LaneClass lc(lane);
    double acc[12];
    for (int k = 0; k < 12; ++k) acc[k] = 0.0;
    for (int q = threadIdx.x + 256 * s; q < nparts; q += 256 * DW_S) {
        if (visbits[(size_t)v * nparts + q] == 0ull) continue;  // a wave with nothing visible wrote none
        const double *p = dwpart + ((size_t)v * nparts + q) * 12;
        for (int k = 0; k < 12; ++k) acc[k] += p[k];
    }
    double tot = reduce12(acc, lc.c0, lc.c1, lc.c2, lc.c3);
    if (lane < 16 && lc.cls < 12) red[wv][lc.cls] = tot;
    __syncthreads();
    if (threadIdx.x < 12) {
        int k = threadIdx.x;
        stage[((size_t)v * DW_S + s) * 12 + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

__global__ void dw2c_finish_kernel(const double *stage, double *dw2c) {
    const int v = blockIdx.x, k = threadIdx.x;
    if (k >= 12) return;
    double t = 0.0;
    for (int s = 0; s < DW_S; ++s) t += stage[((size_t)v * DW_S + s) * 12 + k];
    dw2c[12 * v + k] += t;
}

}  // namespace

int launch_project(const splat_plan &p, void *ws, const splat_gaussians &g, const double *w2c,
                   const double *intr, hipStream_t st) {
    int V = p.n_views, nb = p.n_blocks_proj, nw = 4 * nb;
    uint32_t *status = ws_at<uint32_t>(ws, p.off_status);
    uint32_t *counts = ws_at<uint32_t>(ws, p.off_counts);
    uint32_t *wavecnt = ws_at<uint32_t>(ws, p.off_blockcnt);
    CamC *cam = ws_at<CamC>(ws, p.off_cam);
    uint64_t *visbits = ws_at<uint64_t>(ws, p.off_visbits);
    hipLaunchKernelGGL(camconst_kernel, dim3((V + 63) / 64), dim3(64), 0, st, p.s, intr, w2c, V, p.width, p.height,
                       cam);
    int rc = launch_status("camconst");
    if (rc) return rc;
    if (g.n == 0) {
        rc = launch_fill_u32(wavecnt, 0u, (int64_t)V * nw + 1, st);
        if (rc) return rc;
    } else {
        hipLaunchKernelGGL(project_count_kernel, dim3(nb), dim3(256), 0, st, p.s, g, w2c, cam, p.width, p.height, V,
                           nb, wavecnt, visbits, status);
        rc = launch_status("project_count");
        if (rc) return rc;
        rc = launch_scan_u32(wavecnt, wavecnt, nullptr, (int64_t)V * nw, ws_at<uint32_t>(ws, p.off_scan), nullptr,
                             st);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(project_finish_kernel, dim3((V + 1 + 255) / 256), dim3(256), 0, st, wavecnt, V, nw,
                       p.slot_cap, counts, ws_at<uint32_t>(ws, p.off_view_off), status,
                       p.slot_sort ? kPrepSlotSort : kPrepInstSort);
    rc = launch_status("project_finish");
    if (rc || g.n == 0) return rc;
    hipLaunchKernelGGL(project_write_kernel, dim3(nb), dim3(256), 0, st, p.s, g, w2c, cam, p.width, p.height, V, nb,
                       wavecnt, visbits, p.slot_cap, ws_at<float4>(ws, p.off_rec), ws_at<int2>(ws, p.off_meta),
                       ws_at<Rect16>(ws, p.off_rect), ws_at<uint32_t>(ws, p.off_ntiles),
                       ws_at<uint32_t>(ws, p.off_dkey),
                       SlotPack{p.slot_sort ? ws_at<uint64_t>(ws, p.off_spay) : nullptr, p.pack_bits[0], p.tile_bits,
                                p.pack_bits[1], p.tiles_x, p.tiles_per_view});
    return launch_status("project_write");
}

int launch_slot_meta(const splat_plan &p, void *ws, hipStream_t st) {
    if (p.n_gauss == 0) return 0;
    hipLaunchKernelGGL(slot_meta_kernel, dim3(p.n_blocks_proj), dim3(256), 0, st, p.n_gauss, p.n_views,
                       p.n_blocks_proj, ws_at<uint32_t>(ws, p.off_blockcnt), ws_at<uint64_t>(ws, p.off_visbits),
                       ws_at<uint32_t>(ws, p.off_counts), ws_at<int2>(ws, p.off_meta));
    return launch_status("slot_meta");
}

int launch_project_bwd(const splat_plan &p, void *ws, const splat_gaussians &g, const double *w2c,
                       const double *intr, float *dquat, float *dscale, float *dopac, float *dcolor,
                       float *dmean, double *dw2c, hipStream_t st) {
    if (g.n == 0) return 0;
    int nb = p.n_blocks_proj;
    double *part = ws_at<double>(ws, p.off_dwpart);
    hipLaunchKernelGGL(camconst_kernel, dim3((p.n_views + 63) / 64), dim3(64), 0, st, p.s, intr, w2c, p.n_views,
                       p.width, p.height, ws_at<CamC>(ws, p.off_cam));
    int rc0 = launch_status("camconst");
    if (rc0) return rc0;
    hipLaunchKernelGGL(project_bwd_kernel, dim3(nb), dim3(256), 0, st, p.s, g, w2c, ws_at<CamC>(ws, p.off_cam),
                       p.n_views, nb, ws_at<uint32_t>(ws, p.off_blockcnt), ws_at<uint64_t>(ws, p.off_visbits),
                       p.slot_cap, ws_at<float>(ws, p.off_grad2d), dquat, dscale, dopac, dcolor, dmean, part);
    int rc = launch_status("project_bwd");
    if (rc) return rc;
    // the stage sums sit after the partials (the plan sizes the region for both)
    double *stage = part + (size_t)p.n_views * 4 * nb * 12;
    hipLaunchKernelGGL(dw2c_reduce_kernel, dim3(DW_S, p.n_views), dim3(256), 0, st, part,
                       ws_at<uint64_t>(ws, p.off_visbits), 4 * nb, stage);
    if ((rc = launch_status("dw2c_reduce"))) return rc;
    hipLaunchKernelGGL(dw2c_finish_kernel, dim3(p.n_views), dim3(64), 0, st, stage, dw2c);
    return launch_status("dw2c_finish");
}

}  // namespace splat
