/*
 * splat_oracle.c -- plain, slow FP64 CPU reference of the differentiable
 * splatting path of 3DGS-Calib (arXiv 2403.11577).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source, header, table or helper with the HIP
 * library.
 *
 * What it computes (paper, Sec. III-A and III-B):
 *   - the continuous LiDAR trajectory: linear interpolation of the translation
 *     and SLERP of the rotation between timestamped poses (Sec. III-A);
 *   - the camera pose of Eq. (1): T = T_L(t + delta) * T_cam->LiDAR, and the
 *     world->camera transform of Eq. (2) (its inverse);
 *   - the camera-frame Gaussian covariance of Eq. (3) as W Sigma W^T;
 *   - EWA splatting (the rendering function Phi of Eq. (5)): perspective
 *     Jacobian, 2-D covariance with a screen-space low-pass, and front-to-back
 *     alpha compositing of every Gaussian at every pixel in full depth order
 *     (no tiles);
 *   - the exact reverse-mode derivative of all of the above with respect to
 *     the Gaussian parameters and, through the input pose, to the extrinsic
 *     correction (rho, phi) and the time offset delta (end of Sec. III-B).
 *
 * Readings where the paper is silent (listed with reasons in the design notes):
 *   pixel centres at +0.5; alpha = min(alpha_max, o * exp(power)); Gaussians with
 *   alpha < alpha_min are skipped; compositing stops before a blend that would
 *   take the transmittance below t_min; eps2d is added to the 2-D covariance
 *   diagonal without renormalising opacity; the Jacobian uses x/z and y/z
 *   clamped to a guard band; colours are used directly (view independent);
 *   the extrinsic is R = R0 Exp(phi), t = t0 + rho; depth order is the FP32
 *   fused-multiply-add chain "depth32" with ties broken by Gaussian index, and
 *   the near/far culls use the same depth32.
 *
 * Everything is FP64 except depth32, which both implementations compute the
 * same way on purpose so that the depth order is a specification, not a
 * rounding accident.  Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double near_z, far_z, eps2d, alpha_min, alpha_max, t_min, guard;
    double bg[3];
    double margin;   /* relative margin of a threshold decision that is flagged */
    double pad_px;   /* footprint padding, pixels */
    double pad_rel;  /* footprint padding, relative to the radius */
    int32_t roi_y0;  /* first image row of the region of interest (Sec. III-C, image cropping) */
    int32_t roi_pad_;
} or_settings;

/* ------------------------------------------------------------------------ */
/* small 3x3 helpers (row-major)                                             */
/* ------------------------------------------------------------------------ */
static void mm3(const double *A, const double *B, double *C) {
    double t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            t[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
    memcpy(C, t, sizeof t);
}
static void mtm3(const double *A, const double *B, double *C) { /* A^T B */
    double t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            t[3 * i + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
    memcpy(C, t, sizeof t);
}
static void mmt3(const double *A, const double *B, double *C) { /* A B^T */
    double t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            t[3 * i + j] = A[3 * i] * B[3 * j] + A[3 * i + 1] * B[3 * j + 1] + A[3 * i + 2] * B[3 * j + 2];
    memcpy(C, t, sizeof t);
}
static void mv3(const double *A, const double *x, double *y) {
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
    memcpy(y, t, sizeof t);
}
static void mtv3(const double *A, const double *x, double *y) { /* A^T x */
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = A[i] * x[0] + A[3 + i] * x[1] + A[6 + i] * x[2];
    memcpy(y, t, sizeof t);
}

static void quat_to_R(const double *q, double *R) { /* unit q = (w,x,y,z) */
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Rodrigues: Exp of a rotation vector. */
static void so3_exp(const double *v, double *R) {
    double th2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double th = sqrt(th2);
    double A, B;
    if (th < 1e-6) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
    }
    double K[9] = {0, -v[2], v[1], v[2], 0, -v[0], -v[1], v[0], 0};
    double K2[9];
    mm3(K, K, K2);
    for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0 ? 1.0 : 0.0) + A * K[i] + B * K2[i];
}

/* Log of a rotation matrix (angle < pi assumed; trajectories are sampled densely). */
static void so3_log(const double *R, double *v) {
    double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    double th = acos(c);
    double w[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
    double f;
    if (th < 1e-6)
        f = 0.5 + th * th / 12.0;
    else
        f = th / (2.0 * sin(th));
    v[0] = f * w[0];
    v[1] = f * w[1];
    v[2] = f * w[2];
}

/* Right Jacobian of SO(3): Exp(phi + d) ~= Exp(phi) Exp(Jr(phi) d). */
static void so3_jr(const double *phi, double *J) {
    double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    double th = sqrt(th2);
    double a, b;
    if (th < 1e-6) {
        a = 0.5 - th2 / 24.0;
        b = 1.0 / 6.0 - th2 / 120.0;
    } else {
        a = (1.0 - cos(th)) / th2;
        b = (th - sin(th)) / (th2 * th);
    }
    double K[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
    double K2[9];
    mm3(K, K, K2);
    for (int i = 0; i < 9; ++i) J[i] = (i % 4 == 0 ? 1.0 : 0.0) - a * K[i] + b * K2[i];
}

/* ------------------------------------------------------------------------ */
/* trajectory + Eq. (1), (2)                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int k;           /* segment index */
    double u, dt;    /* position in segment and its duration */
    double Rs[9], ps[3];   /* LiDAR pose at s */
    double om[3];    /* Log(R_k^T R_{k+1}) */
    double dp[3];    /* p_{k+1} - p_k */
    double Re[9], te[3];   /* extrinsic camera->LiDAR */
    double Rcw[9], pcw[3]; /* camera->world */
} pose_state;

static void pose_eval(int K, const double *kt, const double *kq, const double *kp,
                      const double *R0, const double *t0, const double *xi, double s,
                      pose_state *st) {
    int k = 0;
    /* segment: largest k with t_k <= s, clamped to [0, K-2]; a knot starts its right segment */
    for (int i = 0; i < K; ++i)
        if (kt[i] <= s) k = i;
    if (k > K - 2) k = K - 2;
    if (k < 0) k = 0;
    st->k = k;
    st->dt = kt[k + 1] - kt[k];
    st->u = (s - kt[k]) / st->dt;
    double qa[4], qb[4], Ra[9], Rb[9];
    for (int i = 0; i < 4; ++i) { qa[i] = kq[4 * k + i]; qb[i] = kq[4 * (k + 1) + i]; }
    double na = sqrt(qa[0] * qa[0] + qa[1] * qa[1] + qa[2] * qa[2] + qa[3] * qa[3]);
    double nb = sqrt(qb[0] * qb[0] + qb[1] * qb[1] + qb[2] * qb[2] + qb[3] * qb[3]);
    for (int i = 0; i < 4; ++i) { qa[i] /= na; qb[i] /= nb; }
    quat_to_R(qa, Ra);
    quat_to_R(qb, Rb);
    double Rab[9], E[9], uom[3];
    mtm3(Ra, Rb, Rab);
    so3_log(Rab, st->om);
    for (int i = 0; i < 3; ++i) uom[i] = st->u * st->om[i];
    so3_exp(uom, E);
    mm3(Ra, E, st->Rs);
    for (int i = 0; i < 3; ++i) {
        st->dp[i] = kp[3 * (k + 1) + i] - kp[3 * k + i];
        st->ps[i] = (1.0 - st->u) * kp[3 * k + i] + st->u * kp[3 * (k + 1) + i];
    }
    double Ep[9];
    so3_exp(xi + 3, Ep);
    mm3(R0, Ep, st->Re);
    for (int i = 0; i < 3; ++i) st->te[i] = t0[i] + xi[i];
    mm3(st->Rs, st->Re, st->Rcw);
    mv3(st->Rs, st->te, st->pcw);
    for (int i = 0; i < 3; ++i) st->pcw[i] += st->ps[i];
}

/* w2c[V][12]: row-major [W | w] with W = Rcw^T, w = -Rcw^T pcw. */
int or_pose(int K, const double *kt, const double *kq, const double *kp,
            int C, const double *R0, const double *t0, const double *xi, const double *delta,
            int V, const int *vcam, const double *vt,
            double *w2c, int *seg, double *useg) {
    if (K < 2) return -1;
    for (int v = 0; v < V; ++v) {
        int c = vcam[v];
        if (c < 0 || c >= C) return -1;
        pose_state st;
        pose_eval(K, kt, kq, kp, R0 + 9 * c, t0 + 3 * c, xi + 6 * c, vt[v] + delta[c], &st);
        double Wm[9], w[3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Wm[3 * i + j] = st.Rcw[3 * j + i];
        mv3(Wm, st.pcw, w);
        for (int i = 0; i < 3; ++i) {
            w2c[12 * v + 4 * i + 0] = Wm[3 * i + 0];
            w2c[12 * v + 4 * i + 1] = Wm[3 * i + 1];
            w2c[12 * v + 4 * i + 2] = Wm[3 * i + 2];
            w2c[12 * v + 4 * i + 3] = -w[i];
        }
        if (seg) seg[v] = st.k;
        if (useg) useg[v] = st.u;
    }
    return 0;
}

/* vee of the skew part: <M, [v]x> = v . vee(M) */
static void skew_vee(const double *M, double *v) {
    v[0] = M[7] - M[5];
    v[1] = M[2] - M[6];
    v[2] = M[3] - M[1];
}

int or_pose_bwd(int K, const double *kt, const double *kq, const double *kp,
                int C, const double *R0, const double *t0, const double *xi, const double *delta,
                int V, const int *vcam, const double *vt, const double *dw2c,
                double *dxi, double *ddelta) {
    if (K < 2) return -1;
    memset(dxi, 0, sizeof(double) * 6 * C);
    memset(ddelta, 0, sizeof(double) * C);
    for (int v = 0; v < V; ++v) {
        int c = vcam[v];
        if (c < 0 || c >= C) return -1;
        pose_state st;
        pose_eval(K, kt, kq, kp, R0 + 9 * c, t0 + 3 * c, xi + 6 * c, vt[v] + delta[c], &st);
        double GW[9], gw[3];
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) GW[3 * i + j] = dw2c[12 * v + 4 * i + j];
            gw[i] = dw2c[12 * v + 4 * i + 3];
        }
        /* W = Rcw^T, w = -Rcw^T pcw */
        double GRcw[9], gpcw[3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) GRcw[3 * i + j] = GW[3 * j + i] - st.pcw[i] * gw[j];
        mv3(st.Rcw, gw, gpcw);
        for (int i = 0; i < 3; ++i) gpcw[i] = -gpcw[i];
        /* Rcw = Rs Re ; pcw = Rs te + ps */
        double GRs[9], GRe[9], gte[3];
        mmt3(GRcw, st.Re, GRs);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) GRs[3 * i + j] += gpcw[i] * st.te[j];
        mtm3(st.Rs, GRcw, GRe);
        mtv3(st.Rs, gpcw, gte);
        /* te = t0 + rho */
        for (int i = 0; i < 3; ++i) dxi[6 * c + i] += gte[i];
        /* Re = R0 Exp(phi): dL/dphi = Jr(phi)^T vee(Re^T GRe) */
        double M[9], vv[3], Jr[9], dphi[3];
        mtm3(st.Re, GRe, M);
        skew_vee(M, vv);
        so3_jr(xi + 6 * c + 3, Jr);
        mtv3(Jr, vv, dphi);
        for (int i = 0; i < 3; ++i) dxi[6 * c + 3 + i] += dphi[i];
        /* s = t_v + delta: dRs/ds = Rs [om/dt]x, dps/ds = dp/dt */
        double M2[9], v2[3];
        mtm3(st.Rs, GRs, M2);
        skew_vee(M2, v2);
        double ds = 0.0;
        for (int i = 0; i < 3; ++i) ds += (v2[i] * st.om[i] + gpcw[i] * st.dp[i]) / st.dt;
        ddelta[c] += ds;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* projection (Eq. 2, Eq. 3, EWA)                                            */
/* ------------------------------------------------------------------------ */
enum { CULL_NONE = 0, CULL_NEAR = 1, CULL_FAR = 2, CULL_OPACITY = 4, CULL_QUAT = 8,
       CULL_OFFSCREEN = 16, CULL_NONFINITE = 32 };

typedef struct {
    int cull;
    float depth32;
    double t[3];
    double R[9], Sig[9], Sc[9];
    double xh, yh;
    int clx, cly;        /* guard clamp active */
    double J[6];
    double S2[3];        /* xx, xy, yy */
    double Q[3];         /* a, b, c */
    double mu[2];
    double rad[2];
    int rect[4];         /* px_lo, px_hi, py_lo, py_hi (inclusive) */
    int rect_margin;     /* a rect boundary is within 1e-6 px of a rounding step */
    double qn;           /* |q| */
    double qh[4];
} proj_t;

static float depth32_of(const double *w2c, const double *x) {
    /* FP32 FMA chain on FP32-rounded row 2 of W2C and the FP32 mean. */
    float a0 = (float)w2c[8], a1 = (float)w2c[9], a2 = (float)w2c[10], a3 = (float)w2c[11];
    return fmaf(a0, (float)x[0], fmaf(a1, (float)x[1], fmaf(a2, (float)x[2], a3)));
}

static int near_int(double v) {
    double r = floor(v + 0.5);
    return fabs(v - r) < 1e-6;
}

static void project_one(const or_settings *S, const double *x, const double *q, const double *s,
                        double o, const double *w2c, const double *intr, int Wimg, int Himg,
                        proj_t *P) {
    memset(P, 0, sizeof *P);
    double Wm[9] = {w2c[0], w2c[1], w2c[2], w2c[4], w2c[5], w2c[6], w2c[8], w2c[9], w2c[10]};
    double w[3] = {w2c[3], w2c[7], w2c[11]};
    int finite = isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(q[0]) &&
                 isfinite(q[1]) && isfinite(q[2]) && isfinite(q[3]) && isfinite(s[0]) &&
                 isfinite(s[1]) && isfinite(s[2]) && isfinite(o);
    if (!finite) { P->cull = CULL_NONFINITE; return; }
    mv3(Wm, x, P->t);
    for (int i = 0; i < 3; ++i) P->t[i] += w[i];
    P->depth32 = depth32_of(w2c, x);
    if (!(P->depth32 > (float)S->near_z)) { P->cull = CULL_NEAR; return; }
    if (P->depth32 > (float)S->far_z) { P->cull = CULL_FAR; return; }
    if (o < S->alpha_min) { P->cull = CULL_OPACITY; return; }
    double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    if (!(n2 >= 1e-24)) { P->cull = CULL_QUAT; return; }
    P->qn = sqrt(n2);
    for (int i = 0; i < 4; ++i) P->qh[i] = q[i] / P->qn;
    quat_to_R(P->qh, P->R);
    /* Sigma = R diag(s^2) R^T */
    double RS[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) RS[3 * i + j] = P->R[3 * i + j] * s[j] * s[j];
    mmt3(RS, P->R, P->Sig);
    /* Eq. (3) as a covariance: Sigma_c = W Sigma W^T */
    double WS[9];
    mm3(Wm, P->Sig, WS);
    mmt3(WS, Wm, P->Sc);
    double fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
    double tz = P->t[2];
    double lox = (-cx - S->guard * Wimg) / fx, hix = (Wimg - cx + S->guard * Wimg) / fx;
    double loy = (-cy - S->guard * Himg) / fy, hiy = (Himg - cy + S->guard * Himg) / fy;
    double rx = P->t[0] / tz, ry = P->t[1] / tz;
    P->xh = rx; P->yh = ry;
    if (rx < lox) { P->xh = lox; P->clx = 1; }
    if (rx > hix) { P->xh = hix; P->clx = 1; }
    if (ry < loy) { P->yh = loy; P->cly = 1; }
    if (ry > hiy) { P->yh = hiy; P->cly = 1; }
    double *J = P->J;
    J[0] = fx / tz; J[1] = 0.0; J[2] = -fx * P->xh / tz;
    J[3] = 0.0; J[4] = fy / tz; J[5] = -fy * P->yh / tz;
    /* Sigma2 = J Sc J^T + eps I */
    double JS[6];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            JS[3 * i + j] = J[3 * i] * P->Sc[j] + J[3 * i + 1] * P->Sc[3 + j] + J[3 * i + 2] * P->Sc[6 + j];
    double sxx = JS[0] * J[0] + JS[1] * J[1] + JS[2] * J[2];
    double sxy = JS[0] * J[3] + JS[1] * J[4] + JS[2] * J[5];
    double syy = JS[3] * J[3] + JS[4] * J[4] + JS[5] * J[5];
    sxx += S->eps2d;
    syy += S->eps2d;
    P->S2[0] = sxx; P->S2[1] = sxy; P->S2[2] = syy;
    double det = sxx * syy - sxy * sxy;
    P->Q[0] = syy / det;
    P->Q[1] = -sxy / det;
    P->Q[2] = sxx / det;
    P->mu[0] = fx * P->t[0] / tz + cx;
    P->mu[1] = fy * P->t[1] / tz + cy;
    /* opacity-aware footprint: alpha >= alpha_min  <=>  d^T Q d <= k^2 */
    double k2 = 2.0 * log(o / S->alpha_min);
    if (k2 < 0) k2 = 0;
    P->rad[0] = sqrt(k2 * sxx);
    P->rad[1] = sqrt(k2 * syy);
    double ex = P->rad[0] * (1.0 + S->pad_rel) + S->pad_px;
    double ey = P->rad[1] * (1.0 + S->pad_rel) + S->pad_px;
    double bx0 = P->mu[0] - 0.5 - ex, bx1 = P->mu[0] - 0.5 + ex;
    double by0 = P->mu[1] - 0.5 - ey, by1 = P->mu[1] - 0.5 + ey;
    P->rect_margin = near_int(bx0) || near_int(bx1) || near_int(by0) || near_int(by1);
    double fx0 = ceil(bx0), fx1 = floor(bx1), fy0 = ceil(by0), fy1 = floor(by1);
    if (fx0 < 0) fx0 = 0;
    if (fy0 < S->roi_y0) fy0 = S->roi_y0;  /* tiles are listed only inside the region of interest */
    if (fx1 > Wimg - 1) fx1 = Wimg - 1;
    if (fy1 > Himg - 1) fy1 = Himg - 1;
    if (!(fx0 <= fx1) || !(fy0 <= fy1)) { P->cull = CULL_OFFSCREEN; return; }
    P->rect[0] = (int)fx0; P->rect[1] = (int)fx1; P->rect[2] = (int)fy0; P->rect[3] = (int)fy1;
}

/* Single-Gaussian projection, exposed for the closed-form tests.
 * out[0..]: t[3], depth32, Sc[9], S2[3], Q[3], mu[2], rad[2], rect[4], cull, clx, cly, J[6] */
int or_project_one(const or_settings *S, const double *x, const double *q, const double *s, double o,
                   const double *w2c, const double *intr, int W, int H, double *out) {
    proj_t P;
    project_one(S, x, q, s, o, w2c, intr, W, H, &P);
    int n = 0;
    for (int i = 0; i < 3; ++i) out[n++] = P.t[i];
    out[n++] = (double)P.depth32;
    for (int i = 0; i < 9; ++i) out[n++] = P.Sc[i];
    for (int i = 0; i < 3; ++i) out[n++] = P.S2[i];
    for (int i = 0; i < 3; ++i) out[n++] = P.Q[i];
    for (int i = 0; i < 2; ++i) out[n++] = P.mu[i];
    for (int i = 0; i < 2; ++i) out[n++] = P.rad[i];
    for (int i = 0; i < 4; ++i) out[n++] = P.rect[i];
    out[n++] = P.cull;
    out[n++] = P.clx;
    out[n++] = P.cly;
    for (int i = 0; i < 6; ++i) out[n++] = P.J[i];
    return n;
}

/* ------------------------------------------------------------------------ */
/* per-view preparation: project every Gaussian, order visible ones          */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double *mean, *quat, *scale, *opac, *color; /* SoA planes of length G */
    int64_t G;
} or_gauss;

static void gx(const or_gauss *g, int64_t i, double *x, double *q, double *s) {
    int64_t G = g->G;
    for (int k = 0; k < 3; ++k) x[k] = g->mean[k * G + i];
    for (int k = 0; k < 4; ++k) q[k] = g->quat[k * G + i];
    for (int k = 0; k < 3; ++k) s[k] = g->scale[k * G + i];
}

typedef struct {
    int64_t n;        /* visible count */
    int64_t *ids;     /* visible Gaussian ids in (depth32, id) order */
    proj_t *P;        /* per Gaussian (size G) */
} view_prep;

static const float *g_sort_depth;
static int cmp_depth_id(const void *a, const void *b) {
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    float di = g_sort_depth[i], dj = g_sort_depth[j];
    if (di < dj) return -1;
    if (di > dj) return 1;
    return (i < j) ? -1 : (i > j);
}

static void prep_view(const or_settings *S, const or_gauss *g, const double *w2c, const double *intr,
                      int W, int H, view_prep *vp) {
    int64_t G = g->G;
    vp->P = (proj_t *)malloc(sizeof(proj_t) * (size_t)(G > 0 ? G : 1));
    float *dep = (float *)malloc(sizeof(float) * (size_t)(G > 0 ? G : 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < G; ++i) {
        double x[3], q[4], s[3];
        gx(g, i, x, q, s);
        project_one(S, x, q, s, g->opac[i], w2c, intr, W, H, &vp->P[i]);
        dep[i] = vp->P[i].depth32;
    }
    int64_t n = 0;
    for (int64_t i = 0; i < G; ++i) n += (vp->P[i].cull == CULL_NONE);
    vp->n = n;
    vp->ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    n = 0;
    for (int64_t i = 0; i < G; ++i)
        if (vp->P[i].cull == CULL_NONE) vp->ids[n++] = i;
    g_sort_depth = dep;
    qsort(vp->ids, (size_t)n, sizeof(int64_t), cmp_depth_id);
    g_sort_depth = NULL;
    free(dep);
}

static void free_view(view_prep *vp) {
    free(vp->P);
    free(vp->ids);
}

/* per-row candidate lists (AABB pruning); rows[y] lists positions into vp->ids */
typedef struct {
    int64_t *start; /* H+1 */
    int64_t *pos;
} row_lists;

static void build_rows(const view_prep *vp, int H, row_lists *rl) {
    rl->start = (int64_t *)calloc((size_t)H + 1, sizeof(int64_t));
    for (int64_t j = 0; j < vp->n; ++j) {
        const proj_t *P = &vp->P[vp->ids[j]];
        for (int y = P->rect[2]; y <= P->rect[3]; ++y) rl->start[y + 1]++;
    }
    for (int y = 0; y < H; ++y) rl->start[y + 1] += rl->start[y];
    rl->pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(rl->start[H] > 0 ? rl->start[H] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)H);
    for (int y = 0; y < H; ++y) fill[y] = rl->start[y];
    for (int64_t j = 0; j < vp->n; ++j) {
        const proj_t *P = &vp->P[vp->ids[j]];
        for (int y = P->rect[2]; y <= P->rect[3]; ++y) rl->pos[fill[y]++] = j;
    }
    free(fill);
}

static void free_rows(row_lists *rl) {
    free(rl->start);
    free(rl->pos);
}

/* ------------------------------------------------------------------------ */
/* compositing of one pixel                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t g;
    double alpha, e, dx, dy, T;   /* T before the blend */
    int clamped;                  /* alpha hit alpha_max */
} stack_e;

typedef struct {
    int64_t g;   /* Gaussian id of a flagged decision */
    int kind;    /* 0: alpha_min skip, 1: t_min stop */
    int nominal; /* outcome taken: 1 = skip / stop */
} flag_e;

typedef struct {
    double C[3], T;
    int64_t last;
    int nflag;          /* flagged decisions (capped) */
    int nkink;          /* blends whose alpha sits within the margin of alpha_max */
    flag_e flags[8];
    uint64_t hash;
    int64_t n_eval, n_blend;
} pix_out;

static inline uint64_t fnv(uint64_t h, uint64_t v) {
    for (int i = 0; i < 8; ++i) {
        h ^= (v >> (8 * i)) & 0xff;
        h *= 1099511628211ULL;
    }
    return h;
}

/*
 * Composite one pixel.  Candidate list: either all visible Gaussians (brute force)
 * or the row list with the rect test (pruned).  `force` lists decisions whose
 * outcome is inverted (alternatives at threshold margins).  When `stk` is given
 * the contributing Gaussians are recorded in order.
 */
static void composite(const or_settings *S, const or_gauss *g, const view_prep *vp,
                      const row_lists *rl, int x, int y, const flag_e *force, int nforce,
                      pix_out *out, stack_e *stk, int64_t *nstk) {
    double px = x + 0.5, py = y + 0.5;
    double T = 1.0, C[3] = {0, 0, 0};
    int64_t last = -1, ns = 0;
    out->nflag = 0;
    out->nkink = 0;
    out->hash = 1469598103934665603ULL;
    out->n_eval = 0;
    out->n_blend = 0;
    int64_t j0 = 0, j1 = vp->n;
    if (rl) { j0 = rl->start[y]; j1 = rl->start[y + 1]; }
    for (int64_t jj = j0; jj < j1; ++jj) {
        int64_t j = rl ? rl->pos[jj] : jj;
        int64_t id = vp->ids[j];
        const proj_t *P = &vp->P[id];
        if (rl && (x < P->rect[0] || x > P->rect[1])) continue;
        out->n_eval++;
        double dx = px - P->mu[0], dy = py - P->mu[1];
        double power = -0.5 * (P->Q[0] * dx * dx + 2.0 * P->Q[1] * dx * dy + P->Q[2] * dy * dy);
        double e = exp(power);
        double av = g->opac[id] * e;
        int clamped = av >= S->alpha_max;
        if (fabs(av - S->alpha_max) <= S->margin * S->alpha_max) out->nkink++;
        double alpha = clamped ? S->alpha_max : av;
        int skip = alpha < S->alpha_min;
        if (fabs(alpha - S->alpha_min) <= S->margin * S->alpha_min) {
            if (out->nflag < 8) { out->flags[out->nflag].g = id; out->flags[out->nflag].kind = 0; out->flags[out->nflag].nominal = skip; }
            out->nflag++;
        }
        for (int f = 0; f < nforce; ++f)
            if (force[f].g == id && force[f].kind == 0) skip = !force[f].nominal;
        if (skip) continue;
        double Tn = T * (1.0 - alpha);
        int stop = Tn < S->t_min;
        if (fabs(Tn - S->t_min) <= S->margin * S->t_min) {
            if (out->nflag < 8) { out->flags[out->nflag].g = id; out->flags[out->nflag].kind = 1; out->flags[out->nflag].nominal = stop; }
            out->nflag++;
        }
        for (int f = 0; f < nforce; ++f)
            if (force[f].g == id && force[f].kind == 1) stop = !force[f].nominal;
        out->hash = fnv(out->hash, (uint64_t)id * 4 + (uint64_t)(stop ? 1 : 0) * 2 + (uint64_t)clamped);
        if (stop) break;
        if (stk) {
            stk[ns].g = id; stk[ns].alpha = alpha; stk[ns].e = e; stk[ns].dx = dx; stk[ns].dy = dy;
            stk[ns].T = T; stk[ns].clamped = clamped;
        }
        ns++;
        for (int c = 0; c < 3; ++c) C[c] += g->color[c * g->G + id] * alpha * T;
        T = Tn;
        last = id;
        out->n_blend++;
    }
    for (int c = 0; c < 3; ++c) out->C[c] = C[c] + T * S->bg[c];
    out->T = T;
    out->last = last;
    if (nstk) *nstk = ns;
}

/* ------------------------------------------------------------------------ */
/* render                                                                     */
/* ------------------------------------------------------------------------ */
/*
 * img[V][3][H][W], Tf[V][H][W], last[V][H][W] (Gaussian id or -1).
 * Optional (may be NULL): nflag[V][H][W] (number of flagged threshold decisions;
 * alternatives are produced when 1 <= nflag <= 2), nalt[V][H][W],
 * alt[V][H][W][4][5] = (R, G, B, T, last) for every outcome of the flagged
 * decisions (index 0 is the nominal one).  stats[4]: evaluated pairs, blended
 * pairs, visible (view, Gaussian) pairs, flagged pixels.  Returns the decision
 * hash through *hash; optionally the per-pixel decision hash pixhash[V][H][W]
 * (blend/stop/clamp sequence), the per-view cull/guard-clamp hash gausshash[V],
 * and kink[V][H][W]: the number of blends whose unclamped alpha lies within the
 * margin of alpha_max (the image is continuous there but its derivative is not).
 */
int or_render(const or_settings *S, int64_t G, const double *mean, const double *quat,
              const double *scale, const double *opac, const double *color,
              int V, const double *w2c, const double *intr, int W, int H, int pruned,
              double *img, double *Tf, int64_t *last, int8_t *nflag, int8_t *nalt, double *alt,
              int64_t *stats, uint64_t *hash, uint64_t *pixhash, uint64_t *gausshash, int8_t *kink) {
    or_gauss g = {mean, quat, scale, opac, color, G};
    int64_t st_eval = 0, st_blend = 0, st_vis = 0, st_flag = 0;
    uint64_t h = 0;
    for (int v = 0; v < V; ++v) {
        view_prep vp;
        prep_view(S, &g, w2c + 12 * v, intr + 4 * v, W, H, &vp);
        st_vis += vp.n;
        uint64_t hv = 0;
        for (int64_t i = 0; i < G; ++i)
            hv = fnv(hv, (uint64_t)vp.P[i].cull * 4 + (uint64_t)vp.P[i].clx * 2 + (uint64_t)vp.P[i].cly);
        if (gausshash) gausshash[v] = hv;
        row_lists rl;
        if (pruned) build_rows(&vp, H, &rl);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : st_eval, st_blend, st_flag) reduction(^ : hv)
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                pix_out po;
                if (y >= S->roi_y0) {
                    composite(S, &g, &vp, pruned ? &rl : NULL, x, y, NULL, 0, &po, NULL, NULL);
                } else {  /* outside the region of interest: not rendered, background */
                    memset(&po, 0, sizeof po);
                    for (int c = 0; c < 3; ++c) po.C[c] = S->bg[c];
                    po.T = 1.0;
                    po.last = -1;
                }
                size_t p = (size_t)y * W + x;
                size_t vo = (size_t)v * H * W;
                for (int c = 0; c < 3; ++c) img[(size_t)v * 3 * H * W + (size_t)c * H * W + p] = po.C[c];
                Tf[vo + p] = po.T;
                last[vo + p] = po.last;
                st_eval += po.n_eval;
                st_blend += po.n_blend;
                hv ^= fnv(po.hash, (uint64_t)(vo + p));
                if (pixhash) pixhash[vo + p] = po.hash;
                int nf = po.nflag;
                if (nflag) nflag[vo + p] = (int8_t)(nf > 100 ? 100 : nf);
                if (kink) kink[vo + p] = (int8_t)(po.nkink > 100 ? 100 : po.nkink);
                if (nf > 0) st_flag++;
                if (nalt && alt) {
                    double *a = alt + (vo + p) * 20;
                    int na = 1;
                    a[0] = po.C[0]; a[1] = po.C[1]; a[2] = po.C[2]; a[3] = po.T; a[4] = (double)po.last;
                    if (nf >= 1 && nf <= 2) {
                        for (int m = 1; m < (1 << nf); ++m) {
                            flag_e fz[2];
                            int nfz = 0;
                            for (int b = 0; b < nf; ++b)
                                if (m & (1 << b)) fz[nfz++] = po.flags[b];
                            pix_out pa;
                            composite(S, &g, &vp, pruned ? &rl : NULL, x, y, fz, nfz, &pa, NULL, NULL);
                            double *aa = a + 5 * na;
                            aa[0] = pa.C[0]; aa[1] = pa.C[1]; aa[2] = pa.C[2]; aa[3] = pa.T; aa[4] = (double)pa.last;
                            na++;
                        }
                    }
                    nalt[vo + p] = (int8_t)(nf > 2 ? 0 : na);
                }
            }
        }
        h = fnv(h, hv);
        if (pruned) free_rows(&rl);
        free_view(&vp);
    }
    if (stats) { stats[0] = st_eval; stats[1] = st_blend; stats[2] = st_vis; stats[3] = st_flag; }
    if (hash) *hash = h;
    return 0;
}

/* Per (view, Gaussian) projection outputs for the binning reference.
 * vis[V*G] (cull code, 0 = visible), depth32[V*G], mu[V*G*2], conic[V*G*3],
 * rect[V*G*4], rect_margin[V*G]. */
int or_project_all(const or_settings *S, int64_t G, const double *mean, const double *quat,
                   const double *scale, const double *opac, int V, const double *w2c,
                   const double *intr, int W, int H, int8_t *cull, float *depth32, double *mu,
                   double *conic, int32_t *rect, int8_t *rect_margin) {
    or_gauss g = {mean, quat, scale, opac, NULL, G};
    for (int v = 0; v < V; ++v) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < G; ++i) {
            double x[3], q[4], s[3];
            gx(&g, i, x, q, s);
            proj_t P;
            project_one(S, x, q, s, opac[i], w2c + 12 * v, intr + 4 * v, W, H, &P);
            size_t o = (size_t)v * G + i;
            cull[o] = (int8_t)P.cull;
            depth32[o] = P.depth32;
            mu[2 * o] = P.mu[0]; mu[2 * o + 1] = P.mu[1];
            conic[3 * o] = P.Q[0]; conic[3 * o + 1] = P.Q[1]; conic[3 * o + 2] = P.Q[2];
            for (int k = 0; k < 4; ++k) rect[4 * o + k] = P.rect[k];
            rect_margin[o] = (int8_t)P.rect_margin;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* gradient                                                                   */
/* ------------------------------------------------------------------------ */
/*
 * Exact adjoint of the render for a given dL/dimg[V][3][H][W].  Outputs (all
 * overwritten): dquat[4][G], dscale[3][G], dopac[G], dcolor[3][G], dmean[3][G],
 * dw2c[V][12].  Pixels listed with mask[V][H][W] != 0 are left out (their
 * dL/dimg is treated as zero).  The per-pixel stack of contributing Gaussians
 * is stored explicitly and walked backwards; transmittances are the forward
 * products, never recovered by division.
 */
int or_grad(const or_settings *S, int64_t G, const double *mean, const double *quat,
            const double *scale, const double *opac, const double *color,
            int V, const double *w2c, const double *intr, int W, int H,
            const double *dimg, const int8_t *mask,
            double *dquat, double *dscale, double *dopac, double *dcolor, double *dmean,
            double *dw2c) {
    or_gauss g = {mean, quat, scale, opac, color, G};
    memset(dquat, 0, sizeof(double) * 4 * G);
    memset(dscale, 0, sizeof(double) * 3 * G);
    memset(dopac, 0, sizeof(double) * G);
    memset(dcolor, 0, sizeof(double) * 3 * G);
    memset(dmean, 0, sizeof(double) * 3 * G);
    memset(dw2c, 0, sizeof(double) * 12 * V);
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    /* per-thread 2-D accumulators: mu(2), conic(3), opacity(1), colour(3) */
    double *acc = (double *)malloc(sizeof(double) * 9 * (size_t)(G > 0 ? G : 1) * nth);
    for (int v = 0; v < V; ++v) {
        view_prep vp;
        const double *M = w2c + 12 * v;
        prep_view(S, &g, M, intr + 4 * v, W, H, &vp);
        row_lists rl;
        build_rows(&vp, H, &rl);
        memset(acc, 0, sizeof(double) * 9 * (size_t)G * nth);
#pragma omp parallel
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double *A = acc + (size_t)tid * 9 * G;
            stack_e *stk = (stack_e *)malloc(sizeof(stack_e) * (size_t)(vp.n > 0 ? vp.n : 1));
#pragma omp for schedule(dynamic, 1)
            for (int y = 0; y < H; ++y) {
                if (y < S->roi_y0) continue;  /* not rendered */
                for (int x = 0; x < W; ++x) {
                    size_t p = (size_t)y * W + x;
                    if (mask && mask[(size_t)v * H * W + p]) continue;
                    double gC[3];
                    for (int c = 0; c < 3; ++c) gC[c] = dimg[(size_t)v * 3 * H * W + (size_t)c * H * W + p];
                    if (gC[0] == 0.0 && gC[1] == 0.0 && gC[2] == 0.0) continue;
                    pix_out po;
                    int64_t ns = 0;
                    composite(S, &g, &vp, &rl, x, y, NULL, 0, &po, stk, &ns);
                    double Ssum[3];
                    for (int c = 0; c < 3; ++c) Ssum[c] = po.T * S->bg[c];
                    for (int64_t j = ns - 1; j >= 0; --j) {
                        const stack_e *E = &stk[j];
                        int64_t id = E->g;
                        double *a = A + 9 * id;
                        double col[3] = {color[id], color[G + id], color[2 * G + id]};
                        double w = E->alpha * E->T;
                        double dalpha = 0.0;
                        for (int c = 0; c < 3; ++c) {
                            a[6 + c] += w * gC[c];
                            dalpha += gC[c] * (col[c] * E->T - Ssum[c] / (1.0 - E->alpha));
                            Ssum[c] += col[c] * w;
                        }
                        if (!E->clamped) {
                            const proj_t *P = &vp.P[id];
                            a[5] += dalpha * E->e;
                            double dpow = dalpha * E->alpha;
                            double dx = E->dx, dy = E->dy;
                            a[2] += dpow * (-0.5 * dx * dx);
                            a[3] += dpow * (-dx * dy);
                            a[4] += dpow * (-0.5 * dy * dy);
                            a[0] += dpow * (P->Q[0] * dx + P->Q[1] * dy);
                            a[1] += dpow * (P->Q[1] * dx + P->Q[2] * dy);
                        }
                    }
                }
            }
            free(stk);
        }
        for (int t = 1; t < nth; ++t)
            for (size_t i = 0; i < (size_t)9 * G; ++i) acc[i] += acc[(size_t)t * 9 * G + i];
        /* chain rule per visible Gaussian */
        double Wm[9] = {M[0], M[1], M[2], M[4], M[5], M[6], M[8], M[9], M[10]};
        double GWv[9] = {0}, gwv[3] = {0};
        const double *in = intr + 4 * v;
        double fx = in[0], fy = in[1];
        for (int64_t jj = 0; jj < vp.n; ++jj) {
            int64_t id = vp.ids[jj];
            const proj_t *P = &vp.P[id];
            const double *a = acc + 9 * id;
            double x[3], q[4], s[3];
            gx(&g, id, x, q, s);
            for (int c = 0; c < 3; ++c) dcolor[c * G + id] += a[6 + c];
            dopac[id] += a[5];
            /* conic -> Sigma2 : dL/dS2 = -Q GQ Q, GQ = [[ga, gb/2],[gb/2, gc]] */
            double Qm[4] = {P->Q[0], P->Q[1], P->Q[1], P->Q[2]};
            double GQ[4] = {a[2], 0.5 * a[3], 0.5 * a[3], a[4]};
            double T1[4], G2[4];
            for (int i = 0; i < 2; ++i)
                for (int k = 0; k < 2; ++k) T1[2 * i + k] = Qm[2 * i] * GQ[k] + Qm[2 * i + 1] * GQ[2 + k];
            for (int i = 0; i < 2; ++i)
                for (int k = 0; k < 2; ++k) G2[2 * i + k] = -(T1[2 * i] * Qm[k] + T1[2 * i + 1] * Qm[2 + k]);
            /* Sigma2 = J Sc J^T + eps I : dL/dSc = J^T G2 J ; dL/dJ = 2 G2 J Sc */
            const double *J = P->J;
            double G2J[6];
            for (int i = 0; i < 2; ++i)
                for (int k = 0; k < 3; ++k) G2J[3 * i + k] = G2[2 * i] * J[k] + G2[2 * i + 1] * J[3 + k];
            double GSc[9];
            for (int i = 0; i < 3; ++i)
                for (int k = 0; k < 3; ++k) GSc[3 * i + k] = J[i] * G2J[k] + J[3 + i] * G2J[3 + k];
            double GJ[6];
            for (int i = 0; i < 2; ++i)
                for (int k = 0; k < 3; ++k)
                    GJ[3 * i + k] = 2.0 * (G2J[3 * i] * P->Sc[k] + G2J[3 * i + 1] * P->Sc[3 + k] + G2J[3 * i + 2] * P->Sc[6 + k]);
            /* t -> mu, J */
            double tx = P->t[0], ty = P->t[1], tz = P->t[2];
            double gt[3] = {0, 0, 0};
            gt[0] += a[0] * fx / tz;
            gt[2] += -a[0] * fx * tx / (tz * tz);
            gt[1] += a[1] * fy / tz;
            gt[2] += -a[1] * fy * ty / (tz * tz);
            gt[2] += GJ[0] * (-fx / (tz * tz)) + GJ[4] * (-fy / (tz * tz));
            if (!P->clx) {
                gt[0] += GJ[2] * (-fx / (tz * tz));
                gt[2] += GJ[2] * (2.0 * fx * tx / (tz * tz * tz));
            } else {
                gt[2] += GJ[2] * (fx * P->xh / (tz * tz));
            }
            if (!P->cly) {
                gt[1] += GJ[5] * (-fy / (tz * tz));
                gt[2] += GJ[5] * (2.0 * fy * ty / (tz * tz * tz));
            } else {
                gt[2] += GJ[5] * (fy * P->yh / (tz * tz));
            }
            /* Sc = W Sig W^T : dL/dSig = W^T GSc W ; dL/dW += 2 GSc W Sig */
            double T2[9], GSig[9], WSig[9], GWa[9];
            mtm3(Wm, GSc, T2);
            mm3(T2, Wm, GSig);
            mm3(Wm, P->Sig, WSig);
            mm3(GSc, WSig, GWa);
            for (int i = 0; i < 9; ++i) GWv[i] += 2.0 * GWa[i];
            /* t = W x + w */
            for (int i = 0; i < 3; ++i) {
                for (int k = 0; k < 3; ++k) GWv[3 * i + k] += gt[i] * x[k];
                gwv[i] += gt[i];
            }
            double gx3[3];
            mtv3(Wm, gt, gx3);
            for (int k = 0; k < 3; ++k) dmean[k * G + id] += gx3[k];
            /* Sig = R diag(s^2) R^T : dL/dR = 2 GSig R S^2 ; dL/ds_k = 2 s_k (R^T GSig R)_kk */
            double GR[9], RtGR[9], GSR[9];
            mm3(GSig, P->R, GSR);
            for (int i = 0; i < 3; ++i)
                for (int k = 0; k < 3; ++k) GR[3 * i + k] = 2.0 * GSR[3 * i + k] * s[k] * s[k];
            mtm3(P->R, GSR, RtGR);
            for (int k = 0; k < 3; ++k) dscale[k * G + id] += 2.0 * s[k] * RtGR[4 * k];
            /* R(q_hat) -> q_hat */
            double w = P->qh[0], qx = P->qh[1], qy = P->qh[2], qz = P->qh[3];
            double gq[4];
            gq[0] = 2.0 * (-qz * GR[1] + qy * GR[2] + qz * GR[3] - qx * GR[5] - qy * GR[6] + qx * GR[7]);
            gq[1] = 2.0 * (qy * GR[1] + qz * GR[2] + qy * GR[3] - 2.0 * qx * GR[4] - w * GR[5] + qz * GR[6] + w * GR[7] - 2.0 * qx * GR[8]);
            gq[2] = 2.0 * (-2.0 * qy * GR[0] + qx * GR[1] + w * GR[2] + qx * GR[3] + qz * GR[5] - w * GR[6] + qz * GR[7] - 2.0 * qy * GR[8]);
            gq[3] = 2.0 * (-2.0 * qz * GR[0] - w * GR[1] + qx * GR[2] + w * GR[3] - 2.0 * qz * GR[4] + qy * GR[5] + qx * GR[6] + qy * GR[7]);
            /* normalisation q_hat = q / |q| */
            double dot = w * gq[0] + qx * gq[1] + qy * gq[2] + qz * gq[3];
            for (int k = 0; k < 4; ++k) dquat[k * G + id] += (gq[k] - P->qh[k] * dot) / P->qn;
        }
        for (int i = 0; i < 3; ++i) {
            for (int k = 0; k < 3; ++k) dw2c[12 * v + 4 * i + k] = GWv[3 * i + k];
            dw2c[12 * v + 4 * i + 3] = gwv[i];
        }
        free_rows(&rl);
        free_view(&vp);
    }
    free(acc);
    return 0;
}

/* Per-pixel contributor stack of one pixel (for invariance tests).
 * out rows of 4: (gid, alpha, T_before, clamped); returns the count (<= cap). */
int64_t or_pixel_stack(const or_settings *S, int64_t G, const double *mean, const double *quat,
                       const double *scale, const double *opac, const double *color,
                       const double *w2c, const double *intr, int W, int H, int x, int y,
                       double *out, int64_t cap) {
    or_gauss g = {mean, quat, scale, opac, color, G};
    view_prep vp;
    prep_view(S, &g, w2c, intr, W, H, &vp);
    stack_e *stk = (stack_e *)malloc(sizeof(stack_e) * (size_t)(vp.n > 0 ? vp.n : 1));
    pix_out po;
    int64_t ns = 0;
    composite(S, &g, &vp, NULL, x, y, NULL, 0, &po, stk, &ns);
    int64_t n = ns < cap ? ns : cap;
    for (int64_t i = 0; i < n; ++i) {
        out[4 * i] = (double)stk[i].g;
        out[4 * i + 1] = stk[i].alpha;
        out[4 * i + 2] = stk[i].T;
        out[4 * i + 3] = stk[i].clamped;
    }
    free(stk);
    free_view(&vp);
    return ns;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
