// pose.hip -- camera poses from the interpolated LiDAR trajectory and their adjoint.
//
// Paper Sec. III-A: the LiDAR trajectory is continuous in time, with linear
// interpolation of the translation and SLERP of the rotation between the
// timestamped LiDAR poses; Eq. (1) composes it with the camera->LiDAR extrinsic
// at the shifted time t + delta; Eq. (2) uses the inverse (world->camera).
//
// Everything here is float64: the outputs feed both the float64 projection and
// the float32 depth key.  The work is tiny (one thread per view / camera).
#include "common.hpp"

namespace splat {
namespace {

struct Q4 {
    double w, x, y, z;
};

__device__ inline Q4 qmul(const Q4 &a, const Q4 &b) {
    return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
            a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}

__device__ inline Q4 qnorm(Q4 q) {
    double n = sqrt(q.w * q.w + q.x * q.x + q.y * q.y + q.z * q.z);
    return {q.w / n, q.x / n, q.y / n, q.z / n};
}

// rotation matrix (row-major) of a unit quaternion
__device__ inline void qmat(const Q4 &q, double *R) {
    double xx = q.x * q.x, yy = q.y * q.y, zz = q.z * q.z;
    double xy = q.x * q.y, xz = q.x * q.z, yz = q.y * q.z, wx = q.w * q.x, wy = q.w * q.y, wz = q.w * q.z;
    R[0] = 1.0 - 2.0 * (yy + zz); R[1] = 2.0 * (xy - wz); R[2] = 2.0 * (xz + wy);
    R[3] = 2.0 * (xy + wz); R[4] = 1.0 - 2.0 * (xx + zz); R[5] = 2.0 * (yz - wx);
    R[6] = 2.0 * (xz - wy); R[7] = 2.0 * (yz + wx); R[8] = 1.0 - 2.0 * (xx + yy);
}

// unit quaternion of the rotation vector v (exponential map)
__device__ inline Q4 qexp(const double *v) {
    double a = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double h = 0.5 * a;
    double s = (a < 1e-8) ? 0.5 - a * a / 48.0 : sin(h) / a;  // sin(a/2)/a
    return {cos(h), s * v[0], s * v[1], s * v[2]};
}

// rotation vector of a unit quaternion (shortest arc)
__device__ inline void qlog(Q4 q, double *v) {
    if (q.w < 0) q = {-q.w, -q.x, -q.y, -q.z};
    double n = sqrt(q.x * q.x + q.y * q.y + q.z * q.z);
    double f = (n < 1e-12) ? 2.0 / q.w : 2.0 * atan2(n, q.w) / n;
    v[0] = f * q.x;
    v[1] = f * q.y;
    v[2] = f * q.z;
}

__device__ inline void matmul3(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i + 0] * B[0 + j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

struct PoseEval {
    int k;
    double dt;
    double Rs[9], ps[3];   // LiDAR pose at s
    double om[3];          // rotation vector of the segment (R_k^T R_k+1)
    double vel[3];         // (p_k+1 - p_k)
    double Re[9], te[3];   // extrinsic camera->LiDAR
    double Rcw[9], pcw[3]; // camera->world
    bool extrapolated;
};

__device__ void eval_pose(int K, const double *kt, const double *kq, const double *kp, const double *R0,
                          const double *t0, const double *xi, double s, PoseEval &P) {
    // largest k with t_k <= s, clamped to [0, K-2]
    int lo = 0, hi = K - 1;
    if (s < kt[0]) {
        hi = 0;
    } else {
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (kt[mid] <= s) lo = mid; else hi = mid - 1;
        }
    }
    int k = min(max(lo, 0), K - 2);
    P.k = k;
    P.extrapolated = (s < kt[0]) || (s > kt[K - 1]);
    P.dt = kt[k + 1] - kt[k];
    double u = (s - kt[k]) / P.dt;
    Q4 qa = qnorm({kq[4 * k], kq[4 * k + 1], kq[4 * k + 2], kq[4 * k + 3]});
    Q4 qb = qnorm({kq[4 * k + 4], kq[4 * k + 5], kq[4 * k + 6], kq[4 * k + 7]});
    Q4 qrel = qmul({qa.w, -qa.x, -qa.y, -qa.z}, qb);
    qlog(qrel, P.om);
    double hv[3] = {u * P.om[0], u * P.om[1], u * P.om[2]};
    Q4 qs = qmul(qa, qexp(hv));  // SLERP on the shortest arc
    qmat(qs, P.Rs);
    for (int i = 0; i < 3; ++i) {
        P.vel[i] = kp[3 * (k + 1) + i] - kp[3 * k + i];
        P.ps[i] = kp[3 * k + i] + u * P.vel[i];
    }
    double Rphi[9];
    qmat(qexp(xi + 3), Rphi);
    matmul3(R0, Rphi, P.Re);
    for (int i = 0; i < 3; ++i) P.te[i] = t0[i] + xi[i];
    matmul3(P.Rs, P.Re, P.Rcw);
    for (int i = 0; i < 3; ++i)
        P.pcw[i] = P.Rs[3 * i] * P.te[0] + P.Rs[3 * i + 1] * P.te[1] + P.Rs[3 * i + 2] * P.te[2] + P.ps[i];
}

__global__ void pose_fwd_kernel(int K, const double *kt, const double *kq, const double *kp, int C,
                                const double *R0, const double *t0, const double *xi,
                                const double *delta, int V, const int32_t *vcam, const double *vt,
                                double *w2c, uint32_t *status) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    int c = vcam[v];
    if (c < 0 || c >= C) return;  // validated on the host for host-visible inputs
    PoseEval P;
    eval_pose(K, kt, kq, kp, R0 + 9 * c, t0 + 3 * c, xi + 6 * c, vt[v] + delta[c], P);
    if (P.extrapolated && status) atomicOr(status, SPLAT_ST_EXTRAPOLATED);
    double *o = w2c + 12 * v;
    for (int i = 0; i < 3; ++i) {
        // W = Rcw^T, w = -Rcw^T pcw
        o[4 * i + 0] = P.Rcw[i];
        o[4 * i + 1] = P.Rcw[3 + i];
        o[4 * i + 2] = P.Rcw[6 + i];
        o[4 * i + 3] = -(P.Rcw[i] * P.pcw[0] + P.Rcw[3 + i] * P.pcw[1] + P.Rcw[6 + i] * P.pcw[2]);
    }
}

// right Jacobian of SO(3) (row-major)
__device__ void right_jacobian(const double *p, double *J) {
    double t2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    double t = sqrt(t2);
    double a, b;
    if (t < 1e-5) {
        a = 0.5 - t2 / 24.0;
        b = 1.0 / 6.0 - t2 / 120.0;
    } else {
        a = (1.0 - cos(t)) / t2;
        b = (t - sin(t)) / (t2 * t);
    }
    double K[9] = {0.0, -p[2], p[1], p[2], 0.0, -p[0], -p[1], p[0], 0.0};
    double K2[9];
    matmul3(K, K, K2);
    for (int i = 0; i < 9; ++i) J[i] = ((i == 0 || i == 4 || i == 8) ? 1.0 : 0.0) - a * K[i] + b * K2[i];
}

// one workgroup per camera, one thread per view (strided); the per-thread sums are
// combined by a fixed-order tree, so the result does not depend on timing
constexpr int POSE_BWD_T = 256;

__global__ __launch_bounds__(POSE_BWD_T) void pose_bwd_kernel(int K, const double *kt, const double *kq,
                                                             const double *kp, int C, const double *R0,
                                                             const double *t0, const double *xi,
                                                             const double *delta, int V, const int32_t *vcam,
                                                             const double *vt, const double *dw2c, double *dxi,
                                                             double *ddelta) {
    __shared__ double red[7][POSE_BWD_T];
    int c = blockIdx.x;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int v = threadIdx.x; v < V; v += POSE_BWD_T) {
        if (vcam[v] != c) continue;
        PoseEval P;
        eval_pose(K, kt, kq, kp, R0 + 9 * c, t0 + 3 * c, xi + 6 * c, vt[v] + delta[c], P);
        const double *g = dw2c + 12 * v;
        // W = Rcw^T: dL/dRcw[i][j] = gW[j][i];  w = -Rcw^T pcw: dL/dRcw[i][j] -= pcw[i] gw[j]
        double gR[9], gp[3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) gR[3 * i + j] = g[4 * j + i] - P.pcw[i] * g[4 * j + 3];
        for (int i = 0; i < 3; ++i)
            gp[i] = -(P.Rcw[3 * i] * g[3] + P.Rcw[3 * i + 1] * g[7] + P.Rcw[3 * i + 2] * g[11]);
        // Rcw = Rs Re, pcw = Rs te + ps
        double gRs[9], gRe[9], gte[3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double a = 0.0, b = 0.0;
                for (int k = 0; k < 3; ++k) {
                    a += gR[3 * i + k] * P.Re[3 * j + k];   // gR Re^T
                    b += P.Rs[3 * k + i] * gR[3 * k + j];   // Rs^T gR
                }
                gRs[3 * i + j] = a + gp[i] * P.te[j];
                gRe[3 * i + j] = b;
            }
        for (int i = 0; i < 3; ++i) gte[i] = P.Rs[i] * gp[0] + P.Rs[3 + i] * gp[1] + P.Rs[6 + i] * gp[2];
        for (int i = 0; i < 3; ++i) acc[i] += gte[i];
        // Re = R0 Exp(phi): perturbation Re Exp(Jr dphi); <gRe, Re [v]x> = v . vee(Re^T gRe - (.)^T)
        double M[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                M[3 * i + j] = P.Re[i] * gRe[j] + P.Re[3 + i] * gRe[3 + j] + P.Re[6 + i] * gRe[6 + j];
        double vv[3] = {M[7] - M[5], M[2] - M[6], M[3] - M[1]};
        double J[9];
        right_jacobian(xi + 6 * c + 3, J);
        for (int i = 0; i < 3; ++i) acc[3 + i] += J[i] * vv[0] + J[3 + i] * vv[1] + J[6 + i] * vv[2];
        // s = t + delta: dRs/ds = Rs [om]x / dt, dps/ds = vel / dt
        double N[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                N[3 * i + j] = P.Rs[i] * gRs[j] + P.Rs[3 + i] * gRs[3 + j] + P.Rs[6 + i] * gRs[6 + j];
        double wv[3] = {N[7] - N[5], N[2] - N[6], N[3] - N[1]};
        double ds = 0.0;
        for (int i = 0; i < 3; ++i) ds += wv[i] * P.om[i] + gp[i] * P.vel[i];
        acc[6] += ds / P.dt;
    }
    for (int i = 0; i < 7; ++i) red[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int s = POSE_BWD_T / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int i = 0; i < 7; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int i = 0; i < 6; ++i) dxi[6 * c + i] += red[i][0];
        ddelta[c] += red[6][0];
    }
}

}  // namespace

int launch_pose_fwd(int32_t K, const double *kt, const double *kq, const double *kp, int32_t C,
                    const double *R0, const double *t0, const double *xi, const double *delta,
                    int32_t V, const int32_t *vcam, const double *vt, double *w2c, uint32_t *status,
                    hipStream_t st) {
    int nb = (V + 63) / 64;
    hipLaunchKernelGGL(pose_fwd_kernel, dim3(nb), dim3(64), 0, st, K, kt, kq, kp, C, R0, t0, xi, delta,
                       V, vcam, vt, w2c, status);
    return launch_status("pose_fwd");
}

int launch_pose_bwd(int32_t K, const double *kt, const double *kq, const double *kp, int32_t C,
                    const double *R0, const double *t0, const double *xi, const double *delta,
                    int32_t V, const int32_t *vcam, const double *vt, const double *dw2c,
                    double *dxi, double *ddelta, hipStream_t st) {
    hipLaunchKernelGGL(pose_bwd_kernel, dim3(C), dim3(POSE_BWD_T), 0, st, K, kt, kq, kp, C, R0, t0, xi, delta,
                       V, vcam, vt, dw2c, dxi, ddelta);
    return launch_status("pose_bwd");
}

}  // namespace splat
