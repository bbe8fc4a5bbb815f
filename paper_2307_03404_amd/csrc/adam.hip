// Tracking updates, one lane per frame, in FP64 on the device, each ending in
// the left retraction c2w <- exp(xi^) c2w:
//  * Adam on the se(3) tangent of a left, world-frame perturbation;
//  * a damped Gauss-Newton step from the per-frame normal equations.
// The consumed gradient or normal-equation slots are zeroed after they are
// read, so a captured tracking iteration needs no clearing node.
#include "internal.hpp"
#include "se3.hpp"

namespace pxm {

__global__ void k_pose_adam(int F, float* __restrict__ c2w, double* __restrict__ gp,
                            double* __restrict__ state, float lr, float b1, float b2, float eps) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double* st = state + 16 * (int64_t)f;
    const double t = st[12] + 1.0;
    st[12] = t;
    const double c1 = 1.0 - pow((double)b1, t), c2 = 1.0 - pow((double)b2, t);
    double xi[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const double g = gp[6 * (int64_t)f + j];
        gp[6 * (int64_t)f + j] = 0.0;
        const double m = b1 * st[j] + (1.0 - b1) * g;
        const double v = b2 * st[6 + j] + (1.0 - b2) * g * g;
        st[j] = m;
        st[6 + j] = v;
        xi[j] = -(double)lr * (m / c1) / (sqrt(v / c2) + (double)eps);
    }
    se3_apply_left(c2w + 12 * (int64_t)f, xi);
}

hipError_t launch_adam(int F, float* c2w, double* grad_pose, double* state, float lr, float b1,
                       float b2, float eps, hipStream_t st) {
    const unsigned nb = (unsigned)((F + 63) / 64);
    hipLaunchKernelGGL(k_pose_adam, dim3(nb), dim3(64), 0, st, F, c2w, grad_pose, state, lr, b1, b2, eps);
    return hipGetLastError();
}

// gn[f] = (H upper triangle row by row: 21, g: 6, E: 1).  xi = -(H + mu I)^-1 g
// by Cholesky; a frame whose damped H is not positive definite (no ray saw
// the grid) keeps its pose.
__global__ void k_pose_gn(int F, float* __restrict__ c2w, double* __restrict__ gn, float mu) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double* s = gn + GN_VALUES * (int64_t)f;
    double L[6][6], rhs[6];
    int k = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
            L[i][j] = L[j][i] = s[k];
            ++k;
        }
    for (int i = 0; i < 6; ++i) {
        L[i][i] += (double)mu;
        rhs[i] = -s[21 + i];
    }
    for (int i = 0; i < GN_VALUES; ++i) s[i] = 0.0;
    // in-place Cholesky: lower triangle of L becomes the factor
    for (int j = 0; j < 6; ++j) {
        double d = L[j][j];
        for (int p = 0; p < j; ++p) d -= L[j][p] * L[j][p];
        if (!(d > 0.0)) return;
        d = sqrt(d);
        L[j][j] = d;
        for (int i = j + 1; i < 6; ++i) {
            double v = L[i][j];
            for (int p = 0; p < j; ++p) v -= L[i][p] * L[j][p];
            L[i][j] = v / d;
        }
    }
    double y[6], xi[6];
    for (int i = 0; i < 6; ++i) {
        double v = rhs[i];
        for (int p = 0; p < i; ++p) v -= L[i][p] * y[p];
        y[i] = v / L[i][i];
    }
    for (int i = 5; i >= 0; --i) {
        double v = y[i];
        for (int p = i + 1; p < 6; ++p) v -= L[p][i] * xi[p];
        xi[i] = v / L[i][i];
    }
    se3_apply_left(c2w + 12 * (int64_t)f, xi);
}

hipError_t launch_pose_gn(int F, float* c2w, double* gn, float mu, hipStream_t st) {
    const unsigned nb = (unsigned)((F + 63) / 64);
    hipLaunchKernelGGL(k_pose_gn, dim3(nb), dim3(64), 0, st, F, c2w, gn, mu);
    return hipGetLastError();
}

}  // namespace pxm
