// Tracking update: one Adam step per frame on the se(3) tangent of a left,
// world-frame perturbation, then c2w <- exp(xi^) c2w (FP64 on the device).
// One lane per frame; the gradient slot is zeroed after it is read so that a
// captured tracking iteration needs no clearing node.
#include "internal.hpp"

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
    // exp of the twist (rho, phi): rotation by Rodrigues, translation V rho
    const double p0 = xi[3], p1 = xi[4], p2 = xi[5];
    const double th2 = p0 * p0 + p1 * p1 + p2 * p2, th = sqrt(th2);
    double A, B, Cc;
    if (th < 1e-8) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
        Cc = 1.0 / 6.0 - th2 / 120.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        Cc = (th - sin(th)) / (th2 * th);
    }
    const double K[3][3] = {{0, -p2, p1}, {p2, 0, -p0}, {-p1, p0, 0}};
    double K2[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K2[i][j] = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
    double Rx[3][3], V[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double I = i == j ? 1.0 : 0.0;
            Rx[i][j] = I + A * K[i][j] + B * K2[i][j];
            V[i][j] = I + B * K[i][j] + Cc * K2[i][j];
        }
    float* M = c2w + 12 * (int64_t)f;
    double Mo[3][4];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 4; ++j) Mo[i][j] = M[4 * i + j];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 4; ++j) {
            double acc = Rx[i][0] * Mo[0][j] + Rx[i][1] * Mo[1][j] + Rx[i][2] * Mo[2][j];
            if (j == 3) acc += V[i][0] * xi[0] + V[i][1] * xi[1] + V[i][2] * xi[2];
            M[4 * i + j] = (float)acc;
        }
    }
}

hipError_t launch_adam(int F, float* c2w, double* grad_pose, double* state, float lr, float b1,
                       float b2, float eps, hipStream_t st) {
    const unsigned nb = (unsigned)((F + 63) / 64);
    hipLaunchKernelGGL(k_pose_adam, dim3(nb), dim3(64), 0, st, F, c2w, grad_pose, state, lr, b1, b2, eps);
    return hipGetLastError();
}

}  // namespace pxm
