// Left retraction of a camera pose by an se(3) twist, in FP64 on the device:
// c2w <- exp(xi^) c2w with xi = (rho, phi), rotation by Rodrigues' formula
// and translation V rho (the SE(3) exponential).
#pragma once

#include <hip/hip_runtime.h>

namespace pxm {

__device__ inline void se3_apply_left(float* __restrict__ M, const double xi[6]) {
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

}  // namespace pxm
