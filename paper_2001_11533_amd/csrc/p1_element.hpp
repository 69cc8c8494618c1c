// P1 element matrices on a d-simplex (paper, Section 2: [A]_ij = a(phi_j,
// phi_i) with a(y, v) = int kappa grad y . grad v, and [M]_ij = (phi_j, phi_i)),
// shared by the host and the device assembler so that both form every value
// with the same operations in the same order.
//
// Textbook formulas: J has rows x_a - x_0; J^{-1} = adj(J)/det J; grad lambda_a
// (a >= 1) is column a of J^{-1} and grad lambda_0 = -(sum of the others);
// K_T = kappa |T| G G^T, M_T = |T| (1 + delta_ab) / ((d+1)(d+2)), formed
// without fused multiply-add.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace amg {

struct P1Elem {
    double K[4][4];
    double M[4][4];
};

// Gradients of the barycentric functions (g[a][0..dim-1], a = 0..dim) and the
// element measure.  X: (dim+1) x dim vertex coordinates, row-major.
__host__ __device__ inline void p1_grads(int dim, const double *X, double (&g)[4][3], double &meas) {
#pragma clang fp contract(off)
    if (dim == 2) {
        const double j00 = X[2] - X[0], j01 = X[3] - X[1];
        const double j10 = X[4] - X[0], j11 = X[5] - X[1];
        const double det = j00 * j11 - j01 * j10;
        const double i00 = j11 / det, i01 = -j01 / det, i10 = -j10 / det, i11 = j00 / det;
        g[1][0] = i00;
        g[1][1] = i10;
        g[2][0] = i01;
        g[2][1] = i11;
        meas = fabs(det) / 2.0;
    } else {
        const double a = X[3] - X[0], b = X[4] - X[1], c = X[5] - X[2];
        const double ee = X[6] - X[0], f = X[7] - X[1], gg = X[8] - X[2];
        const double h = X[9] - X[0], i = X[10] - X[1], k = X[11] - X[2];
        const double c00 = f * k - gg * i;
        const double c01 = gg * h - ee * k;
        const double c02 = ee * i - f * h;
        const double det = a * c00 + b * c01 + c * c02;
        const double inv[3][3] = {
            {c00 / det, (c * i - b * k) / det, (b * gg - c * f) / det},
            {c01 / det, (a * k - c * h) / det, (c * ee - a * gg) / det},
            {c02 / det, (b * h - a * i) / det, (a * f - b * ee) / det},
        };
        for (int q = 1; q <= 3; ++q)
            for (int r = 0; r < 3; ++r) g[q][r] = inv[r][q - 1];
        meas = fabs(det) / 6.0;
    }
    for (int r = 0; r < dim; ++r) {
        double v = -g[1][r];
        for (int q = 2; q <= dim; ++q) v = v - g[q][r];
        g[0][r] = v;
    }
}

// w gp . gq (w = kappa |T|, gp and gq two rows of the gradients)
__host__ __device__ inline double p1_stiff_vec(int dim, const double *gp, const double *gq, double w) {
#pragma clang fp contract(off)
    double dot = gp[0] * gq[0];
    for (int r = 1; r < dim; ++r) dot = dot + gp[r] * gq[r];
    return w * dot;
}

// K_T[p][q] = w grad lambda_p . grad lambda_q
__host__ __device__ inline double p1_stiff(int dim, const double (&g)[4][3], double w, int p, int q) {
    return p1_stiff_vec(dim, g[p], g[q], w);
}

// M_T[p][q] = |T| (1 + delta_pq) / ((d+1)(d+2))
__host__ __device__ inline double p1_mass(int dim, double meas, int p, int q) {
#pragma clang fp contract(off)
    const double base = meas / (double)((dim + 1) * (dim + 2));
    return p == q ? 2.0 * base : base;
}

// both element matrices
__host__ __device__ inline void p1_element(int dim, const double *X, double kappa, P1Elem &e) {
#pragma clang fp contract(off)
    double g[4][3];
    double meas;
    p1_grads(dim, X, g, meas);
    const double w = kappa * meas;
    const int nl = dim + 1;
    for (int p = 0; p < nl; ++p)
        for (int q = 0; q < nl; ++q) {
            e.K[p][q] = p1_stiff(dim, g, w, p, q);
            e.M[p][q] = p1_mass(dim, meas, p, q);
        }
}

}  // namespace amg
