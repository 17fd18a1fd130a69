// Finite-volume diffusion operator on a box grid (2-D or 3-D, x fastest)
// with cell coefficients kappa = exp(theta): assembly of the CSR values from
// theta, and the gradient of a loss through the adjoint of the solve.
//   interior face (i, j): T = 2 k_i k_j / (k_i + k_j);  boundary face: T = 2 k_i
//   A_ii = sum of the cell's face T, A_ij = -T_ij (columns sorted).
//   dL/dT_ij = -(lam_i - lam_j)(x_i - x_j),  dT_ij/dtheta_i = 2 k_i k_j^2/(k_i + k_j)^2
//   dL/dT_b  = -lam_i x_i,                    dT_b/dtheta_i  = 2 k_i
#pragma once

#include "amp_device.hpp"

namespace amp {

struct Grid {
    int dim;        // 2 or 3
    int n[3];       // cells per axis (x, y, z); n[2] = 1 for 2-D
    int64_t stride[3];
    int64_t cells;
};

// Entries of row i in sorted column order: -z, -y, -x, diag, +x, +y, +z.
__global__ void __launch_bounds__(NT) k_fv_values(Grid g, const float *theta, const int32_t *row_ptr,
                                                  int32_t *col, double *val) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= g.cells) return;
    int64_t c[3];
    c[0] = i % g.n[0];
    c[1] = (i / g.n[0]) % g.n[1];
    c[2] = (g.dim == 3) ? i / ((int64_t)g.n[0] * g.n[1]) : 0;
    const double ki = exp((double)theta[i]);
    double diag = 0.0;
    int64_t pos = row_ptr[i];
    // lower neighbours, from the farthest axis to x
    for (int a = g.dim - 1; a >= 0; --a) {
        if (c[a] > 0) {
            const int64_t j = i - g.stride[a];
            const double kj = exp((double)theta[j]);
            const double t = 2.0 * ki * kj / (ki + kj);
            col[pos] = (int32_t)j;
            val[pos] = -t;
            ++pos;
            diag += t;
        } else {
            diag += 2.0 * ki;
        }
    }
    const int64_t dpos = pos++;
    for (int a = 0; a < g.dim; ++a) {
        if (c[a] < g.n[a] - 1) {
            const int64_t j = i + g.stride[a];
            const double kj = exp((double)theta[j]);
            const double t = 2.0 * ki * kj / (ki + kj);
            col[pos] = (int32_t)j;
            val[pos] = -t;
            ++pos;
            diag += t;
        } else {
            diag += 2.0 * ki;
        }
    }
    col[dpos] = (int32_t)i;
    val[dpos] = diag;
}

// dL/dtheta_i for every cell, FP64 accumulation over the cell's faces in the
// fixed order (-x, +x, -y, +y, -z, +z), FP32 result.
__global__ void __launch_bounds__(NT) k_fv_grad(Grid g, const float *theta, const double *x, const double *lam,
                                                float *dtheta) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= g.cells) return;
    int64_t c[3];
    c[0] = i % g.n[0];
    c[1] = (i / g.n[0]) % g.n[1];
    c[2] = (g.dim == 3) ? i / ((int64_t)g.n[0] * g.n[1]) : 0;
    const double ki = exp((double)theta[i]);
    const double xi = x[i], li = lam[i];
    double acc = 0.0;
    for (int a = 0; a < g.dim; ++a) {
        for (int s = -1; s <= 1; s += 2) {
            const int64_t cn = c[a] + s;
            if (cn >= 0 && cn < g.n[a]) {
                const int64_t j = i + s * g.stride[a];
                const double kj = exp((double)theta[j]);
                const double dLdT = -(li - lam[j]) * (xi - x[j]);
                const double sk = ki + kj;
                acc += dLdT * (2.0 * ki * kj * kj / (sk * sk));
            } else {
                acc += -li * xi * (2.0 * ki);
            }
        }
    }
    dtheta[i] = (float)acc;
}

}  // namespace amp
