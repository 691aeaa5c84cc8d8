// Shape derivative of the constrained solve (adjoint of psi with respect to the
// node positions).
//
// For the frozen-topology map X -> psi, with R(y, X) = T^T K(X) (g + T y) = 0 and
// a functional J(psi_b), the adjoint lambda solves A lambda = dJ/dy (A = T^T K T is
// symmetric) and
//     dJ/dX = - d/dX [ lambda_full^T K(X) psi_full ],   lambda_full = T lambda.
// The derivative of each element's lambda_e^T K_e(X) psi_e is taken analytically at
// the 2x2 Gauss points: with J the reference Jacobian (rows d/dxi, d/deta), M = J^-1,
// u = M grad_xi(lambda), v = M grad_xi(psi) and E_g = det J (u . v),
//     dE_g/dJ_ij = det J [ M_ji (u . v) - (M^T v)_i u_j - (M^T u)_i v_j ],
// and J_ij = sum_a dN_a/dxi_i X_aj.
#pragma once

#include "mfp_internal.h"

namespace mfp {

// One thread per cell: -dE/dX of the cell's four nodes into cg[8 * cell] (x then y
// for each local node 0..3), zero for inactive cells.
__global__ void k_shape_grad_cells(int nx, int ny, double hx, double hy,
                                   const int8_t* __restrict__ body, const double* __restrict__ disp,
                                   const double* __restrict__ lam, const double* __restrict__ psi,
                                   double* __restrict__ cg) {
  const long long nc = (long long)nx * ny;
  const long long nn = (long long)(nx + 1) * (ny + 1);
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < nc;
       c += (long long)gridDim.x * blockDim.x) {
    const int cj = (int)(c / nx), ci = (int)(c - (long long)cj * nx);
    const long long n0 = (long long)cj * (nx + 1) + ci;
    const long long nd[4] = {n0, n0 + 1, n0 + nx + 2, n0 + nx + 1};
    double out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int b0 = body[nd[0]];
    const bool inside = b0 >= 0 && body[nd[1]] == b0 && body[nd[2]] == b0 && body[nd[3]] == b0;
    if (!inside) {
      const double oi[4] = {0.0, 1.0, 1.0, 0.0}, oj[4] = {0.0, 0.0, 1.0, 1.0};
      const double xa[4] = {-1.0, 1.0, 1.0, -1.0}, ea[4] = {-1.0, -1.0, 1.0, 1.0};
      double x[4], y[4], l[4], p[4];
      for (int a = 0; a < 4; ++a) {
        x[a] = oi[a] * hx + disp[nd[a]];
        y[a] = oj[a] * hy + disp[nd[a] + nn];
        l[a] = lam[nd[a]];
        p[a] = psi[nd[a]];
      }
      const double s = 0.57735026918962576451;
      for (int q = 0; q < 4; ++q) {
        const double xi = xa[q] * s, eta = ea[q] * s;
        double nxi[4], net[4];
        double j11 = 0, j12 = 0, j21 = 0, j22 = 0, al0 = 0, al1 = 0, ap0 = 0, ap1 = 0;
        for (int a = 0; a < 4; ++a) {
          nxi[a] = 0.25 * xa[a] * (1.0 + ea[a] * eta);
          net[a] = 0.25 * ea[a] * (1.0 + xa[a] * xi);
          j11 += nxi[a] * x[a];
          j12 += nxi[a] * y[a];
          j21 += net[a] * x[a];
          j22 += net[a] * y[a];
          al0 += nxi[a] * l[a];
          al1 += net[a] * l[a];
          ap0 += nxi[a] * p[a];
          ap1 += net[a] * p[a];
        }
        const double det = j11 * j22 - j12 * j21;
        const double id = 1.0 / det;
        // M = J^-1
        const double m11 = j22 * id, m12 = -j12 * id, m21 = -j21 * id, m22 = j11 * id;
        const double u0 = m11 * al0 + m12 * al1, u1 = m21 * al0 + m22 * al1;
        const double v0 = m11 * ap0 + m12 * ap1, v1 = m21 * ap0 + m22 * ap1;
        const double uv = u0 * v0 + u1 * v1;
        const double mtu0 = m11 * u0 + m21 * u1, mtu1 = m12 * u0 + m22 * u1;
        const double mtv0 = m11 * v0 + m21 * v1, mtv1 = m12 * v0 + m22 * v1;
        // D_ij = dE_g/dJ_ij (i: xi/eta row, j: x/y column)
        const double d11 = det * (m11 * uv - mtv0 * u0 - mtu0 * v0);
        const double d12 = det * (m21 * uv - mtv0 * u1 - mtu0 * v1);
        const double d21 = det * (m12 * uv - mtv1 * u0 - mtu1 * v0);
        const double d22 = det * (m22 * uv - mtv1 * u1 - mtu1 * v1);
        for (int a = 0; a < 4; ++a) {
          out[2 * a] -= d11 * nxi[a] + d21 * net[a];
          out[2 * a + 1] -= d12 * nxi[a] + d22 * net[a];
        }
      }
    }
    for (int k = 0; k < 8; ++k) cg[8 * c + k] = out[k];
  }
}

// Per node: sum of the contributions of its (up to four) cells.
__global__ void k_shape_grad_gather(int nx, int ny, const double* __restrict__ cg,
                                    double* __restrict__ g) {
  const long long nn = (long long)(nx + 1) * (ny + 1);
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn;
       n += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(n / (nx + 1)), i = (int)(n - (long long)j * (nx + 1));
    double gx = 0.0, gy = 0.0;
    // (cell offset, local index of this node in that cell)
    const int ci[4] = {i - 1, i, i - 1, i}, cj[4] = {j - 1, j - 1, j, j}, loc[4] = {2, 3, 1, 0};
    for (int k = 0; k < 4; ++k) {
      if (ci[k] < 0 || ci[k] >= nx || cj[k] < 0 || cj[k] >= ny) continue;
      const long long c = (long long)cj[k] * nx + ci[k];
      gx += cg[8 * c + 2 * loc[k]];
      gy += cg[8 * c + 2 * loc[k] + 1];
    }
    g[n] = gx;
    g[n + nn] = gy;
  }
}

}  // namespace mfp
