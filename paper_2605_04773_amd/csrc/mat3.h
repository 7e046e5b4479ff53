// 3x3 algebra of the Newton loop's element kernel, usable on the host and
// the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace agc {

// Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations
// (each rotation zeroes one off-diagonal pair; Golub and Van Loan, the
// symmetric Schur step): on return a is diagonal (the eigenvalues) and the
// columns of v are the eigenvectors.
__host__ __device__ inline void jacobi_eig3(double a[3][3], double v[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) v[i][j] = i == j ? 1.0 : 0.0;
  const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
  for (int sweep = 0; sweep < 16; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off <= 1e-34 * dia || off == 0.0) break;
    for (int r = 0; r < 3; ++r) {
      const int p = P[r], q = Q[r];
      const double apq = a[p][q];
      if (apq == 0.0) continue;
      const double tau = (a[q][q] - a[p][p]) / (2.0 * apq);
      const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
      const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
      for (int k = 0; k < 3; ++k) {   // A J
        const double akp = a[k][p], akq = a[k][q];
        a[k][p] = c * akp - s * akq;
        a[k][q] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {   // J^T (A J)
        const double apk = a[p][k], aqk = a[q][k];
        a[p][k] = c * apk - s * aqk;
        a[q][k] = s * apk + c * aqk;
      }
      a[p][q] = a[q][p] = 0.0;
      for (int k = 0; k < 3; ++k) {   // V J
        const double vkp = v[k][p], vkq = v[k][q];
        v[k][p] = c * vkp - s * vkq;
        v[k][q] = s * vkp + c * vkq;
      }
    }
  }
}

// R of the rotation-variant polar decomposition F = R S (det R = +1; for
// det F < 0 the sign sits on the smallest singular value): with F^T F = V L
// V^T (V proper, L descending), u_0 and u_1 are F v_0 and F v_1 normalised
// (u_1 orthogonalised against u_0), u_2 = u_0 x u_1, and R = U V^T.
__host__ __device__ inline void polar_rotation(const double f[3][3], double r[3][3]) {
  double c[3][3], v[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c[i][j] = f[0][i] * f[0][j] + f[1][i] * f[1][j] + f[2][i] * f[2][j];
  jacobi_eig3(c, v);
  double l[3] = {c[0][0], c[1][1], c[2][2]};
  int o[3] = {0, 1, 2};   // descending order of l
  if (l[o[0]] < l[o[1]]) { const int t = o[0]; o[0] = o[1]; o[1] = t; }
  if (l[o[1]] < l[o[2]]) { const int t = o[1]; o[1] = o[2]; o[2] = t; }
  if (l[o[0]] < l[o[1]]) { const int t = o[0]; o[0] = o[1]; o[1] = t; }
  double vs[3][3];   // columns in descending order
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i) vs[i][k] = v[i][o[k]];
  const double dv = vs[0][0] * (vs[1][1] * vs[2][2] - vs[2][1] * vs[1][2]) -
                    vs[0][1] * (vs[1][0] * vs[2][2] - vs[2][0] * vs[1][2]) +
                    vs[0][2] * (vs[1][0] * vs[2][1] - vs[2][0] * vs[1][1]);
  if (dv < 0.0)
    for (int i = 0; i < 3; ++i) vs[i][2] = -vs[i][2];
  double u[3][3];   // columns u_0, u_1, u_2
  for (int k = 0; k < 2; ++k)
    for (int i = 0; i < 3; ++i) u[i][k] = f[i][0] * vs[0][k] + f[i][1] * vs[1][k] + f[i][2] * vs[2][k];
  const double n0 = sqrt(u[0][0] * u[0][0] + u[1][0] * u[1][0] + u[2][0] * u[2][0]);
  if (!(n0 > 1e-300)) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) r[i][j] = i == j ? 1.0 : 0.0;
    return;
  }
  for (int i = 0; i < 3; ++i) u[i][0] /= n0;
  const double d01 = u[0][0] * u[0][1] + u[1][0] * u[1][1] + u[2][0] * u[2][1];
  for (int i = 0; i < 3; ++i) u[i][1] -= d01 * u[i][0];
  double n1 = sqrt(u[0][1] * u[0][1] + u[1][1] * u[1][1] + u[2][1] * u[2][1]);
  if (!(n1 > 1e-12 * n0)) {   // rank one: any unit vector orthogonal to u_0
    const int k = fabs(u[0][0]) <= fabs(u[1][0]) ? (fabs(u[0][0]) <= fabs(u[2][0]) ? 0 : 2)
                                                  : (fabs(u[1][0]) <= fabs(u[2][0]) ? 1 : 2);
    double e[3] = {0.0, 0.0, 0.0};
    e[k] = 1.0;
    u[0][1] = u[1][0] * e[2] - u[2][0] * e[1];
    u[1][1] = u[2][0] * e[0] - u[0][0] * e[2];
    u[2][1] = u[0][0] * e[1] - u[1][0] * e[0];
    n1 = sqrt(u[0][1] * u[0][1] + u[1][1] * u[1][1] + u[2][1] * u[2][1]);
  }
  for (int i = 0; i < 3; ++i) u[i][1] /= n1;
  u[0][2] = u[1][0] * u[2][1] - u[2][0] * u[1][1];
  u[1][2] = u[2][0] * u[0][1] - u[0][0] * u[2][1];
  u[2][2] = u[0][0] * u[1][1] - u[1][0] * u[0][1];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r[i][j] = u[i][0] * vs[j][0] + u[i][1] * vs[j][1] + u[i][2] * vs[j][2];
}

}  // namespace agc
