// Conservative equilibrium (Section 3.1: the triplet of the Maxwellian is
// found by a Newton algorithm, Titarev's, so that the discrete relaxation
// term conserves mass, momentum and energy).  The unknowns x = (rho, u, T)
// solve  sum_p psi_p M[x](v_p) w = target  with psi = (1, v, |v|^2/2) (2D
// reduced model: plus the energy T/2 M carried by g).  The sampled
// Maxwellian is separable, so every discrete moment and every entry of the
// Jacobian is a product of one-dimensional sums over the N nodes of an axis,
//   P_k = sum_p v_p^k exp(-(v_p - u)^2 / (2T)) dv,   k = 0..4,
// with dP_k/du = (P_{k+1} - u P_k)/T and dP_k/dT = (P_{k+2} - 2u P_{k+1} +
// u^2 P_k)/(2T^2).  Once a Newton step is below 1e-13 of (rho, sqrt T, T)
// one more step is taken (quadratic convergence reaches the rounding floor)
// and the iteration stops; it fails after kNewtonMax steps.  One thread
// solves one cell.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

namespace ccdvm {

struct AxisSums {
  double P[5];    // P_0 .. P_4
  double dU[3];   // dP_k/du, k = 0..2
  double dT[3];   // dP_k/dT, k = 0..2
};

// Along the uniform grid X_p = exp(-(v_p - u)^2/(2T)) obeys X_{p+1} = X_p r_p
// with r_{p+1} = r_p q, q = exp(-dv^2/T) (and the same downwards with the
// mirrored ratio), so each axis needs four exponentials instead of N.  The
// walk starts at the node nearest to u and goes outwards, where X only
// decreases, so a cold gas underflows to zero without an overflowing ratio.
__host__ __device__ inline void axis_sums(double vmin, double dv, int N, double u, double T, AxisSums& a) {
  double P[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const double inv2T = 0.5 / T;
  int p0 = (int)floor((u - vmin) / dv);
  p0 = p0 < 0 ? 0 : (p0 > N - 1 ? N - 1 : p0);
  const double c0 = vmin + (p0 + 0.5) * dv - u;
  const double X0 = exp(-c0 * c0 * inv2T);
  const double q = exp(-dv * dv / T);
  auto add = [&](int p, double X) {
    const double v = vmin + (p + 0.5) * dv;
    double t = X * dv;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      P[k] += t;
      t *= v;
    }
  };
  add(p0, X0);
  double X = X0, r = exp(-(2.0 * c0 * dv + dv * dv) * inv2T);
  for (int p = p0 + 1; p < N; ++p) {
    X *= r;
    r *= q;
    add(p, X);
  }
  X = X0;
  r = exp((2.0 * c0 * dv - dv * dv) * inv2T);
  for (int p = p0 - 1; p >= 0; --p) {
    X *= r;
    r *= q;
    add(p, X);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) a.P[k] = P[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a.dU[k] = (P[k + 1] - u * P[k]) / T;
    a.dT[k] = (P[k + 2] - 2.0 * u * P[k + 1] + u * u * P[k]) / (2.0 * T * T);
  }
}

// Gaussian elimination with partial pivoting, n <= 5; solution in b.
template <int n>
__host__ __device__ inline bool solve_dense(double (&A)[n][n], double (&b)[n]) {
#pragma unroll
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int r = k + 1; r < n; ++r)
      if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
    if (A[piv][k] == 0.0) return false;
    if (piv != k) {
      for (int c = 0; c < n; ++c) { const double t = A[k][c]; A[k][c] = A[piv][c]; A[piv][c] = t; }
      const double t = b[k]; b[k] = b[piv]; b[piv] = t;
    }
    for (int r = k + 1; r < n; ++r) {
      const double m = A[r][k] / A[k][k];
      for (int c = k; c < n; ++c) A[r][c] -= m * A[k][c];
      b[r] -= m * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int c = k + 1; c < n; ++c) s -= A[k][c] * b[c];
    b[k] = s / A[k][k];
  }
  return true;
}

constexpr int kNewtonMax = 50;

// 2D reduced model: x = (rho, ux, uy, T) in/out, starting from the direct
// moments; target = (rho, rho ux, rho uy, E) of (f, g).  Returns false when
// the iteration does not converge (x then holds the last iterate).
__host__ __device__ inline bool conservative_triplet_2d(double (&x)[4], const double (&target)[4], double vmin,
                                               double dv, int N) {
  bool polish = false;
  for (int it = 0; it < kNewtonMax; ++it) {
    const double rho = x[0], T = x[3];
    AxisSums X, Y;
    axis_sums(vmin, dv, N, x[1], T, X);
    axis_sums(vmin, dv, N, x[2], T, Y);
    const double A = rho / (2.0 * M_PI * T);
    const double* a = X.P;
    const double* b = Y.P;
    double m[4];
    m[0] = A * a[0] * b[0];
    m[1] = A * a[1] * b[0];
    m[2] = A * a[0] * b[1];
    m[3] = A * (0.5 * a[2] * b[0] + 0.5 * a[0] * b[2] + 0.5 * T * a[0] * b[0]);
    double J[4][4];
    for (int i = 0; i < 4; ++i) J[i][0] = m[i] / rho;
    // d/dux: x-axis factor differentiated
    J[0][1] = A * X.dU[0] * b[0];
    J[1][1] = A * X.dU[1] * b[0];
    J[2][1] = A * X.dU[0] * b[1];
    J[3][1] = A * (0.5 * X.dU[2] * b[0] + 0.5 * X.dU[0] * b[2] + 0.5 * T * X.dU[0] * b[0]);
    // d/duy
    J[0][2] = A * a[0] * Y.dU[0];
    J[1][2] = A * a[1] * Y.dU[0];
    J[2][2] = A * a[0] * Y.dU[1];
    J[3][2] = A * (0.5 * a[2] * Y.dU[0] + 0.5 * a[0] * Y.dU[2] + 0.5 * T * a[0] * Y.dU[0]);
    // d/dT: prefactor, both axes, and the explicit T of the g energy
    J[0][3] = -m[0] / T + A * (X.dT[0] * b[0] + a[0] * Y.dT[0]);
    J[1][3] = -m[1] / T + A * (X.dT[1] * b[0] + a[1] * Y.dT[0]);
    J[2][3] = -m[2] / T + A * (X.dT[0] * b[1] + a[0] * Y.dT[1]);
    J[3][3] = -m[3] / T + A * (0.5 * (X.dT[2] * b[0] + a[2] * Y.dT[0]) + 0.5 * (X.dT[0] * b[2] + a[0] * Y.dT[2]) +
                               0.5 * T * (X.dT[0] * b[0] + a[0] * Y.dT[0]) + 0.5 * a[0] * b[0]);
    double r[4];
    for (int i = 0; i < 4; ++i) r[i] = m[i] - target[i];
    if (!solve_dense<4>(J, r)) return false;
    for (int i = 0; i < 4; ++i) x[i] -= r[i];
    if (polish) return true;
    const double su = sqrt(fabs(x[3]));
    polish = fabs(r[0]) <= 1e-13 * fabs(x[0]) && fabs(r[1]) <= 1e-13 * su && fabs(r[2]) <= 1e-13 * su &&
             fabs(r[3]) <= 1e-13 * fabs(x[3]);
  }
  return false;
}

// 3D: x = (rho, ux, uy, uz, T) in/out; target = (rho, rho u, E) of F.
__host__ __device__ inline bool conservative_triplet_3d(double (&x)[5], const double (&target)[5], double vmin,
                                               double dv, int N) {
  bool polish = false;
  for (int it = 0; it < kNewtonMax; ++it) {
    const double rho = x[0], T = x[4];
    AxisSums S[3];
    for (int d = 0; d < 3; ++d) axis_sums(vmin, dv, N, x[1 + d], T, S[d]);
    const double A = rho / pow(2.0 * M_PI * T, 1.5);
    // moment i = A * sum over terms of prod_d P^d_{k(d)}; the energy is
    // 1/2 (k = (2,0,0) + (0,2,0) + (0,0,2))
    auto prod = [&](int kx, int ky, int kz) { return S[0].P[kx] * S[1].P[ky] * S[2].P[kz]; };
    // product with axis e differentiated by `dU` (du_e) or `dT`
    auto dprod = [&](int kx, int ky, int kz, int e, bool wrt_u) {
      const int k[3] = {kx, ky, kz};
      double r = 1.0;
      for (int d = 0; d < 3; ++d)
        r *= d == e ? (wrt_u ? S[d].dU[k[d]] : S[d].dT[k[d]]) : S[d].P[k[d]];
      return r;
    };
    const int K[5][3][3] = {{{0, 0, 0}, {-1, 0, 0}, {-1, 0, 0}},
                            {{1, 0, 0}, {-1, 0, 0}, {-1, 0, 0}},
                            {{0, 1, 0}, {-1, 0, 0}, {-1, 0, 0}},
                            {{0, 0, 1}, {-1, 0, 0}, {-1, 0, 0}},
                            {{2, 0, 0}, {0, 2, 0}, {0, 0, 2}}};
    double m[5], J[5][5];
    for (int i = 0; i < 5; ++i) {
      const double c = i == 4 ? 0.5 : 1.0;
      double mi = 0.0, du[3] = {0.0, 0.0, 0.0}, dt = 0.0;
      for (int t = 0; t < 3; ++t) {
        if (K[i][t][0] < 0) continue;
        const int kx = K[i][t][0], ky = K[i][t][1], kz = K[i][t][2];
        mi += prod(kx, ky, kz);
        for (int e = 0; e < 3; ++e) {
          du[e] += dprod(kx, ky, kz, e, true);
          dt += dprod(kx, ky, kz, e, false);
        }
      }
      m[i] = c * A * mi;
      J[i][0] = m[i] / rho;
      for (int e = 0; e < 3; ++e) J[i][1 + e] = c * A * du[e];
      J[i][4] = -1.5 * m[i] / T + c * A * dt;
    }
    double r[5];
    for (int i = 0; i < 5; ++i) r[i] = m[i] - target[i];
    if (!solve_dense<5>(J, r)) return false;
    for (int i = 0; i < 5; ++i) x[i] -= r[i];
    if (polish) return true;
    const double su = sqrt(fabs(x[4]));
    polish = fabs(r[0]) <= 1e-13 * fabs(x[0]) && fabs(r[1]) <= 1e-13 * su && fabs(r[2]) <= 1e-13 * su &&
             fabs(r[3]) <= 1e-13 * su && fabs(r[4]) <= 1e-13 * fabs(x[4]);
  }
  return false;
}

}  // namespace ccdvm
