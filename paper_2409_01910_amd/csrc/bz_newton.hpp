// Separable moment sums and Newton's method for Gaussians exp(theta.(1, v, -|v|^2))
// on the uniform tensor velocity grid (one wave, lanes = grid index of an axis).
//
// On a tensor grid a Gaussian factorises over the three axes,
//   M(v) = e^alpha E_0(v_1) E_1(v_2) E_2(v_3),   E_a(x) = exp(beta_a x - gamma x^2),
// so every weighted moment sum_k w c(v_1) v^p M(v_k) needed by the discrete
// Maxwellian (eq. discrete_conservation) or by step 1 of the preconditioned
// iteration (eq. step1, weight |v_1|/dx) is a product of 1D sums
// S_a[p] = sum_i x_i^p c_a(x_i) E_a(x_i), p = 0..4.  One Newton step costs O(3N)
// exponentials instead of O(N^3).
#pragma once

#include "bz_common.hpp"

namespace bz {

// weight applied on velocity axis 0: c = |x + u0| / dx with u0 the grid's v_1
// shift (physical v_1 = x + u0), D = c + lambda
enum AxisWeight { W_ONE = 0, W_C = 1, W_DINV = 2, W_CDINV = 3 };

struct AxisW {
  int kind;
  double inv_dx;
  double lam;
  double u0;
};

__device__ __forceinline__ double axis0_weight(const AxisW& aw, double x) {
  const double c = fabs(x + aw.u0) * aw.inv_dx;
  switch (aw.kind) {
    case W_C: return c;
    case W_DINV: return 1.0 / (c + aw.lam);
    case W_CDINV: return c / (c + aw.lam);
    default: return 1.0;
  }
}

// S[a][p] for a Gaussian with parameters th (alpha unused here).  One wave,
// N <= 32: lanes 0..31 take axis 0 and lanes 32..63 axis 1 in a first set of
// five values, lanes 0..31 axis 2 in a second; lane i & 31 < N holds node i.
// Result in every lane.
__device__ __forceinline__ void axis_sums(const double* nodes, int N, const double* th, const AxisW& aw,
                                          double S[3][5]) {
  // Branch-free: every lane computes and then selects, so the lanes the DPP
  // moves read hold defined values under the full execution mask.
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
  const bool act = i < N;
  const double x = nodes[act ? i : 0];
  const double x2 = x * x;
  double e = exp(th[1 + h] * x - th[4] * x2);
  e *= h == 0 ? axis0_weight(aw, x) : 1.0;
  double e2 = exp(th[3] * x - th[4] * x2);
  e = act ? e : 0.0;
  e2 = (act && h == 0) ? e2 : 0.0;
  double va[5], vb[5];
  double xp = 1.0;
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    va[p] = e * xp;
    vb[p] = e2 * xp;
    xp *= x;
  }
  double lo[5], hi[5], lo2[5], hi2[5];
  half_wave_sums<5>(va, lo, hi);
  half_wave_sums<5>(vb, lo2, hi2);
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    S[0][p] = lo[p];
    S[1][p] = hi[p];
    S[2][p] = lo2[p];
  }
}

// Gram matrix G_ij = sum phi_i phi_j M / (w e^alpha) for phi = (1, v_1, v_2, v_3, |v|^2),
// from the 25 monomials S_0[p] S_1[q] S_2[r], p + q + r <= 4, that it needs.
// Symmetric; both triangles are filled.
__device__ __forceinline__ void gauss_gram(const double S[3][5], double G[5][5]) {
  auto m = [&](int p, int q, int r) { return S[0][p] * S[1][q] * S[2][r]; };
  const double m200 = m(2, 0, 0), m020 = m(0, 2, 0), m002 = m(0, 0, 2);
  G[0][0] = m(0, 0, 0);
  G[0][1] = m(1, 0, 0);
  G[0][2] = m(0, 1, 0);
  G[0][3] = m(0, 0, 1);
  G[0][4] = m200 + m020 + m002;
  G[1][1] = m200;
  G[1][2] = m(1, 1, 0);
  G[1][3] = m(1, 0, 1);
  G[2][2] = m020;
  G[2][3] = m(0, 1, 1);
  G[3][3] = m002;
  G[1][4] = m(3, 0, 0) + m(1, 2, 0) + m(1, 0, 2);
  G[2][4] = m(2, 1, 0) + m(0, 3, 0) + m(0, 1, 2);
  G[3][4] = m(2, 0, 1) + m(0, 2, 1) + m(0, 0, 3);
  G[4][4] = m(4, 0, 0) + m(0, 4, 0) + m(0, 0, 4) + 2.0 * (m(2, 2, 0) + m(2, 0, 2) + m(0, 2, 2));
#pragma unroll
  for (int a = 1; a < 5; ++a)
#pragma unroll
    for (int b = 0; b < a; ++b) G[a][b] = G[b][a];
}

// moments m_i = sum w c phi_i M = scale G_i0 (first column of the Gram matrix)
__device__ __forceinline__ void gauss_moments(const double S[3][5], double scale, double m[5]) {
  const double m200 = S[0][2] * S[1][0] * S[2][0], m020 = S[0][0] * S[1][2] * S[2][0],
               m002 = S[0][0] * S[1][0] * S[2][2];
  m[0] = scale * S[0][0] * S[1][0] * S[2][0];
  m[1] = scale * S[0][1] * S[1][0] * S[2][0];
  m[2] = scale * S[0][0] * S[1][1] * S[2][0];
  m[3] = scale * S[0][0] * S[1][0] * S[2][1];
  m[4] = scale * (m200 + m020 + m002);
}

// Solve G y = b for symmetric positive definite G (LDL^T, no pivoting; G is
// a weighted Gram matrix with non-negative weights).  G is overwritten.
__device__ __forceinline__ void solve_spd5(double G[5][5], const double b[5], double y[5]) {
  double d[5], inv[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    double dj = G[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= G[j][k] * G[j][k] * d[k];
    d[j] = dj;
    inv[j] = 1.0 / dj;
#pragma unroll
    for (int i = j + 1; i < 5; ++i) {
      double t = G[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= G[i][k] * G[j][k] * d[k];
      G[i][j] = t * inv[j];  // L_ij
    }
  }
  double z[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double t = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) t -= G[i][k] * z[k];
    z[i] = t;
  }
#pragma unroll
  for (int i = 4; i >= 0; --i) {
    double t = z[i] * inv[i];
#pragma unroll
    for (int k = i + 1; k < 5; ++k) t -= G[k][i] * y[k];
    y[i] = t;
  }
}

__device__ __forceinline__ void theta_from_moments(const double t[5], double w_unused, double th[5]) {
  (void)w_unused;
  const double rho = t[0];
  const double U0 = t[1] / rho, U1 = t[2] / rho, U2 = t[3] / rho;
  const double U2s = U0 * U0 + U1 * U1 + U2 * U2;
  double T = (t[4] / rho - U2s) / 3.0;
  if (!(T > 1e-3)) T = 1e-3;
  th[0] = log(rho / pow(2.0 * kPi * T, 1.5)) - U2s / (2.0 * T);
  th[1] = U0 / T;
  th[2] = U1 / T;
  th[3] = U2 / T;
  th[4] = 1.0 / (2.0 * T);
}

// Newton's method for sum_k w c_k phi_k exp(theta.phi~_k) = target.  Runs in one
// wave (all lanes compute identical values).  th holds the initial guess on
// entry and the result on exit.  Returns the number of steps (>= 0) when
// converged, or -(steps + 1) when not.  Backtracking halves the step while
// the max-norm residual does not decrease.
__device__ __forceinline__ int newton_gauss(const double* nodes, int N, double w, const double target[5], double th[5],
                                            const AxisW& aw, double tol, int max_iter) {
  // The Jacobian is d m_i / d theta_j = w e^alpha G_ij s_j with s = (1, 1, 1, 1, -1)
  // (theta.phi~ carries -gamma |v|^2), so each step solves the Gram system.
  const double scale = fabs(target[0]) + fabs(target[4]) + 1e-300;
  double S[3][5], m[5], r[5];
  axis_sums(nodes, N, th, aw, S);
  gauss_moments(S, w * exp(th[0]), m);
  double nrm = 0.0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    r[i] = m[i] - target[i];
    nrm = fmax(nrm, fabs(r[i]));
  }
  if (!isfinite(nrm)) nrm = INFINITY;
  for (int it = 0; it < max_iter; ++it) {
    if (nrm <= tol * scale) return it;
    double G[5][5], rhs[5], step[5];
    gauss_gram(S, G);
    const double ie = 1.0 / (w * exp(th[0]));
#pragma unroll
    for (int i = 0; i < 5; ++i) rhs[i] = -r[i] * ie;
    solve_spd5(G, rhs, step);
    step[4] = -step[4];
    double t = 1.0, thn[5], n_new = INFINITY, mn[5];
    while (true) {
#pragma unroll
      for (int i = 0; i < 5; ++i) thn[i] = th[i] + t * step[i];
      axis_sums(nodes, N, thn, aw, S);
      gauss_moments(S, w * exp(thn[0]), mn);
      n_new = 0.0;
#pragma unroll
      for (int i = 0; i < 5; ++i) n_new = fmax(n_new, fabs(mn[i] - target[i]));
      if (!isfinite(n_new)) n_new = INFINITY;
      if (isfinite(n_new) && (n_new < nrm || t < 1e-4) && thn[4] > 0.0) break;
      t *= 0.5;
      if (t < 1e-6) break;
    }
    double dmax = 0.0, tmax = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      dmax = fmax(dmax, fabs(thn[i] - th[i]));
      tmax = fmax(tmax, fabs(th[i]));
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      th[i] = thn[i];
      r[i] = mn[i] - target[i];
    }
    nrm = n_new;
    if (dmax <= 1e-15 * (1.0 + tmax)) return nrm <= 1e-10 * scale ? it + 1 : -(it + 2);
  }
  return nrm <= tol * scale ? max_iter : -(max_iter + 1);
}

}  // namespace bz
