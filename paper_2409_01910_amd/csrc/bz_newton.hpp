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

// weight applied on velocity axis 0 (v_1): c = |v_1| / dx, D = c + lambda
enum AxisWeight { W_ONE = 0, W_C = 1, W_DINV = 2, W_CDINV = 3 };

struct AxisW {
  int kind;
  double inv_dx;
  double lam;
};

__device__ __forceinline__ double axis0_weight(const AxisW& aw, double x) {
  const double c = fabs(x) * aw.inv_dx;
  switch (aw.kind) {
    case W_C: return c;
    case W_DINV: return 1.0 / (c + aw.lam);
    case W_CDINV: return c / (c + aw.lam);
    default: return 1.0;
  }
}

// S[a][p] for a Gaussian with parameters th (alpha unused here).  Whole wave
// participates; N <= 64 and lane i < N holds node i.  Result in every lane.
__device__ __forceinline__ void axis_sums(const double* nodes, int N, const double* th, const AxisW& aw,
                                          double S[3][5]) {
  const int lane = threadIdx.x & 63;
  double v[3][5];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int p = 0; p < 5; ++p) v[a][p] = 0.0;
  if (lane < N) {
    const double x = nodes[lane];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double e = exp(th[1 + a] * x - th[4] * x * x);
      if (a == 0) e *= axis0_weight(aw, x);
      double xp = 1.0;
#pragma unroll
      for (int p = 0; p < 5; ++p) {
        v[a][p] = e * xp;
        xp *= x;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int p = 0; p < 5; ++p) S[a][p] = wave_sum(v[a][p]);
}

__device__ __forceinline__ double mono(const double S[3][5], int p0, int p1, int p2) {
  return S[0][p0] * S[1][p1] * S[2][p2];
}

// sum phi_i phi_j M / (w e^alpha) for phi = (1, v_1, v_2, v_3, |v|^2)
__device__ __forceinline__ double phi2(const double S[3][5], int i, int j) {
  int e[3] = {0, 0, 0};
  if (i >= 1 && i <= 3) e[i - 1] += 1;
  if (j >= 1 && j <= 3) e[j - 1] += 1;
  const int n4 = (i == 4) + (j == 4);
  if (n4 == 0) return mono(S, e[0], e[1], e[2]);
  if (n4 == 1) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      int q[3] = {e[0], e[1], e[2]};
      q[c] += 2;
      s += mono(S, q[0], q[1], q[2]);
    }
    return s;
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int c2 = 0; c2 < 3; ++c2) {
      int q[3] = {0, 0, 0};
      q[c] += 2;
      q[c2] += 2;
      s += mono(S, q[0], q[1], q[2]);
    }
  return s;
}

// moments m_i = sum w c phi_i M and optionally J_ij = d m_i / d theta_j
__device__ __forceinline__ void gauss_moments(const double S[3][5], double scale, double m[5], double (*J)[5]) {
#pragma unroll
  for (int i = 0; i < 5; ++i) m[i] = scale * phi2(S, i, 0);
  if (J) {
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
      for (int j = 0; j < 5; ++j) J[i][j] = (j == 4 ? -scale : scale) * phi2(S, i, j);
  }
}

// Solve the 5x5 system A x = b by Gaussian elimination with partial pivoting.
__device__ __forceinline__ void solve5(double A[5][5], double b[5], double x[5]) {
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    int piv = c;
    double best = fabs(A[c][c]);
#pragma unroll
    for (int r = c + 1; r < 5; ++r)
      if (fabs(A[r][c]) > best) {
        best = fabs(A[r][c]);
        piv = r;
      }
    if (piv != c) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const double t = A[c][k];
        A[c][k] = A[piv][k];
        A[piv][k] = t;
      }
      const double t = b[c];
      b[c] = b[piv];
      b[piv] = t;
    }
#pragma unroll
    for (int r = c + 1; r < 5; ++r) {
      const double fct = A[r][c] / A[c][c];
#pragma unroll
      for (int k = c; k < 5; ++k) A[r][k] -= fct * A[c][k];
      b[r] -= fct * b[c];
    }
  }
#pragma unroll
  for (int r = 4; r >= 0; --r) {
    double s = b[r];
#pragma unroll
    for (int k = r + 1; k < 5; ++k) s -= A[r][k] * x[k];
    x[r] = s / A[r][r];
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
// the max-norm residual does not decrease, as in the reference algorithm.
__device__ __forceinline__ int newton_gauss(const double* nodes, int N, double w, const double target[5], double th[5],
                                            const AxisW& aw, double tol, int max_iter) {
  const double scale = fabs(target[0]) + fabs(target[4]) + 1e-300;
  double S[3][5], m[5], J[5][5], r[5];
  axis_sums(nodes, N, th, aw, S);
  gauss_moments(S, w * exp(th[0]), m, J);
  double nrm = 0.0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    r[i] = m[i] - target[i];
    nrm = fmax(nrm, fabs(r[i]));
  }
  if (!isfinite(nrm)) nrm = INFINITY;
  for (int it = 0; it < max_iter; ++it) {
    if (nrm <= tol * scale) return it;
    double rhs[5], step[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) rhs[i] = -r[i];
    solve5(J, rhs, step);
    // J was consumed by solve5; it is rebuilt from the accepted point's 1D sums
    double t = 1.0, thn[5], n_new = INFINITY, mn[5];
    while (true) {
#pragma unroll
      for (int i = 0; i < 5; ++i) thn[i] = th[i] + t * step[i];
      axis_sums(nodes, N, thn, aw, S);
      gauss_moments(S, w * exp(thn[0]), mn, nullptr);
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
    gauss_moments(S, w * exp(th[0]), mn, J);
    nrm = n_new;
    if (dmax <= 1e-15 * (1.0 + tmax)) return nrm <= 1e-10 * scale ? it + 1 : -(it + 2);
  }
  return nrm <= tol * scale ? max_iter : -(max_iter + 1);
}

}  // namespace bz
