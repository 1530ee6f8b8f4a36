// Block-level solve of one cell's inner problem (eq. inner_eqn) in theta-space.
// Shared by the batched cell solve and the sequential scan kernel.
//
// After every update of either iteration of Section 3 the iterate is
//   g^{k+1} = D^{-1} (lambda M_theta - r),  D = |v_1|/dx + lambda,  lambda = nu/eps,
// with theta the step-1 solution (PFP, eq. step1) or the parameters of
// M[g^k] (FP, eq. fix_point).  The moments that drive the next update are
//   sum w phi g^{k+1}          = lambda sum w phi D^{-1} M_theta - R1,
//   sum w phi c g^{k+1}        = lambda sum w phi c D^{-1} M_theta - R2,
// with R0 = sum w phi r, R1 = sum w phi r / D, R2 = sum w phi c r / D fixed per
// visit (c = |v_1|/dx).  The residual of eq. inner_eqn at g^{k+1} is
// lambda |M_theta - M[g^{k+1}]|_{L2}, evaluated pointwise without memory traffic.
#pragma once

#include "bz_common.hpp"
#include "bz_newton.hpp"

namespace bz {

constexpr int kCellThreads = 256;

struct SolveArgs {
  int mode;
  double tol;
  int max_iter;
  int fixed_iters;
};

struct SolveOut {
  int used_b;  // 1 if the second initial guess was kept
  int iterations;
  int fallback;
  int newton_fail;
  int status;
  double residual;
};

// Block of kCellThreads threads.  rf(k) returns r at node k; g0 and g may alias
// (g0 is read in the first passes only, before the final write).  With g0b
// non-null the visit keeps whichever of g0 and g0b has the smaller initial
// residual of eq. inner_eqn (used by the learned warm start).
template <int N, typename RF>
__device__ __forceinline__ SolveOut solve_cell_block(const RF& rf, const double* g0, double* g, double lam, double dx,
                                                     const SolveArgs& opt, const double* nodes, double w,
                                                     const double* g0b = nullptr) {
  constexpr int K = N * N * N;
  const double inv_dx = 1.0 / dx;
  __shared__ double s_red[35 * (kCellThreads / 64)];
  __shared__ double s_Ea[3][N], s_Eb[3][N];  // axis factors of M[g0], M[g0b]
  __shared__ double s_ea[2];
  __shared__ double s_nodes[N];
  __shared__ double s_Et[3][N], s_Ee[3][N];  // axis factors of M_theta and M_eta
  __shared__ double s_th[5], s_eta[5];
  __shared__ int s_flags[4];  // fallback, newton_fail, nonfinite
  __syncthreads();  // the block may be reused across calls (sequential scans)
  if (threadIdx.x < N) s_nodes[threadIdx.x] = nodes[threadIdx.x];
  if (threadIdx.x < 4) s_flags[threadIdx.x] = 0;
  __syncthreads();
  // pass 1: fixed moment vectors of r and the moments of g0 (and g0b)
  double acc[35];
#pragma unroll
  for (int i = 0; i < 35; ++i) acc[i] = 0.0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double v0 = s_nodes[k / (N * N)], v1 = s_nodes[(k / N) % N], v2 = s_nodes[k % N];
    const double phi[5] = {1.0, v0, v1, v2, v0 * v0 + v1 * v1 + v2 * v2};
    const double c = fabs(v0) * inv_dx, Dinv = 1.0 / (c + lam);
    const double rk = rf(k), gk = g0[k];
    const double t0 = rk, t1 = rk * Dinv, t2 = c * rk * Dinv, t3 = gk, t4 = c * gk;
    const double gb = g0b ? g0b[k] : 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      acc[i] += phi[i] * t0;
      acc[5 + i] += phi[i] * t1;
      acc[10 + i] += phi[i] * t2;
      acc[15 + i] += phi[i] * t3;
      acc[20 + i] += phi[i] * t4;
      acc[25 + i] += phi[i] * gb;
      acc[30 + i] += phi[i] * c * gb;
    }
  }
  if (g0b) {
    block_sum<35>(acc, s_red);
  } else {
    block_sum<25>(*reinterpret_cast<double(*)[25]>(acc), s_red);
  }
  double R0[5], R1[5], R2[5], cg[5], th[5], eta[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    R0[i] = w * acc[i];
    R1[i] = w * acc[5 + i];
    R2[i] = w * acc[10 + i];
    cg[i] = w * acc[20 + i];
  }
  bool fallback = opt.mode == 1;
  int newton_fail = 0;
  int used_b = 0;
  double eta_b[5];
  if (threadIdx.x < 64) {
    double mg[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) mg[i] = w * acc[15 + i];
    theta_from_moments(mg, w, eta);
    AxisW aw{W_ONE, inv_dx, lam};
    if (newton_gauss(s_nodes, N, w, mg, eta, aw, 1e-13, 60) < 0) newton_fail++;
    if (g0b) {
#pragma unroll
      for (int i = 0; i < 5; ++i) mg[i] = w * acc[25 + i];
      theta_from_moments(mg, w, eta_b);
      if (newton_gauss(s_nodes, N, w, mg, eta_b, aw, 1e-13, 60) < 0) newton_fail++;
      const int lane = threadIdx.x;
      if (lane < N) {
        const double x = s_nodes[lane];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          s_Ea[a][lane] = exp(eta[1 + a] * x - eta[4] * x * x);
          s_Eb[a][lane] = exp(eta_b[1 + a] * x - eta_b[4] * x * x);
        }
      }
      if (lane == 0) {
        s_ea[0] = exp(eta[0]);
        s_ea[1] = exp(eta_b[0]);
      }
    }
  }
  if (g0b) {
    // pass 2: initial residuals |c g + r - lambda (M[g] - g)| of both guesses
    __syncthreads();
    double part[2] = {0.0, 0.0};
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
      const int a0 = k / (N * N), a1 = (k / N) % N, a2 = k % N;
      const double c = fabs(s_nodes[a0]) * inv_dx;
      const double rk = rf(k), ga = g0[k], gb = g0b[k];
      const double Ma = s_ea[0] * s_Ea[0][a0] * s_Ea[1][a1] * s_Ea[2][a2];
      const double Mb = s_ea[1] * s_Eb[0][a0] * s_Eb[1][a1] * s_Eb[2][a2];
      const double ra = c * ga + rk - lam * (Ma - ga), rb = c * gb + rk - lam * (Mb - gb);
      part[0] += ra * ra;
      part[1] += rb * rb;
    }
    block_sum<2>(part, s_red);
    if (part[1] < part[0]) {
      used_b = 1;
      if (threadIdx.x < 64) {
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          eta[i] = eta_b[i];
          cg[i] = w * acc[30 + i];
        }
      }
    }
  }
  if (threadIdx.x < 64) {
#pragma unroll
    for (int i = 0; i < 5; ++i) th[i] = eta[i];
  }
  const int n_upd = opt.fixed_iters > 0 ? opt.fixed_iters : opt.max_iter;
  int k_done = 0;
  double res = INFINITY;
  for (int k = 0; k < n_upd; ++k) {
    if (threadIdx.x < 64) {
      double S[3][5], mom[5];
      if (!fallback) {
        // step 1 (eq. step1): sum w phi c M' = sum w phi (c (M[g^k] - g^k) - r)
        AxisW awc{W_C, inv_dx, lam};
        axis_sums(s_nodes, N, eta, awc, S);
        gauss_moments(S, w * exp(eta[0]), mom, nullptr);
        double sv[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) sv[i] = mom[i] - cg[i] - R0[i];
        // eq. existence
        bool ok = sv[0] > 0.0 && sv[0] * sv[4] > sv[1] * sv[1] + sv[2] * sv[2] + sv[3] * sv[3];
        double tt[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) tt[i] = th[i];
        if (ok) {
          const int it = newton_gauss(s_nodes, N, w, sv, tt, awc, 1e-13, 60);
          ok = it >= 0 && tt[4] > 0.0;
        }
        if (ok) {
#pragma unroll
          for (int i = 0; i < 5; ++i) th[i] = tt[i];
        } else {
          fallback = true;
        }
      }
      if (fallback) {
#pragma unroll
        for (int i = 0; i < 5; ++i) th[i] = eta[i];
      }
      // moments of g^{k+1} = D^{-1}(lambda M_theta - r)
      AxisW awd{W_DINV, inv_dx, lam}, awcd{W_CDINV, inv_dx, lam};
      axis_sums(s_nodes, N, th, awd, S);
      gauss_moments(S, w * exp(th[0]), mom, nullptr);
      double mg[5];
#pragma unroll
      for (int i = 0; i < 5; ++i) mg[i] = lam * mom[i] - R1[i];
      axis_sums(s_nodes, N, th, awcd, S);
      gauss_moments(S, w * exp(th[0]), mom, nullptr);
#pragma unroll
      for (int i = 0; i < 5; ++i) cg[i] = lam * mom[i] - R2[i];
      AxisW aw1{W_ONE, inv_dx, lam};
      if (newton_gauss(s_nodes, N, w, mg, eta, aw1, 1e-13, 60) < 0) newton_fail++;
      const int lane = threadIdx.x;
      if (lane < N) {
        const double x = s_nodes[lane];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          s_Et[a][lane] = exp(th[1 + a] * x - th[4] * x * x);
          s_Ee[a][lane] = exp(eta[1 + a] * x - eta[4] * x * x);
        }
      }
      if (lane < 5) {
        s_th[lane] = th[lane];
        s_eta[lane] = eta[lane];
      }
      if (lane == 0) {
        s_flags[0] = fallback ? 1 : 0;
        s_flags[1] = newton_fail;
      }
    }
    __syncthreads();
    // residual lambda |M_theta - M[g^{k+1}]|_{L2}, pointwise
    const double ea = exp(s_th[0]), ee = exp(s_eta[0]);
    double part[1] = {0.0};
    for (int kk = threadIdx.x; kk < K; kk += blockDim.x) {
      const int a0 = kk / (N * N), a1 = (kk / N) % N, a2 = kk % N;
      const double d = ea * s_Et[0][a0] * s_Et[1][a1] * s_Et[2][a2] - ee * s_Ee[0][a0] * s_Ee[1][a1] * s_Ee[2][a2];
      part[0] += d * d;
    }
    block_sum<1>(part, s_red);
    res = lam * sqrt(w * part[0]);
    k_done = k + 1;
    if (opt.fixed_iters <= 0 && res <= opt.tol) break;
  }
  // final write g = D^{-1}(lambda M_theta - r)
  const double ea = exp(s_th[0]);
  bool bad = false;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const int a0 = k / (N * N), a1 = (k / N) % N, a2 = k % N;
    const double c = fabs(s_nodes[a0]) * inv_dx;
    const double val = (lam * ea * s_Et[0][a0] * s_Et[1][a1] * s_Et[2][a2] - rf(k)) / (c + lam);
    bad |= !isfinite(val);
    g[k] = val;
  }
  if (bad) s_flags[2] = 1;
  __syncthreads();
  SolveOut out;
  out.used_b = used_b;
  out.iterations = k_done;
  out.fallback = s_flags[0];
  out.newton_fail = s_flags[1];
  out.residual = res;
  out.status = (s_flags[2] || !isfinite(res)) ? 2 : ((opt.fixed_iters > 0 || res <= opt.tol) ? 0 : 1);
  return out;
}

}  // namespace bz
