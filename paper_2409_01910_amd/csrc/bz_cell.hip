// Discrete Maxwellian and the per-cell inner solve on gfx950.
//
// Inner problem (eq. inner_eqn): (|v_1|/dx) g + r = (nu/eps)(M[g] - g).
// Both iterations of Section 3 (plain fixed point, eq. fix_point, and the
// preconditioned one, eqs. step1 / step2) produce after each update
//   g^{k+1} = D^{-1} (lambda M_theta - r),   D = |v_1|/dx + lambda, lambda = nu/eps,
// for some Gaussian parameters theta (the step-1 solution for PFP, the
// parameters of M[g^k] for FP).  Every moment the next update needs is then a
// separable sum in theta plus one of three fixed moment vectors of r
// (sum w phi r, sum w phi r/D, sum w phi (|v_1|/dx) r/D), so a visit reads r and
// g^0 once, iterates in theta-space (O(N) work per Newton step), evaluates
// the residual |(|v_1|/dx) g + r - lambda (M[g] - g)| = lambda |M_theta - M[g]|
// pointwise without touching memory, and writes g once.
#include "bz_common.hpp"
#include "bz_internal.hpp"
#include "bz_newton.hpp"

namespace bz {

constexpr int kCellThreads = 256;

template <int N>
__global__ __launch_bounds__(kCellThreads) void k_maxwellian(const double* __restrict__ f, double* __restrict__ theta,
                                                             double* __restrict__ Mout, int32_t* __restrict__ iters,
                                                             const double* __restrict__ nodes, double w) {
  constexpr int K = N * N * N;
  const int b = blockIdx.x;
  const double* fb = f + (size_t)b * K;
  __shared__ double s_red[5 * (kCellThreads / 64)];
  __shared__ double s_nodes[N];
  __shared__ double s_E[3][N];
  __shared__ double s_th[5];
  if (threadIdx.x < N) s_nodes[threadIdx.x] = nodes[threadIdx.x];
  __syncthreads();
  double m[5] = {0, 0, 0, 0, 0};
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double v0 = s_nodes[k / (N * N)], v1 = s_nodes[(k / N) % N], v2 = s_nodes[k % N];
    const double fk = fb[k];
    m[0] += fk;
    m[1] += fk * v0;
    m[2] += fk * v1;
    m[3] += fk * v2;
    m[4] += fk * (v0 * v0 + v1 * v1 + v2 * v2);
  }
  block_sum<5>(m, s_red);
  if (threadIdx.x < 64) {
    double tgt[5], th[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) tgt[i] = w * m[i];
    theta_from_moments(tgt, w, th);
    AxisW aw{W_ONE, 0.0, 0.0};
    const int it = newton_gauss(s_nodes, N, w, tgt, th, aw, 1e-13, 60);
    if (threadIdx.x < 5) s_th[threadIdx.x] = th[threadIdx.x];
    if (threadIdx.x == 0 && iters) iters[b] = it;
  }
  __syncthreads();
  if (threadIdx.x < 5) theta[(size_t)b * 5 + threadIdx.x] = s_th[threadIdx.x];
  if (!Mout) return;
  if (threadIdx.x < 3 * N) {
    const int a = threadIdx.x / N, i = threadIdx.x % N;
    const double x = s_nodes[i];
    s_E[a][i] = exp(s_th[1 + a] * x - s_th[4] * x * x);
  }
  __syncthreads();
  const double ea = exp(s_th[0]);
  double* Mb = Mout + (size_t)b * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x)
    Mb[k] = ea * s_E[0][k / (N * N)] * s_E[1][(k / N) % N] * s_E[2][k % N];
}

struct SolveArgs {
  int mode;
  double tol;
  int max_iter;
  int fixed_iters;
};

template <int N>
__global__ __launch_bounds__(kCellThreads) void k_cell_solve(const double* __restrict__ r, const double* __restrict__ nu,
                                                             const double* __restrict__ eps, double dx,
                                                             const double* __restrict__ g0, double* __restrict__ g,
                                                             SolveArgs opt, bz_cell_stats* __restrict__ stats,
                                                             const double* __restrict__ nodes, double w) {
  constexpr int K = N * N * N;
  const int b = blockIdx.x;
  const double* rb = r + (size_t)b * K;
  const double* gb0 = g0 + (size_t)b * K;
  const double lam = nu[b] / eps[b];
  const double inv_dx = 1.0 / dx;
  __shared__ double s_red[25 * (kCellThreads / 64)];
  __shared__ double s_nodes[N];
  __shared__ double s_Et[3][N], s_Ee[3][N];  // axis factors of M_theta and M_eta
  __shared__ double s_th[5], s_eta[5];
  __shared__ int s_flags[4];  // fallback, newton_fail, nonfinite
  if (threadIdx.x < N) s_nodes[threadIdx.x] = nodes[threadIdx.x];
  if (threadIdx.x < 4) s_flags[threadIdx.x] = 0;
  __syncthreads();
  // pass 1: fixed moment vectors of r and the moments of g0
  double acc[25];
#pragma unroll
  for (int i = 0; i < 25; ++i) acc[i] = 0.0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double v0 = s_nodes[k / (N * N)], v1 = s_nodes[(k / N) % N], v2 = s_nodes[k % N];
    const double phi[5] = {1.0, v0, v1, v2, v0 * v0 + v1 * v1 + v2 * v2};
    const double c = fabs(v0) * inv_dx, Dinv = 1.0 / (c + lam);
    const double rk = rb[k], gk = gb0[k];
    const double t0 = rk, t1 = rk * Dinv, t2 = c * rk * Dinv, t3 = gk, t4 = c * gk;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      acc[i] += phi[i] * t0;
      acc[5 + i] += phi[i] * t1;
      acc[10 + i] += phi[i] * t2;
      acc[15 + i] += phi[i] * t3;
      acc[20 + i] += phi[i] * t4;
    }
  }
  block_sum<25>(acc, s_red);
  double R0[5], R1[5], R2[5], cg[5], th[5], eta[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    R0[i] = w * acc[i];
    R1[i] = w * acc[5 + i];
    R2[i] = w * acc[10 + i];
    cg[i] = w * acc[20 + i];
  }
  bool fallback = opt.mode == BZ_SOLVE_FP;
  int newton_fail = 0;
  if (threadIdx.x < 64) {
    double mg[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) mg[i] = w * acc[15 + i];
    theta_from_moments(mg, w, eta);
    AxisW aw{W_ONE, inv_dx, lam};
    if (newton_gauss(s_nodes, N, w, mg, eta, aw, 1e-13, 60) < 0) newton_fail++;
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
  double* gb = g + (size_t)b * K;
  bool bad = false;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const int a0 = k / (N * N), a1 = (k / N) % N, a2 = k % N;
    const double c = fabs(s_nodes[a0]) * inv_dx;
    const double val = (lam * ea * s_Et[0][a0] * s_Et[1][a1] * s_Et[2][a2] - rb[k]) / (c + lam);
    bad |= !isfinite(val);
    gb[k] = val;
  }
  if (bad) s_flags[2] = 1;
  __syncthreads();
  if (stats && threadIdx.x == 0) {
    bz_cell_stats st;
    st.iterations = k_done;
    st.fallback = s_flags[0];
    st.newton_fail = s_flags[1];
    st.residual = res;
    st.status = (s_flags[2] || !isfinite(res)) ? 2 : ((opt.fixed_iters > 0 || res <= opt.tol) ? 0 : 1);
    stats[b] = st;
  }
}

// r = inflow - (Q - nu (M_theta - f)) / eps ; nu = 4 pi rho
template <int N>
__global__ __launch_bounds__(kCellThreads) void k_penalty_rhs(const double* __restrict__ f, const double* __restrict__ Q,
                                                              const double* __restrict__ theta,
                                                              const double* __restrict__ inflow,
                                                              const double* __restrict__ eps, double* __restrict__ r,
                                                              double* __restrict__ nu_out,
                                                              const double* __restrict__ nodes, double w) {
  constexpr int K = N * N * N;
  const int b = blockIdx.x;
  __shared__ double s_E[3][N];
  __shared__ double s_nu;
  const double* th = theta + (size_t)b * 5;
  if (threadIdx.x < 3 * N) {
    const int a = threadIdx.x / N, i = threadIdx.x % N;
    const double x = nodes[i];
    s_E[a][i] = exp(th[1 + a] * x - th[4] * x * x);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < N; ++i) s[a] += s_E[a][i];
    s_nu = 4.0 * kPi * w * exp(th[0]) * s[0] * s[1] * s[2];
    nu_out[b] = s_nu;
  }
  __syncthreads();
  const double ea = exp(th[0]), nu = s_nu, ie = 1.0 / eps[b];
  const size_t o = (size_t)b * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double M = ea * s_E[0][k / (N * N)] * s_E[1][(k / N) % N] * s_E[2][k % N];
    const double P = Q[o + k] - nu * (M - f[o + k]);
    r[o + k] = inflow[o + k] - P * ie;
  }
}

#define BZ_DISPATCH_N(NV, CALL)                                           \
  switch (NV) {                                                           \
    case 8: {                                                             \
      constexpr int NN_ = 8;                                              \
      CALL;                                                               \
    } break;                                                              \
    case 16: {                                                            \
      constexpr int NN_ = 16;                                             \
      CALL;                                                               \
    } break;                                                              \
    case 32: {                                                            \
      constexpr int NN_ = 32;                                             \
      CALL;                                                               \
    } break;                                                              \
    default:                                                              \
      return set_err(ctx, BZ_EUNSUPPORTED, "N must be 8, 16 or 32");     \
  }

bz_status maxwellian(bz_ctx* ctx, const double* f, double* theta, double* M, int32_t* iters, int64_t batch,
                     hipStream_t st) {
  if (batch == 0) return BZ_OK;
  BZ_DISPATCH_N(ctx->N, hipLaunchKernelGGL((k_maxwellian<NN_>), dim3((unsigned)batch), dim3(kCellThreads), 0, st, f,
                                           theta, M, iters, ctx->d_nodes, ctx->w));
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

bz_status cell_solve(bz_ctx* ctx, const double* r, const double* nu, const double* eps, double dx, const double* g0,
                     double* g, int64_t batch, const bz_solve_opts* opts, bz_cell_stats* stats, hipStream_t st) {
  if (batch == 0) return BZ_OK;
  SolveArgs a{opts->mode, opts->tol, opts->max_iter, opts->fixed_iters};
  BZ_DISPATCH_N(ctx->N, hipLaunchKernelGGL((k_cell_solve<NN_>), dim3((unsigned)batch), dim3(kCellThreads), 0, st, r,
                                           nu, eps, dx, g0, g, a, stats, ctx->d_nodes, ctx->w));
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

bz_status penalty_rhs(bz_ctx* ctx, const double* f, const double* Q, const double* theta, const double* inflow,
                      const double* eps, double* r, double* nu, int64_t batch, hipStream_t st) {
  if (batch == 0) return BZ_OK;
  BZ_DISPATCH_N(ctx->N, hipLaunchKernelGGL((k_penalty_rhs<NN_>), dim3((unsigned)batch), dim3(kCellThreads), 0, st, f,
                                           Q, theta, inflow, eps, r, nu, ctx->d_nodes, ctx->w));
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

}  // namespace bz
