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
#include "bz_cellsolve.hpp"

namespace bz {

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
    AxisW aw{W_ONE, 0.0, 0.0, 0.0};
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

struct RPlain {
  const double* r;
  __device__ __forceinline__ double operator()(int k) const { return r[k]; }
};

template <int N>
__global__ __launch_bounds__(kCellThreads) void k_cell_solve(const double* __restrict__ r, const double* __restrict__ nu,
                                                             const double* __restrict__ eps, double dx,
                                                             const double* g0, double* g, SolveArgs opt,
                                                             bz_cell_stats* __restrict__ stats,
                                                             const double* __restrict__ nodes, double w,
                                                             const double* __restrict__ g0b,
                                                             const double* __restrict__ dxs) {
  constexpr int K = N * N * N;
  const int b = blockIdx.x;
  RPlain rf{r + (size_t)b * K};
  const double dxb = dxs ? dxs[b] : dx;
  const SolveOut o = solve_cell_block<N, kCellThreads>(rf, g0 + (size_t)b * K, g + (size_t)b * K, nu[b] / eps[b], dxb, opt, nodes, w,
                                         g0b ? g0b + (size_t)b * K : nullptr);
  if (stats && threadIdx.x == 0) {
    bz_cell_stats st;
    st.iterations = o.iterations;
    st.fallback = o.fallback;
    st.newton_fail = o.newton_fail;
    st.status = o.status;
    st.residual = o.residual;
    st.learned = o.used_b;
    st.relaxed = o.relaxed;
    stats[b] = st;
  }
}

// r = inflow - (Q - nu (M_theta - f)) / eps ; nu = penalty_nu (4 pi rho for Maxwell molecules)
template <int N>
__global__ __launch_bounds__(kCellThreads) void k_penalty_rhs(const double* __restrict__ f, const double* __restrict__ Q,
                                                              const double* __restrict__ theta,
                                                              const double* __restrict__ inflow,
                                                              const double* __restrict__ eps, double* __restrict__ r,
                                                              double* __restrict__ nu_out,
                                                              const double* __restrict__ nodes, double w, double gam,
                                                              double gfac, const double* __restrict__ nu_in) {
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
    s_nu = nu_in ? nu_in[b] : penalty_nu(w * exp(th[0]) * s[0] * s[1] * s[2], th[4], gam, gfac);
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

// Q <- Q - M_theta (sum_k Q_k) / (sum_k M_theta,k): removes, along the cell's
// Maxwellian, the mass that the sigma quadrature of the gain term creates, so
// that the collision term conserves mass to rounding.  Deterministic block sums.
template <int N>
__global__ __launch_bounds__(kCellThreads) void k_mass_project(double* __restrict__ Q, const double* __restrict__ theta,
                                                               const double* __restrict__ nodes) {
  constexpr int K = N * N * N;
  const int b = blockIdx.x;
  __shared__ double s_E[3][N];
  __shared__ double s_red[2 * (kCellThreads / 64)];
  const double* th = theta + (size_t)b * 5;
  if (threadIdx.x < 3 * N) {
    const int a = threadIdx.x / N, i = threadIdx.x % N;
    const double x = nodes[i];
    s_E[a][i] = exp(th[1 + a] * x - th[4] * x * x);
  }
  __syncthreads();
  const double ea = exp(th[0]);
  double* q = Q + (size_t)b * K;
  double acc[2] = {0.0, 0.0};
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    acc[0] += q[k];
    acc[1] += ea * s_E[0][k / (N * N)] * s_E[1][(k / N) % N] * s_E[2][k % N];
  }
  block_sum<2>(acc, s_red);
  const double c = acc[0] / acc[1];
  for (int k = threadIdx.x; k < K; k += blockDim.x)
    q[k] -= c * ea * s_E[0][k / (N * N)] * s_E[1][(k / N) % N] * s_E[2][k % N];
}

// Q <- Q - M_theta (a . phi), phi = (1, v, |v|^2), with G a = sum_k phi Q_k and
// G = sum_k phi phi^T M_theta: mass, momentum and energy conserved to rounding.
// G is separable (1D sums of x^p E_a(x)), so one thread builds and solves it.
template <int N>
__global__ __launch_bounds__(kCellThreads) void k_conserve_project(double* __restrict__ Q,
                                                                   const double* __restrict__ theta,
                                                                   const double* __restrict__ nodes) {
  constexpr int K = N * N * N;
  const int b = blockIdx.x;
  __shared__ double s_E[3][N];
  __shared__ double s_nodes[N];
  __shared__ double s_red[5 * (kCellThreads / 64)];
  __shared__ double s_a[5];
  const double* th = theta + (size_t)b * 5;
  if (threadIdx.x < N) s_nodes[threadIdx.x] = nodes[threadIdx.x];
  if (threadIdx.x < 3 * N) {
    const int a = threadIdx.x / N, i = threadIdx.x % N;
    const double x = nodes[i];
    s_E[a][i] = exp(th[1 + a] * x - th[4] * x * x);
  }
  __syncthreads();
  double* q = Q + (size_t)b * K;
  double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double v0 = s_nodes[k / (N * N)], v1 = s_nodes[(k / N) % N], v2 = s_nodes[k % N];
    const double qk = q[k];
    m[0] += qk;
    m[1] += qk * v0;
    m[2] += qk * v1;
    m[3] += qk * v2;
    m[4] += qk * (v0 * v0 + v1 * v1 + v2 * v2);
  }
  block_sum<5>(m, s_red);
  const double ea = exp(th[0]);
  if (threadIdx.x == 0) {
    double S[3][5], G[5][5], a[5];
    for (int ax = 0; ax < 3; ++ax)
      for (int p = 0; p < 5; ++p) S[ax][p] = 0.0;
    for (int ax = 0; ax < 3; ++ax)
      for (int i = 0; i < N; ++i) {
        double t = s_E[ax][i];
        for (int p = 0; p < 5; ++p) {
          S[ax][p] += t;
          t *= s_nodes[i];
        }
      }
    gauss_gram(S, G);
    double rhs[5];
    for (int i = 0; i < 5; ++i) rhs[i] = m[i] / ea;
    solve_spd5(G, rhs, a);
    for (int i = 0; i < 5; ++i) s_a[i] = a[i];
  }
  __syncthreads();
  const double a0 = s_a[0], a1 = s_a[1], a2 = s_a[2], a3 = s_a[3], a4 = s_a[4];
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const int i0 = k / (N * N), i1 = (k / N) % N, i2 = k % N;
    const double v0 = s_nodes[i0], v1 = s_nodes[i1], v2 = s_nodes[i2];
    const double M = ea * s_E[0][i0] * s_E[1][i1] * s_E[2][i2];
    q[k] -= M * (a0 + a1 * v0 + a2 * v1 + a3 * v2 + a4 * (v0 * v0 + v1 * v1 + v2 * v2));
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
                     double* g, int64_t batch, const bz_solve_opts* opts, bz_cell_stats* stats, hipStream_t st,
                     const double* g0b, const double* dxs) {
  if (batch == 0) return BZ_OK;
  SolveArgs a{opts->mode, opts->tol, opts->max_iter, opts->fixed_iters, ctx->p.v1_shift,
              opts->fallback == BZ_FALLBACK_RELAX ? 1 : 0};
  BZ_DISPATCH_N(ctx->N, hipLaunchKernelGGL((k_cell_solve<NN_>), dim3((unsigned)batch), dim3(kCellThreads), 0, st, r,
                                           nu, eps, dx, g0, g, a, stats, ctx->d_nodes, ctx->w, g0b, dxs));
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

bz_status mass_project(bz_ctx* ctx, double* Q, const double* theta, int64_t batch, hipStream_t st) {
  if (batch == 0) return BZ_OK;
  BZ_DISPATCH_N(ctx->N, hipLaunchKernelGGL((k_mass_project<NN_>), dim3((unsigned)batch), dim3(kCellThreads), 0, st, Q,
                                           theta, ctx->d_nodes));
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

bz_status conserve_project(bz_ctx* ctx, double* Q, const double* theta, int64_t batch, hipStream_t st) {
  if (batch == 0) return BZ_OK;
  BZ_DISPATCH_N(ctx->N, hipLaunchKernelGGL((k_conserve_project<NN_>), dim3((unsigned)batch), dim3(kCellThreads), 0, st,
                                           Q, theta, ctx->d_nodes));
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

bz_status penalty_rhs(bz_ctx* ctx, const double* f, const double* Q, const double* theta, const double* inflow,
                      const double* eps, double* r, double* nu, int64_t batch, hipStream_t st, const double* nu_in) {
  if (batch == 0) return BZ_OK;
  BZ_DISPATCH_N(ctx->N, hipLaunchKernelGGL((k_penalty_rhs<NN_>), dim3((unsigned)batch), dim3(kCellThreads), 0, st, f,
                                           Q, theta, inflow, eps, r, nu, ctx->d_nodes, ctx->w, ctx->p.gamma,
                                           ctx->nu_gfac, nu_in));
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

}  // namespace bz
