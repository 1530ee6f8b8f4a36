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
// lambda |M_theta - M[g^{k+1}]|_{L2}; both Gaussians factorise over the axes, so
// its square is a short sum of products of 1D sums (gauss_diff_norm2), and each
// update costs O(N) work in one wave.  That sum can cancel when the two
// parameter sets differ more than the sampled Gaussians do (coarse grids), so
// whenever its rounding bound straddles the tolerance, and in fixed-count mode,
// the block evaluates the norm pointwise instead.
#pragma once

#include "bz_common.hpp"
#include "bz_newton.hpp"

namespace bz {

constexpr int kCellThreads = 256;   // batched cell solve: one work-group per cell
constexpr int kChainThreads = 256;  // sequential scan (one wave per SIMD: the update loop needs > 256 registers)

// |e^a E_0 E_1 E_2 - e^a' E'_0 E'_1 E'_2|^2 summed over the grid (no weight), for
// E_a(x) = exp(th[1+a] x - th[4] x^2) and E'_a from et.  The difference is
// telescoped into four separable terms,
//   (e^a - e^a') E0 E1 E2 + e^a' (E0 - E0') E1 E2 + e^a' E0' (E1 - E1') E2
//   + e^a' E0' E1' (E2 - E2'),
// with the differences formed through expm1, so that each term is accurate when
// the two Gaussians are close (the terms can still cancel one another where
// the grid samples the Gaussians coarsely; the caller checks the bound).  Their
// 16 inner products are products of three 1D sums of pairwise products of
// {E, E', E - E'}.  Returns the squared norm and, in bound, the sum of the
// magnitudes of the 16 products (the scale of its rounding error).
// One full wave, N <= 32; results in every lane.
__device__ __forceinline__ double gauss_diff_norm2(const double* nodes, int N, const double th[5], const double et[5],
                                                   double& bound) {
  // lanes 0..31: axis 0 (first set) and axis 2 (second set); lanes 32..63: axis 1.
  // Branch-free, so that the lanes the DPP moves read hold defined values.
  const int lane = threadIdx.x & 63, ix = lane & 31, h = lane >> 5;
  const bool act = ix < N;
  const double x = nodes[act ? ix : 0], x2 = x * x;
  double va[6], vb[6];
  auto pairs = [&](int a, bool on, double (&v)[6]) {
    const double ep = exp(et[1 + a] * x - et[4] * x2);
    const double e = exp(th[1 + a] * x - th[4] * x2);
    const double d = ep * expm1((th[1 + a] - et[1 + a]) * x - (th[4] - et[4]) * x2);
    // pairs: 0 EE, 1 EE', 2 Ed, 3 E'E', 4 E'd, 5 dd
    v[0] = on ? e * e : 0.0;
    v[1] = on ? e * ep : 0.0;
    v[2] = on ? e * d : 0.0;
    v[3] = on ? ep * ep : 0.0;
    v[4] = on ? ep * d : 0.0;
    v[5] = on ? d * d : 0.0;
  };
  pairs(h, act, va);
  pairs(2, act && h == 0, vb);
  double S[3][6], unused[6];
  half_wave_sums<6>(va, S[0], S[1]);
  half_wave_sums<6>(vb, S[2], unused);
  // factor of term i on axis a: 0 = E, 1 = E', 2 = d
  constexpr int F[4][3] = {{0, 0, 0}, {2, 0, 0}, {1, 2, 0}, {1, 1, 2}};
  constexpr int P[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  const double ce = exp(et[0]);
  const double c[4] = {ce * expm1(th[0] - et[0]), ce, ce, ce};
  double n2 = 0.0, b = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double t = c[i] * c[j] * S[0][P[F[i][0]][F[j][0]]] * S[1][P[F[i][1]][F[j][1]]] * S[2][P[F[i][2]][F[j][2]]];
      n2 += t;
      b += fabs(t);
    }
  bound = b;
  return fmax(n2, 0.0);
}

template <bool B>
struct BoolTag {
  static constexpr bool value = B;
};

struct SolveArgs {
  int mode;
  double tol;
  int max_iter;
  int fixed_iters;
  double u0;  // grid v_1 shift: physical v_1 = node + u0
  int relax;  // 1: relaxed step 1 when eq. existence fails (BZ_FALLBACK_RELAX)
};

struct SolveOut {
  int used_b;  // 1 if the second initial guess was kept
  int iterations;
  int fallback;
  int relaxed;  // updates whose step 1 used the relaxation factor
  int newton_fail;
  int status;
  double residual;
};

// Per-visit inputs of the theta-space iteration, all multiplied by w and held by
// wave 0: R0 = sum phi r, R1 = sum phi r / D, R2 = sum phi c r / D, the moments
// mg = sum phi g^0 and cg = sum phi c g^0 of the initial guess, and eta, the
// parameters of M[g^0].
struct VisitMoments {
  double R0[5], R1[5], R2[5], mg[5], cg[5];
};

// Optional by-product of the final write for a sequential scan: the
// neighbour part of the next visit's R0, R1, R2, i.e. the sums of phi t,
// phi t / D', phi c t / D' with t = coef(v_1) g, where g is this visit's result
// (the next cell's fresh upwind neighbour) and D' the next cell's D.  coef and
// dinv are LDS tables over the v_1 index; coef == nullptr disables it.
struct NextMoments {
  const double* coef;
  const double* dinv;
  double out[15];
};

// Block of NT threads, after VisitMoments and eta are known (wave 0): the
// update loop in theta-space and the final write g = D^{-1}(lambda M_theta - r).
// rf(k) returns r at node k; g0 is the initial guess, which g may alias.  A
// visit whose final theta or residual is not finite (a diverged plain
// iteration) keeps g0 and reports status 2, so one failed cell does not turn
// the whole field non-finite.
// s_nodes, s_c, s_dinv are LDS tables over an axis index: nodes, c = |v_1|/dx
// and 1 / (c + lambda).
template <int N, int NT, typename RF>
__device__ __forceinline__ SolveOut solve_core(const RF& rf, const double* g0, double* g, double lam, double inv_dx,
                                               const SolveArgs& opt, const double* s_nodes, const double* s_c,
                                               const double* s_dinv, double w, VisitMoments& vm, double (&eta)[5],
                                               int newton_fail, bool fallback, int used_b, NextMoments* nx) {
  constexpr int K = N * N * N;
  __shared__ double s_red[15 * (NT / 64)];
  __shared__ double s_Et[3][N], s_Ee[3][N];  // axis factors of M_theta and M_eta
  __shared__ double s_th[5], s_eta[5], s_res[2];
  __shared__ int s_chk[2];
  __shared__ int s_flags[5];  // fallback, newton_fail, nonfinite, keep g0, relaxed updates
  if (threadIdx.x < 5) s_flags[threadIdx.x] = 0;
  int relaxed = 0;
  __syncthreads();
  // the update loop: wave 0 iterates in theta-space, the block joins only for a
  // pointwise residual when the separable one cannot decide
  // the source iteration (mode 2) is the one plain update from the given eta
  // and has no inner residual: it goes straight to the final write
  const bool si = opt.mode == 2;
  const int n_upd = si ? 0 : (opt.fixed_iters > 0 ? opt.fixed_iters : opt.max_iter);
  int k_done = si ? 1 : 0;
  double res = si ? 0.0 : INFINITY;
  double th[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) th[i] = eta[i];
  for (int k = 0; k < n_upd; ++k) {
    const int slot = k & 1;  // double-buffered so that the next write cannot race this read
    if (threadIdx.x < 64) {
      double S[3][5], mom[5];
      if (!fallback) {
        // step 1 (eq. step1): sum w phi c M' = sum w phi (c (M[g^k] - g^k) - r)
        AxisW awc{W_C, inv_dx, lam, opt.u0};
        axis_sums(s_nodes, N, eta, awc, S);
        gauss_moments(S, w * exp(eta[0]), mom);
        double sv[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) sv[i] = mom[i] - vm.cg[i] - vm.R0[i];
        // eq. existence
        bool ok = sv[0] > 0.0 && sv[0] * sv[4] > sv[1] * sv[1] + sv[2] * sv[2] + sv[3] * sv[3];
        if (!ok && opt.relax) {
          // relaxed step 1 (Section 3.2, remark): (s + tau sum w phi c M[g]) / (1 + tau),
          // mom being that weighted moment of M[g^k] = M_eta
          for (double tau = 1.0; tau <= 1048576.0; tau *= 2.0) {
            double st[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) st[i] = (sv[i] + tau * mom[i]) / (1.0 + tau);
            if (st[0] > 0.0 && st[0] * st[4] > st[1] * st[1] + st[2] * st[2] + st[3] * st[3]) {
#pragma unroll
              for (int i = 0; i < 5; ++i) sv[i] = st[i];
              ok = true;
              ++relaxed;
              break;
            }
          }
        }
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
      AxisW awd{W_DINV, inv_dx, lam, opt.u0}, awcd{W_CDINV, inv_dx, lam, opt.u0};
      axis_sums(s_nodes, N, th, awd, S);
      gauss_moments(S, w * exp(th[0]), mom);
      double mg[5];
#pragma unroll
      for (int i = 0; i < 5; ++i) mg[i] = lam * mom[i] - vm.R1[i];
      axis_sums(s_nodes, N, th, awcd, S);
      gauss_moments(S, w * exp(th[0]), mom);
#pragma unroll
      for (int i = 0; i < 5; ++i) vm.cg[i] = lam * mom[i] - vm.R2[i];
      AxisW aw1{W_ONE, inv_dx, lam, opt.u0};
      // start from M_theta: at the fixed point M[g] = M_theta
      if (!fallback) {
#pragma unroll
        for (int i = 0; i < 5; ++i) eta[i] = th[i];
      }
      if (newton_gauss(s_nodes, N, w, mg, eta, aw1, 1e-13, 60) < 0) newton_fail++;
      // residual lambda |M_theta - M[g^{k+1}]|_{L2}, separable form with its rounding bound
      double bnd;
      const double n2 = gauss_diff_norm2(s_nodes, N, th, eta, bnd);
      const double rs = lam * sqrt(w * n2), fl = lam * sqrt(w * 1e-14 * bnd);
      const int chk = opt.fixed_iters > 0 || !isfinite(rs) || !(fabs(rs - opt.tol) > fl);
      const int lane = threadIdx.x;
      if (chk && lane < N) {
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
        s_res[slot] = rs;
        s_chk[slot] = chk;
        s_flags[0] = fallback ? 1 : 0;
        s_flags[1] = newton_fail;
        s_flags[4] = relaxed;
      }
    }
    __syncthreads();
    if (s_chk[slot]) {
      const double ea = exp(s_th[0]), ee = exp(s_eta[0]);
      double part[1] = {0.0};
      for (int kk = threadIdx.x; kk < K; kk += NT) {
        const int a0 = kk / (N * N), a1 = (kk / N) % N, a2 = kk % N;
        const double d = ea * s_Et[0][a0] * s_Et[1][a1] * s_Et[2][a2] - ee * s_Ee[0][a0] * s_Ee[1][a1] * s_Ee[2][a2];
        part[0] += d * d;
      }
      block_sum<1>(part, s_red);
      res = lam * sqrt(w * part[0]);
    } else {
      res = s_res[slot];
    }
    k_done = k + 1;
    if (opt.fixed_iters <= 0 && res <= opt.tol) break;
  }
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (lane < N) {
      const double x = s_nodes[lane];
#pragma unroll
      for (int a = 0; a < 3; ++a) s_Et[a][lane] = exp(th[1 + a] * x - th[4] * x * x);
    }
    if (lane < 5) s_th[lane] = th[lane];
    bool finite = isfinite(res);
#pragma unroll
    for (int i = 0; i < 5; ++i) finite = finite && isfinite(th[i]);
    if (lane == 0 && !finite) {
      s_flags[2] = 1;
      s_flags[3] = 1;
    }
  }
  __syncthreads();
  const bool keep = s_flags[3] != 0;
  // final write g = D^{-1}(lambda M_theta - r).  g may alias the initial guess
  // and nothing proves it does not alias r's sources, so the loads of a batch
  // of U points are staged in registers before any store, keeping U loads in
  // flight.
  const double ea = exp(s_th[0]);
  const bool want_next = nx && nx->coef;
  double acc[15];
#pragma unroll
  for (int i = 0; i < 15; ++i) acc[i] = 0.0;
  bool bad = false;
  // one instantiation per case, so that every load of a batch is unconditional
  // and can be issued before the first use
  auto final_pass = [&](auto keep_tag) {
    constexpr bool KEEP = decltype(keep_tag)::value;
    auto load = [&](int k) -> double {
      if constexpr (KEEP) {
        return g0[k];
      } else {
        return rf(k);
      }
    };
    if constexpr ((N * N) % NT == 0) {
      // plane by plane: the last-axis index is constant per thread (NT is a
      // multiple of N), the first-axis factors are read once per plane, and the
      // next visit's moments are summed per plane over (v_2, v_3) and weighted
      // by the plane's constants afterwards (4 FMAs per point instead of 15)
      constexpr int NN = N * N, PP = NN / NT, PB = (16 / PP) > 0 ? 16 / PP : 1;
      static_assert(N % PB == 0, "planes per batch must divide N");
      const int a2 = threadIdx.x % N;
      const double E2 = s_Et[2][a2], v2 = s_nodes[a2];
      for (int p0 = 0; p0 < N; p0 += PB) {
        double rv[PB * PP];
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
#pragma unroll
          for (int j = 0; j < PP; ++j) rv[pb * PP + j] = load((p0 + pb) * NN + j * NT + threadIdx.x);
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
          const int a0 = p0 + pb;
          const double E0 = lam * ea * s_Et[0][a0], di = s_dinv[a0];
          double sg[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int j = 0; j < PP; ++j) {
            const int kk = j * NT + threadIdx.x, k = a0 * NN + kk, a1 = kk / N;
            const double val = KEEP ? rv[pb * PP + j] : (E0 * s_Et[1][a1] * E2 - rv[pb * PP + j]) * di;
            bad |= !isfinite(val);
            g[k] = val;
            if (want_next) {
              const double v1 = s_nodes[a1];
              sg[0] += val;
              sg[1] += val * v1;
              sg[2] += val * v2;
              sg[3] += val * (v1 * v1 + v2 * v2);
            }
          }
          if (want_next) {
            const double v0 = s_nodes[a0], c0 = nx->coef[a0];
            const double sc[3] = {c0, c0 * nx->dinv[a0], s_c[a0] * c0 * nx->dinv[a0]};
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              acc[5 * q + 0] += sc[q] * sg[0];
              acc[5 * q + 1] += sc[q] * v0 * sg[0];
              acc[5 * q + 2] += sc[q] * sg[1];
              acc[5 * q + 3] += sc[q] * sg[2];
              acc[5 * q + 4] += sc[q] * (v0 * v0 * sg[0] + sg[3]);
            }
          }
        }
      }
    } else {
      constexpr int U = (K / NT) < 16 ? (K / NT) : 16;
      static_assert((K / NT) % U == 0, "unroll must divide the per-thread count");
      for (int k0 = threadIdx.x; k0 < K; k0 += U * NT) {
        double rv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) rv[u] = load(k0 + u * NT);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = k0 + u * NT;
          const int a0 = k / (N * N), a1 = (k / N) % N, a2 = k % N;
          const double val =
              KEEP ? rv[u] : (lam * ea * s_Et[0][a0] * s_Et[1][a1] * s_Et[2][a2] - rv[u]) * s_dinv[a0];
          bad |= !isfinite(val);
          g[k] = val;
          if (want_next) {
            const double v0 = s_nodes[a0], v1 = s_nodes[a1], v2 = s_nodes[a2];
            const double phi[5] = {1.0, v0, v1, v2, v0 * v0 + v1 * v1 + v2 * v2};
            const double t = nx->coef[a0] * val, td = t * nx->dinv[a0], tcd = s_c[a0] * td;
#pragma unroll
            for (int i = 0; i < 5; ++i) {
              acc[i] += phi[i] * t;
              acc[5 + i] += phi[i] * td;
              acc[10 + i] += phi[i] * tcd;
            }
          }
        }
      }
    }
  };
  if (keep) {
    final_pass(BoolTag<true>{});
  } else {
    final_pass(BoolTag<false>{});
  }
  if (bad) s_flags[2] = 1;
  if (want_next) {
    block_sum<15>(acc, s_red);
#pragma unroll
    for (int i = 0; i < 15; ++i) nx->out[i] = w * acc[i];
  }
  __syncthreads();
  SolveOut out;
  out.used_b = used_b;
  out.iterations = k_done;
  out.fallback = s_flags[0];
  out.relaxed = s_flags[4];
  out.newton_fail = s_flags[1];
  out.residual = res;
  out.status = (s_flags[2] || !isfinite(res)) ? 2 : ((opt.fixed_iters > 0 || res <= opt.tol) ? 0 : 1);
  return out;
}

// Tables over the v_1 index for a cell: nodes, c = |x + u0|/dx, 1/(c + lambda).
template <int N>
__device__ __forceinline__ void axis_tables(const double* nodes, double inv_dx, double lam, double u0,
                                            double* s_nodes, double* s_c, double* s_dinv) {
  if (threadIdx.x < N) {
    const double x = nodes[threadIdx.x], c = fabs(x + u0) * inv_dx;
    s_nodes[threadIdx.x] = x;
    s_c[threadIdx.x] = c;
    s_dinv[threadIdx.x] = 1.0 / (c + lam);
  }
}

// Initial Maxwellian parameters from the moments of g^0 (wave 0); with guess
// non-null Newton starts there (the parameters of M[g^0] if already known).
template <int N>
__device__ __forceinline__ int initial_eta(const double* s_nodes, double w, const double mg[5], double inv_dx,
                                           double lam, double (&eta)[5], const double* guess = nullptr) {
  if (guess) {
#pragma unroll
    for (int i = 0; i < 5; ++i) eta[i] = guess[i];
  } else {
    theta_from_moments(mg, w, eta);
  }
  AxisW aw{W_ONE, inv_dx, lam, 0.0};
  return newton_gauss(s_nodes, N, w, mg, eta, aw, 1e-13, 60) < 0 ? 1 : 0;
}

// Full visit of one cell by a block of NT threads: a pass over memory for the
// fixed moment vectors of r and the moments of g^0, then solve_core.  g0 and g
// may alias.  With g0b non-null the visit keeps whichever of g0 and g0b has
// the smaller initial residual of eq. inner_eqn (used by the learned warm start).
template <int N, int NT, typename RF>
__device__ __forceinline__ SolveOut solve_cell_block(const RF& rf, const double* g0, double* g, double lam, double dx,
                                                     const SolveArgs& opt, const double* nodes, double w,
                                                     const double* g0b = nullptr) {
  constexpr int K = N * N * N;
  const double inv_dx = 1.0 / dx;
  static_assert(NT % 64 == 0 && K % NT == 0, "block size must divide the grid");
  __shared__ double s_red[35 * (NT / 64)];
  __shared__ double s_Ea[3][N], s_Eb[3][N];  // axis factors of M[g0], M[g0b]
  __shared__ double s_ea[2];
  __shared__ double s_nodes[N], s_c[N], s_dinv[N];
  __syncthreads();  // the block may be reused across calls
  axis_tables<N>(nodes, inv_dx, lam, opt.u0, s_nodes, s_c, s_dinv);
  __syncthreads();
  // pass 1: fixed moment vectors of r and the moments of g0 (and g0b); one
  // instantiation per case so that the loads are unconditional
  double acc[35];
#pragma unroll
  for (int i = 0; i < 35; ++i) acc[i] = 0.0;
  auto pass1 = [&](auto with_b) {
    constexpr bool WB = decltype(with_b)::value;
#pragma unroll 8
    for (int k = threadIdx.x; k < K; k += NT) {
      const int a0 = k / (N * N);
      const double v0 = s_nodes[a0], v1 = s_nodes[(k / N) % N], v2 = s_nodes[k % N];
      const double phi[5] = {1.0, v0, v1, v2, v0 * v0 + v1 * v1 + v2 * v2};
      const double c = s_c[a0], Dinv = s_dinv[a0];
      const double rk = rf(k), gk = g0[k];
      const double t0 = rk, t1 = rk * Dinv, t2 = c * rk * Dinv, t3 = gk, t4 = c * gk;
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        acc[i] += phi[i] * t0;
        acc[5 + i] += phi[i] * t1;
        acc[10 + i] += phi[i] * t2;
        acc[15 + i] += phi[i] * t3;
        acc[20 + i] += phi[i] * t4;
      }
      if constexpr (WB) {
        const double gb = g0b[k];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          acc[25 + i] += phi[i] * gb;
          acc[30 + i] += phi[i] * c * gb;
        }
      }
    }
  };
  if (g0b) {
    pass1(BoolTag<true>{});
  } else {
    pass1(BoolTag<false>{});
  }
  if (g0b) {
    block_sum<35>(acc, s_red);
  } else {
    block_sum<25>(*reinterpret_cast<double(*)[25]>(acc), s_red);
  }
  VisitMoments vm;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    vm.R0[i] = w * acc[i];
    vm.R1[i] = w * acc[5 + i];
    vm.R2[i] = w * acc[10 + i];
    vm.mg[i] = w * acc[15 + i];
    vm.cg[i] = w * acc[20 + i];
  }
  const bool fallback = opt.mode == 1;
  int newton_fail = 0;
  int used_b = 0;
  double eta[5], eta_b[5];
  if (threadIdx.x < 64) {
    newton_fail += initial_eta<N>(s_nodes, w, vm.mg, inv_dx, lam, eta);
    if (g0b) {
      double mgb[5];
#pragma unroll
      for (int i = 0; i < 5; ++i) mgb[i] = w * acc[25 + i];
      newton_fail += initial_eta<N>(s_nodes, w, mgb, inv_dx, lam, eta_b);
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
    for (int k = threadIdx.x; k < K; k += NT) {
      const int a0 = k / (N * N), a1 = (k / N) % N, a2 = k % N;
      const double c = s_c[a0];
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
          vm.cg[i] = w * acc[30 + i];
        }
      }
    }
  }
  return solve_core<N, NT>(rf, g0, g, lam, inv_dx, opt, s_nodes, s_c, s_dinv, w, vm, eta, newton_fail, fallback, used_b,
                           nullptr);
}

}  // namespace bz
