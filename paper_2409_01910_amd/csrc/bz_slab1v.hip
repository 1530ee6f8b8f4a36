// The BGK slab with one velocity dimension (the 1D1V model of Section 4.1,
// v f_x = nu (M[f] - f) / eps): SGS scans (eq. SGS_BGK) with the visit solved by
// the plain iteration (eq. fix_point), the preconditioned iteration (eqs.
// step1, step2, existence) or the single update of the source iteration (eq.
// SI), first or second order (eqs. reconstruction, slope), diffuse walls
// (eq. boundary), the mass rescale (eq. mass_conserv), the outer residual of
// Section 4 and the FAS V-cycle of eq. coarse.
//
// A velocity grid of N <= 64 nodes fits one wave: lane k holds node v_k of
// every cell it touches, and every velocity sum is a wave reduction.  One
// work-group of one wave runs one instance from the first scan to the last
// V-cycle of a call, so nothing waits on the host between visits.  Each
// instance keeps its coarse levels, FAS sources, slopes, residual fields and
// per-cell Maxwellian parameters in a scratch region of the slab.
#include <cmath>
#include <vector>

#include "bz_common.hpp"
#include "bz_internal.hpp"

namespace bz {

struct Inst1 {
  int64_t off;  // first cell in f
  int64_t ws;   // first double of the instance's scratch
  int nx;       // fine cells
  int nlev;     // levels allocated (nx, nx/2, ... while even)
  double dx, eps, mass;
  double T[2];  // wall temperatures (left, right)
};

struct Opts1 {
  int mode;  // BZ_SOLVE_PFP, BZ_SOLVE_FP or BZ_SOLVE_SI
  double tol;
  int max_iter;
  int fixed_iters;
  int order;    // 1 or 2
  int limiter;  // 0 none, 1 minmod
  double bgk_nu;  // <= 0: |S^0| rho = 2 rho
};

struct MG1 {
  int coarsest, nu1, nu2, coarse_iters, fixed;
  double tol;
};

// per-level scratch: F, B, C0, R, S ([nx][N] each), nu [nx], theta [nx][3]
__host__ __device__ inline int64_t level1_doubles(int nx, int N) { return (int64_t)nx * (5 * N + 4); }

namespace {

constexpr int kOps = 3;  // 0: SGS iterations, 1: V-cycles, 2: residual only

struct Lev1 {
  double *f, *b, *c0, *R, *S, *nu, *th;
  int nx;
  double dx;
};

__device__ Lev1 level_of(const Inst1& I, double* f0, double* ws, int N, int l) {
  double* p = ws + I.ws;
  int nx = I.nx;
  double dx = I.dx;
  for (int q = 0; q < l; ++q) {
    p += level1_doubles(nx, N);
    nx /= 2;
    dx *= 2.0;
  }
  Lev1 L;
  L.nx = nx;
  L.dx = dx;
  const int64_t a = (int64_t)nx * N;
  L.f = l == 0 ? f0 + I.off * N : p;
  L.b = l == 0 ? nullptr : p + a;
  L.c0 = p + 2 * a;
  L.R = p + 3 * a;
  L.S = p + 4 * a;
  L.nu = p + 5 * a;
  L.th = L.nu + nx;
  return L;
}

// wave sums (the whole wave takes part; lanes beyond N hold zeros)
template <int NV>
__device__ __forceinline__ void wsum(double (&v)[NV]) {
  wave_sums_dpp<NV>(v);
}

__device__ __forceinline__ double gau(const double (&th)[3], double v) { return exp(th[0] + th[1] * v - th[2] * v * v); }

// x = A^{-1} y for a 3x3 system by the adjugate (fixed indexing keeps it in
// registers); false if the determinant vanishes or the result is not finite
__device__ bool solve3(const double (&A)[3][3], const double (&y)[3], double (&x)[3]) {
  const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
  if (det == 0.0) return false;
  const double c10 = A[0][2] * A[2][1] - A[0][1] * A[2][2];
  const double c11 = A[0][0] * A[2][2] - A[0][2] * A[2][0];
  const double c12 = A[0][1] * A[2][0] - A[0][0] * A[2][1];
  const double c20 = A[0][1] * A[1][2] - A[0][2] * A[1][1];
  const double c21 = A[0][2] * A[1][0] - A[0][0] * A[1][2];
  const double c22 = A[0][0] * A[1][1] - A[0][1] * A[1][0];
  const double id = 1.0 / det;
  x[0] = (c00 * y[0] + c10 * y[1] + c20 * y[2]) * id;
  x[1] = (c01 * y[0] + c11 * y[1] + c21 * y[2]) * id;
  x[2] = (c02 * y[0] + c12 * y[1] + c22 * y[2]) * id;
  return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
}

// Newton for sum_k w c_k phi_k exp(th . phi~_k) = t with phi = (1, v, v^2) and
// phi~ = (1, v, -v^2): c = 1 gives the discrete Maxwellian (eqs.
// discrete_conservation, discrete_Gaussian), c = |v|/dx step 1 (eq. step1).
// Start from the continuous moments of t (from_moments) or from th; halving
// backtracking while the residual grows; stop at max|F| <= 1e-13 (|t_0| + |t_2|).
__device__ bool gauss_newton(double (&th)[3], const double (&t)[3], double v, double c, bool on, double w,
                             bool from_moments) {
  if (from_moments) {
    const double rho = t[0], U = t[1] / rho;
    const double T = fmax(t[2] / rho - U * U, 1e-3);
    th[0] = log(rho / sqrt(2.0 * kPi * T)) - U * U / (2.0 * T);
    th[1] = U / T;
    th[2] = 1.0 / (2.0 * T);
  }
  const double scale = fabs(t[0]) + fabs(t[2]) + 1e-300;
  auto eval = [&](const double (&x)[3], double (&S)[5]) {
    const double g = on ? w * c * exp(x[0] + x[1] * v - x[2] * v * v) : 0.0;
    S[0] = g;
    S[1] = g * v;
    S[2] = g * v * v;
    S[3] = g * v * v * v;
    S[4] = g * v * v * v * v;
    wsum<5>(S);
  };
  double S[5];
  eval(th, S);
  double r[3] = {S[0] - t[0], S[1] - t[1], S[2] - t[2]};
  double nrm = fmax(fabs(r[0]), fmax(fabs(r[1]), fabs(r[2])));
  for (int it = 0; it < 60; ++it) {
    if (nrm <= 1e-13 * scale) return true;
    double J[3][3] = {{S[0], S[1], -S[2]}, {S[1], S[2], -S[3]}, {S[2], S[3], -S[4]}};
    bool finite = true;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) finite = finite && isfinite(J[a][b]);
    if (!finite) return false;
    double mr[3] = {-r[0], -r[1], -r[2]}, step[3];
    if (!solve3(J, mr, step)) return false;
    double tt = 1.0, xn[3], Sn[5], rn[3], nn = 0.0;
    while (true) {
      for (int a = 0; a < 3; ++a) xn[a] = th[a] + tt * step[a];
      eval(xn, Sn);
      for (int a = 0; a < 3; ++a) rn[a] = Sn[a] - t[a];
      nn = fmax(fabs(rn[0]), fmax(fabs(rn[1]), fabs(rn[2])));
      if (isfinite(nn) && (nn < nrm || tt < 1e-4) && xn[2] > 0.0) break;
      tt *= 0.5;
      if (tt < 1e-6) break;
    }
    const double dmax = fmax(fabs(xn[0] - th[0]), fmax(fabs(xn[1] - th[1]), fabs(xn[2] - th[2])));
    const double tmax = fmax(fabs(th[0]), fmax(fabs(th[1]), fabs(th[2])));
    for (int a = 0; a < 3; ++a) th[a] = xn[a];
    if (dmax <= 1e-15 * (1.0 + tmax)) return nn <= 1e-10 * scale;
    for (int a = 0; a < 5; ++a) S[a] = Sn[a];
    for (int a = 0; a < 3; ++a) r[a] = rn[a];
    nrm = nn;
  }
  return nrm <= 1e-13 * scale;
}

__device__ __forceinline__ bool maxwellian1(double g, double v, bool on, double w, double (&th)[3]) {
  double m[3] = {on ? w * g : 0.0, on ? w * g * v : 0.0, on ? w * g * v * v : 0.0};
  wsum<3>(m);
  return gauss_newton(th, m, v, 1.0, on, w, true);
}

struct Ctx1 {
  const Inst1* I;
  int N;
  double v, w;
  bool on;
  Opts1 o;
  unsigned long long it_sum, visit_sum, fb_sum;
};

// one visit: eq. inner_eqn (|v|/dx) g + r = lam (M[g] - g) from g0 by the
// iteration of the mode; SI makes the one update with the given Maxwellian Mn
__device__ double visit(Ctx1& C, double g0, double r, double nu, double dx, double Mn) {
  const double v = C.v, w = C.w;
  const bool on = C.on;
  const double c = fabs(v) / dx, lam = nu / C.I->eps, D = c + lam;
  C.visit_sum += 1;
  if (C.o.mode == BZ_SOLVE_SI) {
    C.it_sum += 1;
    return on ? (lam * Mn - r) / D : 0.0;
  }
  double g = g0, th_g[3];
  (void)maxwellian1(g, v, on, w, th_g);
  double Mg = gau(th_g, v);
  double th_step[3] = {th_g[0], th_g[1], th_g[2]};
  bool fallback = C.o.mode == BZ_SOLVE_FP, fell = false;
  const int n = C.o.fixed_iters > 0 ? C.o.fixed_iters : C.o.max_iter;
  double res = INFINITY;
  int k = 0;
  for (; k < n;) {
    double Mstep = Mg;
    if (!fallback) {
      const double e = on ? w * (c * (Mg - g) - r) : 0.0;
      double s[3] = {e, e * v, e * v * v};
      wsum<3>(s);
      bool ok = s[0] > 0.0 && s[0] * s[2] > s[1] * s[1];  // eq. existence
      double th[3] = {th_step[0], th_step[1], th_step[2]};
      if (ok) ok = gauss_newton(th, s, v, c, on, w, false) && th[2] > 0.0;
      if (ok) {
        for (int a = 0; a < 3; ++a) th_step[a] = th[a];
        Mstep = gau(th, v);
      } else {
        fallback = true;
        fell = true;
        Mstep = Mg;
      }
    }
    g = on ? (lam * Mstep - r) / D : 0.0;
    (void)maxwellian1(g, v, on, w, th_g);
    Mg = gau(th_g, v);
    const double q = on ? c * g + r - lam * (Mg - g) : 0.0;
    double e2[1] = {q * q};
    wsum<1>(e2);
    res = sqrt(w * e2[0]);
    ++k;
    if (C.o.fixed_iters <= 0 && res <= C.o.tol) break;
  }
  C.it_sum += k;
  C.fb_sum += fell ? 1 : 0;
  return isfinite(res) ? g : g0;  // a diverged visit keeps its start
}

__device__ __forceinline__ double minmod1(double a, double b) {
  return a * b > 0.0 ? copysign(fmin(fabs(a), fabs(b)), a) : 0.0;
}

// slopes of eq. slope (one-sided at the ends, centred or minmod inside) into L.S
__device__ void slopes1(const Ctx1& C, Lev1& L) {
  const int N = C.N, k = threadIdx.x;
  if (!C.on) return;
  for (int j = 0; j < L.nx; ++j) {
    double s = 0.0;
    if (C.o.order == 2 && L.nx >= 2) {
      const double fc = L.f[(int64_t)j * N + k];
      if (j == 0) s = L.f[(int64_t)N + k] - fc;
      else if (j == L.nx - 1) s = fc - L.f[(int64_t)(j - 1) * N + k];
      else {
        const double fr = L.f[(int64_t)(j + 1) * N + k], fl = L.f[(int64_t)(j - 1) * N + k];
        s = C.o.limiter ? minmod1(fr - fc, fc - fl) : 0.5 * (fr - fl);
      }
    }
    L.S[(int64_t)j * N + k] = s;
  }
}

// the two wall ghosts rho_w M_w from the zero-mass-flux balance of the
// wall-adjacent face values of the current field (eq. boundary)
__device__ void ghosts1(const Ctx1& C, const Lev1& L, double& gl, double& gr) {
  const int N = C.N, k = threadIdx.x;
  const double v = C.v;
  const double fl = C.on ? L.f[k] - 0.5 * L.S[k] : 0.0;
  const double fr = C.on ? L.f[(int64_t)(L.nx - 1) * N + k] + 0.5 * L.S[(int64_t)(L.nx - 1) * N + k] : 0.0;
  const double ML = C.on ? exp(-v * v / (2.0 * C.I->T[0])) / sqrt(2.0 * kPi * C.I->T[0]) : 0.0;
  const double MR = C.on ? exp(-v * v / (2.0 * C.I->T[1])) / sqrt(2.0 * kPi * C.I->T[1]) : 0.0;
  double s[4] = {v < 0.0 ? -v * fl : 0.0, v > 0.0 ? v * ML : 0.0, v > 0.0 ? v * fr : 0.0, v < 0.0 ? -v * MR : 0.0};
  wsum<4>(s);
  gl = s[0] / s[1] * ML;
  gr = s[2] / s[3] * MR;
}

// per-cell nu (and the Maxwellian parameters when want_th) of the current field
__device__ void cell_params(Ctx1& C, Lev1& L, bool want_th) {
  const int N = C.N, k = threadIdx.x;
  for (int j = 0; j < L.nx; ++j) {
    const double fj = C.on ? L.f[(int64_t)j * N + k] : 0.0;
    double m[1] = {C.w * fj};
    wsum<1>(m);
    const double nu = C.o.bgk_nu > 0.0 ? C.o.bgk_nu : 2.0 * m[0];
    if (k == 0) L.nu[j] = nu;
    if (want_th) {
      double th[3];
      (void)maxwellian1(fj, C.v, C.on, C.w, th);
      if (k < 3) L.th[(int64_t)j * 3 + k] = th[k];
    }
  }
}

// one scan (a line of eq. SGS_BGK); lagged: SI with nu and theta of the
// iterate before the forward scan, kept in L.nu and L.th
__device__ void scan1(Ctx1& C, Lev1& L, bool fwd, bool lagged) {
  const int N = C.N, k = threadIdx.x;
  const double v = C.v, vp = fmax(v, 0.0), vm = fmin(v, 0.0);
  slopes1(C, L);
  if (!lagged) cell_params(C, L, false);
  __syncthreads();
  double gl = 0.0, gr = 0.0;
  for (int step = 0; step < L.nx; ++step) {
    const int j = fwd ? step : L.nx - 1 - step;
    if (j == 0 || j == L.nx - 1) ghosts1(C, L, gl, gr);
    double r = 0.0, g0 = 0.0, Mn = 0.0;
    if (C.on) {
      const double left = j > 0 ? L.f[(int64_t)(j - 1) * N + k] : gl;
      const double right = j < L.nx - 1 ? L.f[(int64_t)(j + 1) * N + k] : gr;
      const double sl = j > 0 ? L.S[(int64_t)(j - 1) * N + k] : 0.0;
      const double sr = j < L.nx - 1 ? L.S[(int64_t)(j + 1) * N + k] : 0.0;
      r = (-vp * left + vm * right) / L.dx - (vp * sl - v * L.S[(int64_t)j * N + k] + vm * sr) / (2.0 * L.dx);
      if (L.b) r -= L.b[(int64_t)j * N + k];
      g0 = L.f[(int64_t)j * N + k];
      if (lagged) {
        const double th[3] = {L.th[(int64_t)j * 3], L.th[(int64_t)j * 3 + 1], L.th[(int64_t)j * 3 + 2]};
        Mn = gau(th, v);
      }
    }
    const double g = visit(C, g0, r, L.nu[j], L.dx, Mn);
    if (C.on) L.f[(int64_t)j * N + k] = g;
    __syncthreads();
  }
}

__device__ void sgs1(Ctx1& C, Lev1& L) {
  if (C.o.mode == BZ_SOLVE_SI) {
    cell_params(C, L, true);
    __syncthreads();
    scan1(C, L, true, true);
    scan1(C, L, false, true);
  } else {
    scan1(C, L, true, false);
    scan1(C, L, false, false);
  }
}

__device__ void rescale1(const Ctx1& C, Lev1& L) {
  const int N = C.N, k = threadIdx.x;
  double s[1] = {0.0};
  if (C.on)
    for (int j = 0; j < L.nx; ++j) s[0] += L.f[(int64_t)j * N + k];
  wsum<1>(s);
  const double a = C.I->mass / (L.dx * C.w * s[0]);
  if (C.on)
    for (int j = 0; j < L.nx; ++j) L.f[(int64_t)j * N + k] *= a;
  __syncthreads();
}

// R = v.grad f - Q/eps with the reconstruction of eq. slope (Q = nu (M - f));
// with sub, R <- b - R (b the level's FAS source) into L.R; returns
// sqrt(dx w sum R^2) of what it stores (or of R - b when !store)
__device__ double residual1(Ctx1& C, Lev1& L, bool store) {
  const int N = C.N, k = threadIdx.x;
  const double v = C.v, vp = fmax(v, 0.0), vm = fmin(v, 0.0);
  slopes1(C, L);
  __syncthreads();
  double gl, gr;
  ghosts1(C, L, gl, gr);
  double acc[1] = {0.0};
  for (int j = 0; j < L.nx; ++j) {
    const double fj = C.on ? L.f[(int64_t)j * N + k] : 0.0;
    double m[1] = {C.w * fj};
    wsum<1>(m);
    const double nu = C.o.bgk_nu > 0.0 ? C.o.bgk_nu : 2.0 * m[0];
    double th[3];
    (void)maxwellian1(fj, v, C.on, C.w, th);
    if (!C.on) continue;
    const double sj = L.S[(int64_t)j * N + k];
    const double m_j = fj + 0.5 * sj, p_j = fj - 0.5 * sj;
    const double m_l = j > 0 ? L.f[(int64_t)(j - 1) * N + k] + 0.5 * L.S[(int64_t)(j - 1) * N + k] : gl;
    const double p_r = j < L.nx - 1 ? L.f[(int64_t)(j + 1) * N + k] - 0.5 * L.S[(int64_t)(j + 1) * N + k] : gr;
    double R = (vp * (m_j - m_l) + vm * (p_r - p_j)) / L.dx - nu * (gau(th, v) - fj) / C.I->eps;
    if (L.b) R = L.b[(int64_t)j * N + k] - R;
    else R = -R;
    if (store) L.R[(int64_t)j * N + k] = R;
    acc[0] += R * R;
  }
  wsum<1>(acc);
  __syncthreads();
  return sqrt(L.dx * C.w * acc[0]);
}

// one FAS V-cycle from level 0 (eq. coarse; the exits of the 1D multigrid
// unless mg.fixed), per instance
__device__ void vcycle1(Ctx1& C, double* f0, double* ws, const MG1& mg) {
  const int N = C.N, k = threadIdx.x;
  int lstop = 0;
  for (int l = 0;; ++l) {
    Lev1 L = level_of(*C.I, f0, ws, N, l);
    for (int q = 0; q < mg.nu1; ++q) sgs1(C, L);
    if (L.nx <= mg.coarsest) {
      const double r0 = mg.fixed ? 0.0 : residual1(C, L, false);
      for (int q = 0; q < mg.coarse_iters; ++q) {
        if (!mg.fixed && residual1(C, L, false) <= 0.1 * r0) break;
        sgs1(C, L);
      }
      lstop = l;
      break;
    }
    const double rn = residual1(C, L, true);  // L.R = b - R(f)
    if (!mg.fixed && rn < mg.tol) {
      lstop = l;
      break;
    }
    Lev1 Cl = level_of(*C.I, f0, ws, N, l + 1);
    // f_H = restrict(f_h), C0 = f_H; b_H = R_H(f_H) + restrict(b_h - R_h(f_h))
    if (C.on)
      for (int J = 0; J < Cl.nx; ++J) {
        const double a = 0.5 * (L.f[(int64_t)(2 * J) * N + k] + L.f[(int64_t)(2 * J + 1) * N + k]);
        Cl.f[(int64_t)J * N + k] = a;
        Cl.c0[(int64_t)J * N + k] = a;
      }
    __syncthreads();
    double* bsave = Cl.b;
    Cl.b = nullptr;
    (void)residual1(C, Cl, true);  // Cl.R = -R_H(f_H)
    Cl.b = bsave;
    if (C.on)
      for (int J = 0; J < Cl.nx; ++J) {
        const double rr = 0.5 * (L.R[(int64_t)(2 * J) * N + k] + L.R[(int64_t)(2 * J + 1) * N + k]);
        Cl.b[(int64_t)J * N + k] = -Cl.R[(int64_t)J * N + k] + rr;
      }
    __syncthreads();
  }
  for (int l = lstop - 1; l >= 0; --l) {
    Lev1 L = level_of(*C.I, f0, ws, N, l);
    Lev1 Cl = level_of(*C.I, f0, ws, N, l + 1);
    if (C.on)
      for (int j = 0; j < L.nx; ++j)
        L.f[(int64_t)j * N + k] += Cl.f[(int64_t)(j / 2) * N + k] - Cl.c0[(int64_t)(j / 2) * N + k];
    __syncthreads();
    for (int q = 0; q < mg.nu2; ++q) sgs1(C, L);
  }
}

__global__ __launch_bounds__(64) void k_slab1v(const Inst1* __restrict__ inst, double* f, double* ws,
                                               const double* __restrict__ nodes, int N, double w, Opts1 o, int op,
                                               int n, MG1 mg, double* __restrict__ res_out,
                                               unsigned long long* __restrict__ stats) {
  const Inst1 I = inst[blockIdx.x];
  Ctx1 C{&I, N, threadIdx.x < N ? nodes[threadIdx.x] : 0.0, w, (int)threadIdx.x < N, o, 0, 0, 0};
  Lev1 L0 = level_of(I, f, ws, N, 0);
  for (int it = 0; it < (op == 2 ? 0 : n); ++it) {
    if (op == 0) sgs1(C, L0);
    else vcycle1(C, f, ws, mg);
    rescale1(C, L0);
  }
  const double r = residual1(C, L0, false);
  if (threadIdx.x == 0) {
    res_out[blockIdx.x] = r;
    atomicAdd(&stats[0], C.it_sum);
    atomicAdd(&stats[1], C.visit_sum);
    atomicAdd(&stats[2], C.fb_sum);
  }
}

}  // namespace

struct Slab1V {
  std::vector<Inst1> h;
  Inst1* d_inst = nullptr;
  double* ws = nullptr;
  double* d_res = nullptr;
  unsigned long long* d_stats = nullptr;
  Opts1 o{};
};

bz_status slab1v_create(bz_ctx* ctx, const bz_slab_desc* d, Slab1V** out) {
  *out = nullptr;
  if (d->collision != BZ_COLL_BGK)
    return set_err(ctx, BZ_EUNSUPPORTED, "one velocity dimension: the BGK slab of Section 4.1 only");
  if (d->inner.fallback != BZ_FALLBACK_FP)
    return set_err(ctx, BZ_EUNSUPPORTED, "one velocity dimension: fallback to the plain iteration only");
  auto* s = new Slab1V();
  s->o = Opts1{d->inner.mode, d->inner.tol, d->inner.max_iter, d->inner.fixed_iters, d->order == 2 ? 2 : 1,
               d->limiter, d->bgk_nu};
  int64_t off = 0, wsz = 0;
  for (int i = 0; i < d->n_instances; ++i) {
    const bz_slab_instance& in = d->instances[i];
    if (in.bc_L != BZ_BC_WALL || in.bc_R != BZ_BC_WALL || in.U_L[1] != 0.0 || in.U_L[2] != 0.0 ||
        in.U_R[1] != 0.0 || in.U_R[2] != 0.0) {
      delete s;
      return set_err(ctx, BZ_EUNSUPPORTED, "one velocity dimension: walls at rest only");
    }
    Inst1 I{};
    I.off = off;
    I.ws = wsz;
    I.nx = in.nx;
    I.dx = (in.xR - in.xL) / in.nx;
    I.eps = in.eps;
    I.mass = in.mass;
    I.T[0] = in.T_L;
    I.T[1] = in.T_R;
    int nx = in.nx, nl = 1;
    wsz += level1_doubles(nx, ctx->N);
    while (nx % 2 == 0 && nx > 1) {
      nx /= 2;
      wsz += level1_doubles(nx, ctx->N);
      ++nl;
    }
    I.nlev = nl;
    s->h.push_back(I);
    off += in.nx;
  }
  const size_t ni = s->h.size();
  bool ok = hipMalloc((void**)&s->d_inst, ni * sizeof(Inst1)) == hipSuccess &&
            hipMalloc((void**)&s->ws, (size_t)wsz * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&s->d_res, ni * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&s->d_stats, 3 * sizeof(unsigned long long)) == hipSuccess;
  if (ok) ok = hipMemcpy(s->d_inst, s->h.data(), ni * sizeof(Inst1), hipMemcpyHostToDevice) == hipSuccess;
  if (ok) ok = hipMemset(s->ws, 0, (size_t)wsz * sizeof(double)) == hipSuccess;
  if (!ok) {
    slab1v_destroy(s);
    return set_err(ctx, BZ_ENOMEM, "one-velocity slab workspace");
  }
  *out = s;
  return BZ_OK;
}

void slab1v_destroy(Slab1V* s) {
  if (!s) return;
  void* ptrs[] = {s->d_inst, s->ws, s->d_res, s->d_stats};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete s;
}

bz_status slab1v_run(bz_ctx* ctx, Slab1V* s, double* f, int op, int n, const bz_mg_opts* mg, double* residual_out,
                     bz_sweep_stats* stats, hipStream_t st) {
  if (op < 0 || op >= kOps || n < 0) return set_err(ctx, BZ_EINVAL, "bad one-velocity slab call");
  MG1 m{};
  if (op == 1) {
    if (!mg || mg->coarsest < 1 || mg->nu1 < 0 || mg->nu2 < 0 || mg->coarse_iters < 0 || !(mg->tol >= 0))
      return set_err(ctx, BZ_EINVAL, "bad multigrid options");
    for (const Inst1& I : s->h) {
      int nx = I.nx, l = 1;
      while (nx > mg->coarsest && nx % 2 == 0) {
        nx /= 2;
        ++l;
      }
      if (nx != mg->coarsest || l > I.nlev) return set_err(ctx, BZ_EINVAL, "cell count must be coarsest * 2^k");
    }
    m = MG1{mg->coarsest, mg->nu1, mg->nu2, mg->coarse_iters, mg->fixed_cycle != 0 ? 1 : 0, mg->tol};
  }
  BZ_HIP(hipMemsetAsync(s->d_stats, 0, 3 * sizeof(unsigned long long), st));
  hipLaunchKernelGGL(k_slab1v, dim3((unsigned)s->h.size()), dim3(64), 0, st, s->d_inst, f, s->ws, ctx->d_nodes,
                     ctx->N, ctx->w, s->o, op, n, m, s->d_res, s->d_stats);
  BZ_HIP(hipGetLastError());
  std::vector<double> res(s->h.size());
  unsigned long long h[3] = {0, 0, 0};
  BZ_HIP(hipMemcpyAsync(res.data(), s->d_res, res.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  BZ_HIP(hipMemcpyAsync(h, s->d_stats, sizeof(h), hipMemcpyDeviceToHost, st));
  BZ_HIP(hipStreamSynchronize(st));
  if (residual_out)
    for (size_t i = 0; i < res.size(); ++i) residual_out[i] = res[i];
  if (stats) {
    stats->n_iters = n;
    stats->inner_iters = (int64_t)h[0];
    stats->visits = (int64_t)h[1];
    stats->fallbacks = (int64_t)h[2];
    stats->learned = 0;
  }
  return BZ_OK;
}

}  // namespace bz
