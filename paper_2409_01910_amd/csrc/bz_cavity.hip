// SGS scans on the unit square with two-dimensional velocities: the
// lid-driven cavity family of Section 4.2.
//
// One SGS iteration is four scans, lexicographic along (+x, +y), (-x, -y),
// (-x, +y) and (+x, -y), then the uniform mass rescale of eq. mass_conserv.
// Before each scan one batched pass computes every cell's collision split
// P = Q - nu (M - f) (eq. Pf, explicit in eq. SGS) and stores -P/eps.  Within a
// scan a visit reads the latest values of its four neighbours.  Cells with
// equal i + j (in scan order) do not neighbour each other, so the scan runs as
// nx + ny - 1 launches, one per anti-diagonal, with one workgroup per cell;
// the result is that of the lexicographic order exactly.
//
// A visit assembles the transport right-hand side
//   r = (-v1+ f_W + v1- f_E) / dx + (-v2+ f_S + v2- f_N) / dy - P / eps,
// with diffuse-wall ghosts rho_w M_w (eq. boundary; rho_w from the discrete
// zero-mass-flux balance with the cell's latest value), and solves
// eq. inner_eqn, c g + r = (nu/eps)(M[g] - g), c = |v1|/dx + |v2|/dy, by the
// preconditioned iteration of eqs. step1 and step2 (or the plain eq. fix_point):
// step 1's weighted Newton and the discrete Maxwellian are 4-parameter Newton
// solves whose sums separate over the two velocity axes (1D sums per wave).
#include <cmath>
#include <vector>

#include "bz_common.hpp"
#include "bz_internal.hpp"

// One grid level: level 0 works on the caller's field; coarser levels (nx and
// ny halved each time) own theirs, with the FAS source b and the restricted
// copy f0 of eq. coarse.
struct CavLevel {
  int nx = 0, ny = 0, ncell = 0;
  double dx = 0, dy = 0;
  double* f = nullptr;
  double* b = nullptr;        // [ncell][K] FAS source (null on level 0)
  double* f0 = nullptr;       // [ncell][K] restricted fine state (coarse levels)
  double* res = nullptr;      // [ncell][K] b - R(f)
  double* Q = nullptr;        // [ncell][K]
  double* rs = nullptr;       // [ncell][K] -P / eps - b
  double* theta = nullptr;    // [ncell][4]
  double* nu = nullptr;       // [ncell]
  double* part = nullptr;     // [ncell + 1] per-cell partial sums and their total
  double* sx = nullptr;       // [ncell][K] slopes along x and y (second order)
  double* sy = nullptr;
  double* T = nullptr;        // [ncell][K] transport part of the scan's iterate (learned start)
  double* G = nullptr;        // [ncell][K] learned candidates
};

struct bz_cavity {
  bz_ctx* ctx = nullptr;
  double eps = 0, mass = 0;
  bz_wall walls[4]{};
  int collision = 0;
  double bgk_nu = 0;
  bz_solve_opts opts{};
  int order = 1;
  int uy = 0;  // uniform along y: no y transport or y walls, two scans, x-only coarsening
  int limiter = 0;  // second order: 0 none, 1 minmod
  std::vector<CavLevel> lv;
  unsigned long long* d_stats = nullptr;  // inner updates, visits, fallbacks, learned starts taken
  bz_mlp* ws = nullptr;                   // learned start (bz_cavity_ws_attach), or null
};

namespace bz {
namespace {

constexpr int kCavThreads = 256;
constexpr int kCavOwn = 9;  // ceil(48^2 / 256)

struct CavWalls {
  double T[4], U1[4], U2[4];
};

__device__ __forceinline__ double gauss2c(const double* th, double x, double y) {
  return exp(th[0] + th[1] * x + th[2] * y - th[3] * (x * x + y * y));
}

__device__ __forceinline__ double wall_m(const CavWalls& wl, int s, double x, double y) {
  const double a = x - wl.U1[s], b = y - wl.U2[s];
  return exp(-(a * a + b * b) / (2.0 * wl.T[s])) / (2.0 * kPi * wl.T[s]);
}

// s[0..3] = sum w c phi_i exp(theta.phi~), s[4..13] = sum w c phi_i phi_j exp(theta.phi~)
// (upper triangle by rows), phi = (1, x, y, x^2 + y^2), over the N x N grid.  On
// the tensor grid the Gaussian factorises, exp(alpha) E0(x) E1(y) with
// E_a(u) = exp(beta_a u - gamma u^2), and the weight is c = 1 or the additive
// c = a0 |x| + a1 |y|, so every sum is a combination of 1D sums over the N nodes:
//   sum c x^p y^q E0 E1 = a0 Ac_p B_q + a1 A_p Bc_q   (or A_p B_q for c = 1),
//   A_p = sum x^p E0, Ac_p = sum |x| x^p E0, B_q, Bc_q the same with E1.
// Each wave forms the 1D sums itself (lane l holds node l, N <= 64) with DPP
// reductions: no LDS and no block synchronisation.
__device__ __forceinline__ void sep_sums(const double* th, const double* nodes, int N, double w, bool weighted,
                                         double a0, double a1, double (&s)[14]) {
  const int l = threadIdx.x & 63;
  const bool on = l < N;
  const double u = on ? nodes[l] : 0.0;
  const double e0 = on ? exp(th[1] * u - th[3] * u * u) : 0.0;
  const double e1 = on ? exp(th[2] * u - th[3] * u * u) : 0.0;
  const double au = fabs(u);
  double v[20];
  double up = 1.0;
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    v[p] = e0 * up;
    v[5 + p] = e1 * up;
    v[10 + p] = au * e0 * up;
    v[15 + p] = au * e1 * up;
    up *= u;
  }
  if (weighted) {
    wave_sums_dpp<20>(v);
  } else {  // c = 1 needs only A_p and B_q
    double* v10 = v;
    wave_sums_dpp<10>(*reinterpret_cast<double(*)[10]>(v10));
  }
  auto S = [&](int p, int q) { return weighted ? a0 * v[10 + p] * v[5 + q] + a1 * v[p] * v[15 + q] : v[p] * v[5 + q]; };
  const double sc = w * exp(th[0]);
  s[0] = sc * S(0, 0);
  s[1] = sc * S(1, 0);
  s[2] = sc * S(0, 1);
  s[3] = sc * (S(2, 0) + S(0, 2));
  s[4] = s[0];
  s[5] = s[1];
  s[6] = s[2];
  s[7] = s[3];
  s[8] = sc * S(2, 0);
  s[9] = sc * S(1, 1);
  s[10] = sc * (S(3, 0) + S(1, 2));
  s[11] = sc * S(0, 2);
  s[12] = sc * (S(2, 1) + S(0, 3));
  s[13] = sc * (S(4, 0) + 2.0 * S(2, 2) + S(0, 4));
}

__device__ __forceinline__ bool spd4_solve(double G[4][4], const double b[4], double y[4]) {
  double d[4], z[4];
  for (int j = 0; j < 4; ++j) {
    double dj = G[j][j];
    for (int k = 0; k < j; ++k) dj -= G[j][k] * G[j][k] * d[k];
    d[j] = dj;
    for (int i = j + 1; i < 4; ++i) {
      double t = G[i][j];
      for (int k = 0; k < j; ++k) t -= G[i][k] * G[j][k] * d[k];
      G[i][j] = t / dj;
    }
  }
  for (int i = 0; i < 4; ++i) {
    double t = b[i];
    for (int k = 0; k < i; ++k) t -= G[i][k] * z[k];
    z[i] = t;
  }
  for (int i = 3; i >= 0; --i) {
    double t = z[i] / d[i];
    for (int k = i + 1; k < 4; ++k) t -= G[k][i] * y[k];
    y[i] = t;
  }
  bool ok = true;
  for (int i = 0; i < 4; ++i) ok = ok && isfinite(y[i]);
  return ok;
}

// Newton for sum w c phi exp(theta.phi~) = t (c = 1: the discrete Maxwellian,
// eq. discrete_conservation; c = |v1|/dx + |v2|/dy: step 1, eq. step1).  With
// guess, theta starts from the continuous moments of t; otherwise from th.
// Step halving while the max-norm residual does not decrease.  Returns true
// when converged (residual <= 1e-13 (|t_0| + |t_3|), or a stalled step with
// residual <= 1e-10 of that scale).
__device__ bool newton4(double (&th)[4], const double (&t)[4], bool guess, const double* nodes, int N, double w,
                        bool weighted, double a0, double a1) {
  if (guess) {
    const double rho = t[0], U0 = t[1] / rho, U1 = t[2] / rho;
    double T = (t[3] / rho - U0 * U0 - U1 * U1) / 2.0;
    if (!(T > 1e-3)) T = 1e-3;
    th[0] = log(rho / (2.0 * kPi * T)) - (U0 * U0 + U1 * U1) / (2.0 * T);
    th[1] = U0 / T;
    th[2] = U1 / T;
    th[3] = 1.0 / (2.0 * T);
  }
  const double scale = fabs(t[0]) + fabs(t[3]) + 1e-300, tol = 1e-13;
  double s[14], r[4];
  sep_sums(th, nodes, N, w, weighted, a0, a1, s);
  double nrm = 0.0;
  for (int i = 0; i < 4; ++i) {
    r[i] = s[i] - t[i];
    nrm = fmax(nrm, fabs(r[i]));
  }
  if (!isfinite(nrm)) nrm = INFINITY;
  for (int it = 0; it < 60; ++it) {
    if (nrm <= tol * scale) return true;
    double G[4][4], rhs[4], step[4];
    int o = 4;
    bool fin = true;
    for (int a = 0; a < 4; ++a)
      for (int b = a; b < 4; ++b) {
        G[a][b] = G[b][a] = s[o];
        fin = fin && isfinite(s[o]);
        ++o;
      }
    if (!fin) return false;
    for (int a = 0; a < 4; ++a) rhs[a] = -r[a];
    if (!spd4_solve(G, rhs, step)) return false;
    step[3] = -step[3];
    double a = 1.0, thn[4], sn[14], n_new = INFINITY;
    while (true) {
      for (int i = 0; i < 4; ++i) thn[i] = th[i] + a * step[i];
      sep_sums(thn, nodes, N, w, weighted, a0, a1, sn);
      n_new = 0.0;
      for (int i = 0; i < 4; ++i) n_new = fmax(n_new, fabs(sn[i] - t[i]));
      if (!isfinite(n_new)) n_new = INFINITY;
      if (isfinite(n_new) && (n_new < nrm || a < 1e-4) && thn[3] > 0.0) break;
      a *= 0.5;
      if (a < 1e-6) break;
    }
    double dmax = 0.0, tmax = 0.0;
    for (int i = 0; i < 4; ++i) {
      dmax = fmax(dmax, fabs(thn[i] - th[i]));
      tmax = fmax(tmax, fabs(th[i]));
    }
    for (int i = 0; i < 4; ++i) {
      th[i] = thn[i];
      r[i] = sn[i] - t[i];
    }
    for (int q = 0; q < 14; ++q) s[q] = sn[q];
    nrm = n_new;
    if (dmax <= 1e-15 * (1.0 + tmax)) return nrm <= 1e-10 * scale;
  }
  return nrm <= tol * scale;
}

// the cell (i, j) of anti-diagonal dd of scan (sx, sy), block b of the launch
__device__ __forceinline__ void diag_cell(int nx, int ny, int dd, int sx, int sy, int b, int& i, int& j) {
  const int lo = dd - (ny - 1) > 0 ? dd - (ny - 1) : 0;
  const int ip = lo + b, jp = dd - ip;
  i = sx > 0 ? ip : nx - 1 - ip;
  j = sy > 0 ? jp : ny - 1 - jp;
}

// Wall densities of cell (i, j): dens[s] = rho_w for each side s the cell
// touches (sum over the outgoing half-space of |v_n| times the adjacent face
// value, f -+ s/2 with the cell's slopes when given, against the incoming flux
// of the unit wall Maxwellian), 0 elsewhere.  Every thread returns them.
__device__ __forceinline__ void wall_densities(const double* fc, const double* sxc, const double* syc, int i, int j,
                                               int nx, int ny, int uy, const CavWalls& wl, const double* nodes, int N,
                                               double* red, double (&dens)[4]) {
  const int K = N * N;
  double v[8];
  for (int q = 0; q < 8; ++q) v[q] = 0.0;
  const bool touch[4] = {i == 0, i == nx - 1, !uy && j == 0, !uy && j == ny - 1};
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double x = nodes[k / N], y = nodes[k % N], fv = fc[k];
    const double hx = sxc ? 0.5 * sxc[k] : 0.0, hy = syc ? 0.5 * syc[k] : 0.0;
    for (int s = 0; s < 4; ++s) {
      if (!touch[s]) continue;
      const double vn = (s < 2 ? x : y) * (s % 2 == 0 ? 1.0 : -1.0);  // along the inward normal
      // the adjacent face value f -+ s/2
      const double face = s == 0 ? fv - hx : s == 1 ? fv + hx : s == 2 ? fv - hy : fv + hy;
      if (vn < 0) v[2 * s] += -vn * face;
      if (vn > 0) v[2 * s + 1] += vn * wall_m(wl, s, x, y);
    }
  }
  block_sum<8>(v, red);
  for (int s = 0; s < 4; ++s) dens[s] = touch[s] ? v[2 * s] / v[2 * s + 1] : 0.0;
}

// One visit per workgroup: the cells of anti-diagonal dd of scan (sx, sy).
template <int OWN>
__global__ void __launch_bounds__(kCavThreads) k_cav_visit(double* __restrict__ f, const double* __restrict__ rs,
                                                           const double* __restrict__ nu,
                                                           const double* __restrict__ slx,
                                                           const double* __restrict__ sly, int nx, int ny, int uy,
                                                           int dd,
                                                           int sx, int sy, double dx, double dy, double eps,
                                                           CavWalls wl, const double* __restrict__ nodes, int N,
                                                           double w, int mode, double tol, int max_iter, int fixed,
                                                           int relax, unsigned long long* __restrict__ stats,
                                                           const double* __restrict__ Gc) {
  __shared__ double red[14 * (kCavThreads / 64)];
  const int K = N * N;
  int i, j;
  diag_cell(nx, ny, dd, sx, sy, blockIdx.x, i, j);
  const size_t cell = (size_t)i * ny + j;
  double* fc = f + cell * K;
  double dens[4];
  wall_densities(fc, slx ? slx + cell * K : nullptr, sly ? sly + cell * K : nullptr, i, j, nx, ny, uy, wl, nodes, N,
                 red, dens);
  const double* fW = i > 0 ? f + (cell - ny) * K : nullptr;
  const double* fE = i < nx - 1 ? f + (cell + ny) * K : nullptr;
  const double* fS = j > 0 ? f + (cell - 1) * K : nullptr;
  const double* fN = j < ny - 1 ? f + (cell + 1) * K : nullptr;
  const double lam = nu[cell] / eps;
  double x[OWN], y[OWN], c[OWN], g[OWN], r[OWN], Mg[OWN];
#pragma unroll
  for (int q = 0; q < OWN; ++q) {
    const int k = threadIdx.x + q * kCavThreads;
    x[q] = y[q] = c[q] = g[q] = r[q] = Mg[q] = 0.0;
    if (k < K) {
      x[q] = nodes[k / N];
      y[q] = nodes[k % N];
      const double W = fW ? fW[k] : dens[0] * wall_m(wl, 0, x[q], y[q]);
      const double E = fE ? fE[k] : dens[1] * wall_m(wl, 1, x[q], y[q]);
      if (uy) {
        c[q] = fabs(x[q]) / dx;
        r[q] = (-fmax(x[q], 0.0) * W + fmin(x[q], 0.0) * E) / dx + rs[cell * K + k];
      } else {
        const double S = fS ? fS[k] : dens[2] * wall_m(wl, 2, x[q], y[q]);
        const double Nn = fN ? fN[k] : dens[3] * wall_m(wl, 3, x[q], y[q]);
        c[q] = fabs(x[q]) / dx + fabs(y[q]) / dy;
        r[q] = (-fmax(x[q], 0.0) * W + fmin(x[q], 0.0) * E) / dx + (-fmax(y[q], 0.0) * S + fmin(y[q], 0.0) * Nn) / dy +
               rs[cell * K + k];
      }
      g[q] = fc[k];
    }
  }
  // M[g] of the initial guess
  auto moments_of = [&](const double (&a)[OWN], double (&t)[4]) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < OWN; ++q) {
      const double e = threadIdx.x + q * kCavThreads < K ? w * a[q] : 0.0;
      v[0] += e;
      v[1] += x[q] * e;
      v[2] += y[q] * e;
      v[3] += (x[q] * x[q] + y[q] * y[q]) * e;
    }
    block_sum<4>(v, red);
    for (int q = 0; q < 4; ++q) t[q] = v[q];
  };
  const double a0 = 1.0 / dx, a1 = uy ? 0.0 : 1.0 / dy;  // c = a0 |v1| + a1 |v2|
  double th_g[4], t4[4];
  moments_of(g, t4);
  (void)newton4(th_g, t4, true, nodes, N, w, false, a0, a1);
#pragma unroll
  for (int q = 0; q < OWN; ++q) Mg[q] = gauss2c(th_g, x[q], y[q]);
  bool learned = false;
  if (Gc) {
    // learned candidate: taken when M[G] exists, step 1 from G satisfies eq.
    // existence and G's inner residual (with this visit's r) is below g's
    double gG[OWN], MG[OWN], th_G[4], tG[4];
#pragma unroll
    for (int q = 0; q < OWN; ++q) {
      const int k = threadIdx.x + q * kCavThreads;
      gG[q] = k < K ? Gc[cell * K + k] : 0.0;
    }
    moments_of(gG, tG);
    bool ok = newton4(th_G, tG, true, nodes, N, w, false, a0, a1);
    double e[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < OWN; ++q) {
      const int k = threadIdx.x + q * kCavThreads;
      MG[q] = ok ? gauss2c(th_G, x[q], y[q]) : 0.0;
      if (k < K) {
        const double eg = c[q] * g[q] + r[q] - lam * (Mg[q] - g[q]);
        const double eG = c[q] * gG[q] + r[q] - lam * (MG[q] - gG[q]);
        e[0] += eg * eg;
        e[1] += eG * eG;
        const double sv = w * (c[q] * (MG[q] - gG[q]) - r[q]);
        e[2] += sv;
        e[3] += x[q] * sv;
        e[4] += y[q] * sv;
        e[5] += (x[q] * x[q] + y[q] * y[q]) * sv;
      }
    }
    block_sum<6>(e, red);
    ok = ok && e[2] > 0.0 && e[2] * e[5] > e[3] * e[3] + e[4] * e[4] && e[1] < e[0];
    if (ok) {
      learned = true;
      for (int a = 0; a < 4; ++a) th_g[a] = th_G[a];
#pragma unroll
      for (int q = 0; q < OWN; ++q) {
        g[q] = gG[q];
        Mg[q] = MG[q];
      }
    }
  }
  double th_step[4] = {th_g[0], th_g[1], th_g[2], th_g[3]};
  bool fallback = mode == BZ_SOLVE_FP, fell = false;
  const int n = fixed > 0 ? fixed : max_iter;
  int it = 0;
  double res = INFINITY;
  // step 1's right-hand side s = sum w phi (c (M[g] - g) - r); after the first
  // update it comes from the same block pass as the inner residual
  double s4[4];
  bool have_s = false;
  for (; it < n;) {
    double Mstep[OWN];
    if (!fallback) {
      if (!have_s) {
        double sv[OWN];
#pragma unroll
        for (int q = 0; q < OWN; ++q) sv[q] = c[q] * (Mg[q] - g[q]) - r[q];
        moments_of(sv, s4);
      }
      bool ok = s4[0] > 0.0 && s4[0] * s4[3] > s4[1] * s4[1] + s4[2] * s4[2];
      if (!ok && relax) {
        // relaxed step 1 (Section 3.2, remark): (s + tau sum w phi c M[g]) / (1 + tau)
        double cm[OWN], m4[4];
#pragma unroll
        for (int q = 0; q < OWN; ++q) cm[q] = c[q] * Mg[q];
        moments_of(cm, m4);
        for (double tau = 1.0; tau <= 1048576.0; tau *= 2.0) {
          double st[4];
          for (int a = 0; a < 4; ++a) st[a] = (s4[a] + tau * m4[a]) / (1.0 + tau);
          if (st[0] > 0.0 && st[0] * st[3] > st[1] * st[1] + st[2] * st[2]) {
            for (int a = 0; a < 4; ++a) s4[a] = st[a];
            ok = true;
            break;
          }
        }
      }
      double th[4] = {th_step[0], th_step[1], th_step[2], th_step[3]};
      if (ok) ok = newton4(th, s4, false, nodes, N, w, true, a0, a1) && th[3] > 0.0;
      if (ok) {
        for (int a = 0; a < 4; ++a) th_step[a] = th[a];
#pragma unroll
        for (int q = 0; q < OWN; ++q) Mstep[q] = gauss2c(th, x[q], y[q]);
      } else {
        fallback = true;
        fell = true;
      }
    }
    if (fallback) {
#pragma unroll
      for (int q = 0; q < OWN; ++q) Mstep[q] = Mg[q];
    }
#pragma unroll
    for (int q = 0; q < OWN; ++q)
      g[q] = threadIdx.x + q * kCavThreads < K ? (lam * Mstep[q] - r[q]) / (c[q] + lam) : 0.0;
    moments_of(g, t4);
    // M[g]: Newton warm-started from the previous iterate's parameters (the
    // converged parameters do not depend on the start); from the continuous
    // moments when that start fails
    {
      double th_w[4] = {th_g[0], th_g[1], th_g[2], th_g[3]};
      if (newton4(th_w, t4, false, nodes, N, w, false, a0, a1)) {
        for (int a = 0; a < 4; ++a) th_g[a] = th_w[a];
      } else {
        (void)newton4(th_g, t4, true, nodes, N, w, false, a0, a1);
      }
    }
    // one block pass: the inner residual and the next update's step-1 moments
    double e2[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < OWN; ++q) {
      const int k = threadIdx.x + q * kCavThreads;
      Mg[q] = gauss2c(th_g, x[q], y[q]);
      if (k < K) {
        const double e = c[q] * g[q] + r[q] - lam * (Mg[q] - g[q]);
        e2[0] += e * e;
        const double sv = w * (c[q] * (Mg[q] - g[q]) - r[q]);
        e2[1] += sv;
        e2[2] += x[q] * sv;
        e2[3] += y[q] * sv;
        e2[4] += (x[q] * x[q] + y[q] * y[q]) * sv;
      }
    }
    block_sum<5>(e2, red);
    res = sqrt(w * e2[0]);
    for (int a = 0; a < 4; ++a) s4[a] = e2[1 + a];
    have_s = true;
    ++it;
    if (fixed <= 0 && res <= tol) break;
  }
  const bool finite = isfinite(res);
  if (finite) {
#pragma unroll
    for (int q = 0; q < OWN; ++q) {
      const int k = threadIdx.x + q * kCavThreads;
      if (k < K) fc[k] = g[q];
    }
  }
  if (threadIdx.x == 0) {
    atomicAdd(&stats[0], (unsigned long long)it);
    atomicAdd(&stats[1], 1ull);
    atomicAdd(&stats[2], fell ? 1ull : 0ull);
    if (learned) atomicAdd(&stats[3], 1ull);
  }
}

// transport part of a visit's right-hand side for every cell with all
// neighbours (and wall ghosts) from the iterate f: the upwind neighbour terms
// and, at second order, the static reconstruction terms of the slopes
__global__ void __launch_bounds__(kCavThreads) k_cav_transport(const double* __restrict__ f,
                                                               const double* __restrict__ slx,
                                                               const double* __restrict__ sly, int nx, int ny, int uy,
                                                               double dx, double dy, CavWalls wl,
                                                               const double* __restrict__ nodes, int N,
                                                               double* __restrict__ T) {
  __shared__ double red[8 * (kCavThreads / 64)];
  const int K = N * N;
  const size_t cell = blockIdx.x;
  const int i = (int)(cell / ny), j = (int)(cell - (size_t)i * ny);
  const double* fc = f + cell * K;
  double dens[4];
  wall_densities(fc, slx ? slx + cell * K : nullptr, sly ? sly + cell * K : nullptr, i, j, nx, ny, uy, wl, nodes, N,
                 red, dens);
  const double* fW = i > 0 ? f + (cell - ny) * K : nullptr;
  const double* fE = i < nx - 1 ? f + (cell + ny) * K : nullptr;
  const double* fS = j > 0 ? f + (cell - 1) * K : nullptr;
  const double* fN = j < ny - 1 ? f + (cell + 1) * K : nullptr;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double x = nodes[k / N], y = nodes[k % N];
    const double W = fW ? fW[k] : dens[0] * wall_m(wl, 0, x, y);
    const double E = fE ? fE[k] : dens[1] * wall_m(wl, 1, x, y);
    double t = (-fmax(x, 0.0) * W + fmin(x, 0.0) * E) / dx;
    if (!uy) {
      const double S = fS ? fS[k] : dens[2] * wall_m(wl, 2, x, y);
      const double Nn = fN ? fN[k] : dens[3] * wall_m(wl, 3, x, y);
      t += (-fmax(y, 0.0) * S + fmin(y, 0.0) * Nn) / dy;
    }
    if (slx) {
      const double xw = i > 0 ? slx[(cell - ny) * K + k] : 0.0, xe = i < nx - 1 ? slx[(cell + ny) * K + k] : 0.0;
      t -= (fmax(x, 0.0) * xw - x * slx[cell * K + k] + fmin(x, 0.0) * xe) / (2.0 * dx);
      if (!uy) {
        const double ys = j > 0 ? sly[(cell - 1) * K + k] : 0.0, yn = j < ny - 1 ? sly[(cell + 1) * K + k] : 0.0;
        t -= (fmax(y, 0.0) * ys - y * sly[cell * K + k] + fmin(y, 0.0) * yn) / (2.0 * dy);
      }
    }
    T[cell * K + k] = t;
  }
}

// rs = -(Q - nu (M_theta - f)) / eps (binary) or 0 (BGK), minus the FAS source b
// when given, and nu, per cell
__global__ void __launch_bounds__(kCavThreads) k_cav_static(const double* __restrict__ f, const double* __restrict__ Q,
                                                            const double* __restrict__ theta,
                                                            const double* __restrict__ b,
                                                            const double* __restrict__ slx,
                                                            const double* __restrict__ sly, int nx, int ny, int uy,
                                                            double dx, double dy, double* __restrict__ rs,
                                                            double* __restrict__ nu, const double* __restrict__ nodes,
                                                            int N, double w, double eps, int bgk, double bgk_nu,
                                                            double gam, double gfac) {
  __shared__ double red[1 * (kCavThreads / 64)];
  const int K = N * N;
  const size_t cell = blockIdx.x;
  const double* fc = f + cell * K;
  double v[1] = {0.0};
  for (int k = threadIdx.x; k < K; k += blockDim.x) v[0] += fc[k];
  block_sum<1>(v, red);
  const double rho = w * v[0];
  double nv;
  if (bgk) {
    nv = bgk_nu > 0 ? bgk_nu : 2.0 * kPi * rho;
  } else {
    const double* th = theta + cell * 4;
    nv = gam == 0.0 ? 2.0 * kPi * rho : 2.0 * kPi * rho * gfac * pow(0.5 / th[3], 0.5 * gam);
  }
  if (threadIdx.x == 0) nu[cell] = nv;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    double v0 = 0.0;
    if (slx) {  // second order: -(v1+ s_W - v1 s + v1- s_E) / 2dx - (same along y) / 2dy
      const int i = (int)(cell / ny), j = (int)(cell - (size_t)i * ny);
      const double x = nodes[k / N], y = nodes[k % N];
      const double xw = i > 0 ? slx[(cell - ny) * K + k] : 0.0, xe = i < nx - 1 ? slx[(cell + ny) * K + k] : 0.0;
      const double ys = j > 0 ? sly[(cell - 1) * K + k] : 0.0, yn = j < ny - 1 ? sly[(cell + 1) * K + k] : 0.0;
      v0 = -((fmax(x, 0.0) * xw - x * slx[cell * K + k] + fmin(x, 0.0) * xe) / (2.0 * dx));
      if (!uy) v0 -= (fmax(y, 0.0) * ys - y * sly[cell * K + k] + fmin(y, 0.0) * yn) / (2.0 * dy);
    }
    if (!bgk) {
      const double M = gauss2c(theta + cell * 4, nodes[k / N], nodes[k % N]);
      v0 -= (Q[cell * K + k] - nv * (M - fc[k])) / eps;
    }
    rs[cell * K + k] = b ? v0 - b[cell * K + k] : v0;
  }
}

// per-cell sum of w (b - R)^2 with R = v.grad f - Q/eps (BGK: Q = nu (M - f)), b the FAS
// source (0 when null); the field b - R into res when non-null
__global__ void __launch_bounds__(kCavThreads) k_cav_resid(const double* __restrict__ f, const double* __restrict__ Q,
                                                           const double* __restrict__ theta, int nx, int ny, int uy,
                                                           double dx, double dy, double eps, CavWalls wl,
                                                           const double* __restrict__ nodes, int N, double w, int bgk,
                                                           double bgk_nu, const double* __restrict__ b,
                                                           const double* __restrict__ slx,
                                                           const double* __restrict__ sly,
                                                           double* __restrict__ res, double* __restrict__ part) {
  __shared__ double red[8 * (kCavThreads / 64)];
  const int K = N * N;
  const int cell = blockIdx.x, i = cell / ny, j = cell - i * ny;
  const double* fc = f + (size_t)cell * K;
  const double* sxc = slx ? slx + (size_t)cell * K : nullptr;
  const double* syc = sly ? sly + (size_t)cell * K : nullptr;
  double dens[4];
  wall_densities(fc, sxc, syc, i, j, nx, ny, uy, wl, nodes, N, red, dens);
  double nv = 0.0;
  if (bgk) {
    double v[1] = {0.0};
    for (int k = threadIdx.x; k < K; k += blockDim.x) v[0] += fc[k];
    block_sum<1>(v, red);
    nv = bgk_nu > 0 ? bgk_nu : 2.0 * kPi * w * v[0];
  }
  const double* fW = i > 0 ? fc - (size_t)ny * K : nullptr;
  const double* fE = i < nx - 1 ? fc + (size_t)ny * K : nullptr;
  const double* fS = j > 0 ? fc - K : nullptr;
  const double* fN = j < ny - 1 ? fc + K : nullptr;
  double acc[1] = {0.0};
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double x = nodes[k / N], y = nodes[k % N], fv = fc[k];
    const double W = fW ? fW[k] : dens[0] * wall_m(wl, 0, x, y);
    const double E = fE ? fE[k] : dens[1] * wall_m(wl, 1, x, y);
    const double S = fS ? fS[k] : dens[2] * wall_m(wl, 2, x, y);
    const double Nn = fN ? fN[k] : dens[3] * wall_m(wl, 3, x, y);
    const double q = bgk ? nv * (gauss2c(theta + (size_t)cell * 4, x, y) - fv) : Q[(size_t)cell * K + k];
    // face values: f +- s/2 of the cell, neighbours' faces toward it, ghosts without slope
    double xw = 0.0, xe = 0.0, ys = 0.0, yn = 0.0, hx = 0.0, hy = 0.0;
    if (sxc) {
      xw = fW ? 0.5 * sxc[k - (ptrdiff_t)ny * K] : 0.0;
      xe = fE ? 0.5 * sxc[k + (ptrdiff_t)ny * K] : 0.0;
      ys = fS ? 0.5 * syc[k - K] : 0.0;
      yn = fN ? 0.5 * syc[k + K] : 0.0;
      hx = 0.5 * sxc[k];
      hy = 0.5 * syc[k];
    }
    double R = (fmax(x, 0.0) * ((fv + hx) - (W + xw)) + fmin(x, 0.0) * ((E - xe) - (fv - hx))) / dx;
    if (!uy) R += (fmax(y, 0.0) * ((fv + hy) - (S + ys)) + fmin(y, 0.0) * ((Nn - yn) - (fv - hy))) / dy;
    R -= q / eps;
    const double rb = (b ? b[(size_t)cell * K + k] : 0.0) - R;  // b - R(f)
    if (res) res[(size_t)cell * K + k] = rb;
    acc[0] += rb * rb;
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) part[cell] = w * acc[0];
}

__global__ void __launch_bounds__(kCavThreads) k_cav_cellsum(const double* __restrict__ f, int K,
                                                             double* __restrict__ part) {
  __shared__ double red[kCavThreads / 64];
  const double* fc = f + (size_t)blockIdx.x * K;
  double v[1] = {0.0};
  for (int k = threadIdx.x; k < K; k += blockDim.x) v[0] += fc[k];
  block_sum<1>(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// f <- f C / (dx dy w sum f); every block sums the per-cell partials itself
__global__ void __launch_bounds__(kCavThreads) k_cav_rescale(double* __restrict__ f, int K, int ncell,
                                                             const double* __restrict__ part, double cw, double C) {
  __shared__ double red[kCavThreads / 64];
  double v[1] = {0.0};
  for (int q = threadIdx.x; q < ncell; q += blockDim.x) v[0] += part[q];
  block_sum<1>(v, red);
  const double sc = C / (cw * v[0]);
  double* fc = f + (size_t)blockIdx.x * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) fc[k] *= sc;
}

__global__ void __launch_bounds__(kCavThreads) k_cav_total(const double* __restrict__ part, int ncell,
                                                           double* __restrict__ out) {
  __shared__ double red[kCavThreads / 64];
  double v[1] = {0.0};
  for (int q = threadIdx.x; q < ncell; q += blockDim.x) v[0] += part[q];
  block_sum<1>(v, red);
  if (threadIdx.x == 0) out[0] = v[0];
}

__device__ __forceinline__ double minmod2(double d1, double d0) {
  return d1 * d0 > 0.0 ? copysign(fmin(fabs(d1), fabs(d0)), d1) : 0.0;
}

// slopes of eq. slope along x and y: centred inside (minmod of the one-sided
// differences with the limiter), one-sided at the ends of each line
__global__ void __launch_bounds__(kCavThreads) k_cav_slopes(const double* __restrict__ f, int nx, int ny, int K,
                                                            int lim, double* __restrict__ sx, double* __restrict__ sy) {
  const size_t cell = blockIdx.x;
  const int i = (int)(cell / ny), j = (int)(cell - (size_t)i * ny);
  const double* c = f + cell * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    double a = 0.0, b = 0.0;
    if (nx > 1) {
      if (i == 0) a = c[k + (size_t)ny * K] - c[k];
      else if (i == nx - 1) a = c[k] - c[k - (size_t)ny * K];
      else if (lim) a = minmod2(c[k + (size_t)ny * K] - c[k], c[k] - c[k - (size_t)ny * K]);
      else a = 0.5 * (c[k + (size_t)ny * K] - c[k - (size_t)ny * K]);
    }
    if (ny > 1) {
      if (j == 0) b = c[k + K] - c[k];
      else if (j == ny - 1) b = c[k] - c[k - K];
      else if (lim) b = minmod2(c[k + K] - c[k], c[k] - c[k - K]);
      else b = 0.5 * (c[k + K] - c[k - K]);
    }
    sx[cell * K + k] = a;
    sy[cell * K + k] = b;
  }
}

__global__ void __launch_bounds__(kCavThreads) k_cav_negate(double* __restrict__ a, int K) {
  double* o = a + (size_t)blockIdx.x * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) o[k] = -o[k];
}

// coarse cell (I, J) <- average of its four children
__global__ void __launch_bounds__(kCavThreads) k_cav_restrict(const double* __restrict__ fine, int nyf,
                                                              double* __restrict__ coarse, int nyc, int K, int uy) {
  double* o = coarse + (size_t)blockIdx.x * K;
  if (uy) {  // two children along x
    const double* a = fine + (size_t)(2 * blockIdx.x) * K;
    const double* b = a + K;
    for (int k = threadIdx.x; k < K; k += blockDim.x) o[k] = 0.5 * (a[k] + b[k]);
    return;
  }
  const int I = blockIdx.x / nyc, J = blockIdx.x - (blockIdx.x / nyc) * nyc;
  const double* a = fine + ((size_t)(2 * I) * nyf + 2 * J) * K;
  const double* b = fine + ((size_t)(2 * I + 1) * nyf + 2 * J) * K;
  const double* c = fine + ((size_t)(2 * I) * nyf + 2 * J + 1) * K;
  const double* d = fine + ((size_t)(2 * I + 1) * nyf + 2 * J + 1) * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) o[k] = 0.25 * (a[k] + b[k] + c[k] + d[k]);
}

// bc <- bc + restrict(res): bc holds R_H(f0) on entry (eq. coarse)
__global__ void __launch_bounds__(kCavThreads) k_cav_fas_rhs(double* __restrict__ bc, int nyc,
                                                             const double* __restrict__ res, int nyf, int K, int uy) {
  if (uy) {
    const double* a = res + (size_t)(2 * blockIdx.x) * K;
    const double* b = a + K;
    double* o = bc + (size_t)blockIdx.x * K;
    for (int k = threadIdx.x; k < K; k += blockDim.x) o[k] += 0.5 * (a[k] + b[k]);
    return;
  }
  const int I = blockIdx.x / nyc, J = blockIdx.x - (blockIdx.x / nyc) * nyc;
  const double* a = res + ((size_t)(2 * I) * nyf + 2 * J) * K;
  const double* b = res + ((size_t)(2 * I + 1) * nyf + 2 * J) * K;
  const double* c = res + ((size_t)(2 * I) * nyf + 2 * J + 1) * K;
  const double* d = res + ((size_t)(2 * I + 1) * nyf + 2 * J + 1) * K;
  double* o = bc + (size_t)blockIdx.x * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) o[k] += 0.25 * (a[k] + b[k] + c[k] + d[k]);
}

// fine cell (i, j) += fc - fc0 of its parent (piecewise-constant prolongation)
__global__ void __launch_bounds__(kCavThreads) k_cav_prolong_add(double* __restrict__ fine, int nyf,
                                                                 const double* __restrict__ fc,
                                                                 const double* __restrict__ fc0, int nyc, int K) {
  const int i = blockIdx.x / nyf, j = blockIdx.x - (blockIdx.x / nyf) * nyf;
  const size_t p = ((size_t)(i / 2) * nyc + j / 2) * K;
  double* o = fine + (size_t)blockIdx.x * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) o[k] += fc[p + k] - fc0[p + k];
}

CavWalls walls_of(const bz_cavity* cv) {
  CavWalls wl{};
  for (int s = 0; s < 4; ++s) {
    wl.T[s] = cv->walls[s].T > 0 ? cv->walls[s].T : 1.0;  // y sides of a uniform_y cavity are unused
    wl.U1[s] = cv->walls[s].U[0];
    wl.U2[s] = cv->walls[s].U[1];
  }
  return wl;
}

bz_status alloc_level(bz_ctx* ctx, CavLevel& L, bool own, bool slopes) {
  const size_t K = ctx->K, nc = L.ncell;
  bool ok = hipMalloc((void**)&L.Q, nc * K * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&L.rs, nc * K * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&L.theta, nc * 4 * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&L.nu, nc * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&L.part, (nc + 1) * sizeof(double)) == hipSuccess;
  if (ok && slopes)
    ok = hipMalloc((void**)&L.sx, nc * K * sizeof(double)) == hipSuccess &&
         hipMalloc((void**)&L.sy, nc * K * sizeof(double)) == hipSuccess;
  if (ok && own)
    ok = hipMalloc((void**)&L.f, nc * K * sizeof(double)) == hipSuccess &&
         hipMalloc((void**)&L.b, nc * K * sizeof(double)) == hipSuccess &&
         hipMalloc((void**)&L.f0, nc * K * sizeof(double)) == hipSuccess;
  return ok ? BZ_OK : set_err(ctx, BZ_ENOMEM, "cavity workspace");
}

void free_level(CavLevel& L, bool own) {
  void* ptrs[] = {L.Q, L.rs, L.theta, L.nu, L.part, L.res, own ? L.f : nullptr, L.b, L.f0, L.sx, L.sy, L.T, L.G};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  L = CavLevel{};
}

bz_status cav_slopes(bz_ctx* ctx, bz_cavity* cv, CavLevel& L, hipStream_t st) {
  if (cv->order != 2) return BZ_OK;
  hipLaunchKernelGGL(k_cav_slopes, dim3(L.ncell), dim3(kCavThreads), 0, st, L.f, L.nx, L.ny, ctx->K, cv->limiter,
                     L.sx, L.sy);
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

// collision split of every cell of a level: theta, nu and rs = -P/eps - b, with
// the static reconstruction terms at second order (slopes of the iterate before
// the scan)
bz_status cav_static(bz_ctx* ctx, bz_cavity* cv, CavLevel& L, hipStream_t st) {
  const bool bgk = cv->collision == BZ_COLL_BGK;
  bz_status s0 = cav_slopes(ctx, cv, L, st);
  if (s0 != BZ_OK) return s0;
  if (!bgk) {
    bz_status s = v2_eval_q(ctx, L.f, L.Q, L.ncell, true, true, L.theta, st);
    if (s != BZ_OK) return s;
  }
  hipLaunchKernelGGL(k_cav_static, dim3(L.ncell), dim3(kCavThreads), 0, st, L.f, L.Q, L.theta, L.b, L.sx, L.sy, L.nx,
                     L.ny, cv->uy, L.dx, L.dy, L.rs, L.nu,
                     ctx->d_nodes, ctx->N, ctx->w, cv->eps, bgk ? 1 : 0, cv->bgk_nu, ctx->p.gamma, ctx->nu_gfac);
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

// ||b - R(f)|| of a level (host value; synchronises), the field b - R(f) into res
// when non-null
bz_status cav_residual(bz_ctx* ctx, bz_cavity* cv, CavLevel& L, double* res, double* out, hipStream_t st) {
  const bool bgk = cv->collision == BZ_COLL_BGK;
  bz_status s = bgk ? v2_maxwellian(ctx, L.f, L.theta, nullptr, nullptr, L.ncell, st)
                    : v2_eval_q(ctx, L.f, L.Q, L.ncell, true, true, L.theta, st);
  if (s == BZ_OK) s = cav_slopes(ctx, cv, L, st);
  if (s != BZ_OK) return s;
  hipLaunchKernelGGL(k_cav_resid, dim3(L.ncell), dim3(kCavThreads), 0, st, L.f, L.Q, L.theta, L.nx, L.ny, cv->uy,
                     L.dx, L.dy,
                     cv->eps, walls_of(cv), ctx->d_nodes, ctx->N, ctx->w, bgk ? 1 : 0, cv->bgk_nu, L.b, L.sx, L.sy,
                     res, L.part);
  BZ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_cav_total, dim3(1), dim3(kCavThreads), 0, st, L.part, L.ncell, L.part + L.ncell);
  BZ_HIP(hipGetLastError());
  double tot = 0.0;
  BZ_HIP(hipMemcpyAsync(&tot, L.part + L.ncell, sizeof(double), hipMemcpyDeviceToHost, st));
  BZ_HIP(hipStreamSynchronize(st));
  *out = std::sqrt(L.dx * L.dy * tot);
  return BZ_OK;
}

// transport part of every cell of a level from its current iterate (slopes
// recomputed at second order)
bz_status cav_transport(bz_ctx* ctx, bz_cavity* cv, CavLevel& L, double* T, hipStream_t st) {
  bz_status s = cav_slopes(ctx, cv, L, st);
  if (s != BZ_OK) return s;
  hipLaunchKernelGGL(k_cav_transport, dim3(L.ncell), dim3(kCavThreads), 0, st, L.f, cv->order == 2 ? L.sx : nullptr,
                     cv->order == 2 ? L.sy : nullptr, L.nx, L.ny, cv->uy, L.dx, L.dy, walls_of(cv), ctx->d_nodes,
                     ctx->N, T);
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

// the learned candidates of a scan (after cav_static, which leaves the slopes
// of the iterate and, for binary collisions, its Maxwellian parameters)
bz_status cav_candidates(bz_ctx* ctx, bz_cavity* cv, CavLevel& L, hipStream_t st) {
  const size_t bytes = (size_t)L.ncell * ctx->K * sizeof(double);
  if (!L.T && hipMalloc((void**)&L.T, bytes) != hipSuccess) return set_err(ctx, BZ_ENOMEM, "learned-start field");
  if (!L.G && hipMalloc((void**)&L.G, bytes) != hipSuccess) return set_err(ctx, BZ_ENOMEM, "learned-start field");
  bz_status s;
  if (cv->collision == BZ_COLL_BGK && (s = v2_maxwellian(ctx, L.f, L.theta, nullptr, nullptr, L.ncell, st)) != BZ_OK)
    return s;
  hipLaunchKernelGGL(k_cav_transport, dim3(L.ncell), dim3(kCavThreads), 0, st, L.f, cv->order == 2 ? L.sx : nullptr,
                     cv->order == 2 ? L.sy : nullptr, L.nx, L.ny, cv->uy, L.dx, L.dy, walls_of(cv), ctx->d_nodes,
                     ctx->N, L.T);
  BZ_HIP(hipGetLastError());
  return ws_candidates2(ctx, cv->ws, L.T, L.theta, cv->eps, L.dx, L.G, L.ncell, st);
}

// one SGS iteration of a level (four scans, FAS source b when the level has one), no rescale
bz_status cav_sgs(bz_ctx* ctx, bz_cavity* cv, CavLevel& L, hipStream_t st) {
  static const int scans[4][2] = {{1, 1}, {-1, -1}, {-1, 1}, {1, -1}};
  const CavWalls wl = walls_of(cv);
  // points per thread: 4 up to 32 x 32 velocities, 9 up to 48 x 48
  const auto visit = ctx->K <= 4 * kCavThreads ? k_cav_visit<4> : k_cav_visit<kCavOwn>;
  for (int sc = 0; sc < (cv->uy ? 2 : 4); ++sc) {
    bz_status s = cav_static(ctx, cv, L, st);
    if (s == BZ_OK && cv->ws) s = cav_candidates(ctx, cv, L, st);
    if (s != BZ_OK) return s;
    for (int dd = 0; dd <= L.nx + L.ny - 2; ++dd) {
      const int lo = dd - (L.ny - 1) > 0 ? dd - (L.ny - 1) : 0;
      const int hi = dd < L.nx - 1 ? dd : L.nx - 1;
      hipLaunchKernelGGL(visit, dim3(hi - lo + 1), dim3(kCavThreads), 0, st, L.f, L.rs, L.nu, L.sx, L.sy, L.nx,
                         L.ny, cv->uy, dd,
                         scans[sc][0], scans[sc][1], L.dx, L.dy, cv->eps, wl, ctx->d_nodes, ctx->N, ctx->w,
                         cv->opts.mode, cv->opts.tol, cv->opts.max_iter, cv->opts.fixed_iters,
                         cv->opts.fallback == BZ_FALLBACK_RELAX ? 1 : 0, cv->d_stats,
                         cv->ws ? (const double*)L.G : nullptr);
      BZ_HIP(hipGetLastError());
    }
  }
  return BZ_OK;
}

bz_status cav_rescale(bz_ctx* ctx, bz_cavity* cv, hipStream_t st) {
  CavLevel& L = cv->lv[0];
  hipLaunchKernelGGL(k_cav_cellsum, dim3(L.ncell), dim3(kCavThreads), 0, st, L.f, ctx->K, L.part);
  BZ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_cav_rescale, dim3(L.ncell), dim3(kCavThreads), 0, st, L.f, ctx->K, L.ncell, L.part,
                     L.dx * L.dy * ctx->w, cv->mass);
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

// FAS V-cycle on level l for R(f) = b (eq. coarse); levels halve nx and ny
// until min(nx, ny) <= coarsest
bz_status cav_vcycle(bz_ctx* ctx, bz_cavity* cv, size_t l, const bz_mg_opts& o, hipStream_t st) {
  CavLevel& L = cv->lv[l];
  const int K = ctx->K;
  bz_status s;
  for (int q = 0; q < o.nu1; ++q)
    if ((s = cav_sgs(ctx, cv, L, st)) != BZ_OK) return s;
  double r = 0.0;
  if ((cv->uy ? L.nx : (L.nx < L.ny ? L.nx : L.ny)) <= o.coarsest) {
    double r0 = 0.0;
    if ((s = cav_residual(ctx, cv, L, nullptr, &r0, st)) != BZ_OK) return s;
    for (int q = 0; q < o.coarse_iters; ++q) {
      if ((s = cav_residual(ctx, cv, L, nullptr, &r, st)) != BZ_OK) return s;
      if (r <= 0.1 * r0) break;
      if ((s = cav_sgs(ctx, cv, L, st)) != BZ_OK) return s;
    }
    return BZ_OK;
  }
  if (!L.res && hipMalloc((void**)&L.res, (size_t)L.ncell * K * sizeof(double)) != hipSuccess)
    return set_err(ctx, BZ_ENOMEM, "cavity residual field");
  if ((s = cav_residual(ctx, cv, L, L.res, &r, st)) != BZ_OK) return s;
  if (r < o.tol) return BZ_OK;
  if (l + 1 >= cv->lv.size()) {
    CavLevel C;
    C.nx = L.nx / 2;
    C.ny = cv->uy ? L.ny : L.ny / 2;
    C.ncell = C.nx * C.ny;
    C.dx = 1.0 / C.nx;
    C.dy = 1.0 / C.ny;
    if ((s = alloc_level(ctx, C, true, cv->order == 2)) != BZ_OK) {
      free_level(C, true);
      return s;
    }
    cv->lv.push_back(C);
  }
  CavLevel& Lf = cv->lv[l];  // the vector may have moved
  CavLevel& C = cv->lv[l + 1];
  hipLaunchKernelGGL(k_cav_restrict, dim3(C.ncell), dim3(kCavThreads), 0, st, Lf.f, Lf.ny, C.f0, C.ny, K, cv->uy);
  BZ_HIP(hipGetLastError());
  BZ_HIP(hipMemcpyAsync(C.f, C.f0, (size_t)C.ncell * K * sizeof(double), hipMemcpyDeviceToDevice, st));
  // b_H = R_H(f0) + restrict(b - R_h(f)): the residual field of f0 with no source, negated
  double* bsave = C.b;
  C.b = nullptr;
  double dummy = 0.0;
  s = cav_residual(ctx, cv, C, bsave, &dummy, st);  // bsave <- 0 - R_H(f0)
  C.b = bsave;
  if (s != BZ_OK) return s;
  hipLaunchKernelGGL(k_cav_negate, dim3(C.ncell), dim3(kCavThreads), 0, st, C.b, K);
  BZ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_cav_fas_rhs, dim3(C.ncell), dim3(kCavThreads), 0, st, C.b, C.ny, Lf.res, Lf.ny, K, cv->uy);
  BZ_HIP(hipGetLastError());
  if ((s = cav_vcycle(ctx, cv, l + 1, o, st)) != BZ_OK) return s;
  CavLevel& Lf2 = cv->lv[l];
  CavLevel& C2 = cv->lv[l + 1];
  hipLaunchKernelGGL(k_cav_prolong_add, dim3(Lf2.ncell), dim3(kCavThreads), 0, st, Lf2.f, Lf2.ny, C2.f, C2.f0, C2.ny,
                     K);
  BZ_HIP(hipGetLastError());
  for (int q = 0; q < o.nu2; ++q)
    if ((s = cav_sgs(ctx, cv, cv->lv[l], st)) != BZ_OK) return s;
  return BZ_OK;
}

bz_status read_stats(bz_ctx* ctx, bz_cavity* cv, bz_sweep_stats* stats, int n, hipStream_t st) {
  unsigned long long h[4] = {0, 0, 0, 0};
  BZ_HIP(hipMemcpyAsync(h, cv->d_stats, sizeof(h), hipMemcpyDeviceToHost, st));
  BZ_HIP(hipStreamSynchronize(st));
  if (stats) {
    stats->n_iters = n;
    stats->inner_iters = (int64_t)h[0];
    stats->visits = (int64_t)h[1];
    stats->fallbacks = (int64_t)h[2];
    stats->learned = (int64_t)h[3];
  }
  return BZ_OK;
}

}  // namespace
}  // namespace bz

using bz::set_err;

extern "C" {

bz_status bz_cavity_create(bz_ctx* ctx, const bz_cavity_desc* d, bz_cavity** out) {
  if (!ctx || !out) return BZ_EINVAL;
  *out = nullptr;
  if (ctx->d != 2) return set_err(ctx, BZ_EUNSUPPORTED, "the cavity needs a context with d = 2");
  if (!d || !d->f) return set_err(ctx, BZ_EINVAL, "bad cavity description");
  if (d->nx < 1 || d->ny < 1 || d->nx > 4096 || d->ny > 4096 || (int64_t)d->nx * d->ny > (1 << 24))
    return set_err(ctx, BZ_EINVAL, "nx, ny must be in [1, 4096]");
  if (!(d->eps > 0) || !std::isfinite(d->eps)) return set_err(ctx, BZ_EINVAL, "eps must be > 0");
  if (!(d->mass > 0) || !std::isfinite(d->mass)) return set_err(ctx, BZ_EINVAL, "mass must be > 0");
  if (d->collision != BZ_COLL_BINARY && d->collision != BZ_COLL_BGK)
    return set_err(ctx, BZ_EINVAL, "collision must be BZ_COLL_BINARY or BZ_COLL_BGK");
  if (d->order < 0 || d->order > 2) return set_err(ctx, BZ_EINVAL, "order must be 1 or 2 (0 reads as 1)");
  if (d->uniform_y != 0 && d->ny != 1) return set_err(ctx, BZ_EINVAL, "uniform_y needs ny = 1");
  if (d->limiter != BZ_LIMITER_NONE && d->limiter != BZ_LIMITER_MINMOD) return set_err(ctx, BZ_EINVAL, "bad limiter");
  for (int s = 0; s < (d->uniform_y ? 2 : 4); ++s) {
    const bz_wall& wl = d->walls[s];
    if (!(wl.T > 0) || !std::isfinite(wl.T) || !std::isfinite(wl.U[0]) || !std::isfinite(wl.U[1]))
      return set_err(ctx, BZ_EINVAL, "wall temperature must be > 0 and velocities finite");
    if (wl.U[s / 2] != 0.0) return set_err(ctx, BZ_EINVAL, "wall velocities must be tangential");
  }
  const bz_solve_opts& o = d->inner;
  if (o.mode != BZ_SOLVE_PFP && o.mode != BZ_SOLVE_FP) return set_err(ctx, BZ_EINVAL, "bad solve mode");
  if (o.fixed_iters < 0 || o.fixed_iters > 100000 || (o.fixed_iters == 0 && (o.max_iter < 1 || o.max_iter > 100000)) ||
      !(o.tol >= 0) || !std::isfinite(o.tol) || (o.fallback != BZ_FALLBACK_FP && o.fallback != BZ_FALLBACK_RELAX))
    return set_err(ctx, BZ_EINVAL, "bad inner solve options");
  if (ctx->K > bz::kCavOwn * bz::kCavThreads) return set_err(ctx, BZ_EINVAL, "the cavity needs N <= 48");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  bz_cavity* cv = new bz_cavity();
  cv->ctx = ctx;
  cv->eps = d->eps;
  cv->mass = d->mass;
  for (int s = 0; s < 4; ++s) cv->walls[s] = d->walls[s];
  cv->collision = d->collision;
  cv->bgk_nu = d->bgk_nu;
  cv->opts = o;
  cv->order = d->order == 2 ? 2 : 1;
  cv->uy = d->uniform_y != 0;
  cv->limiter = d->limiter;
  CavLevel L0;
  L0.nx = d->nx;
  L0.ny = d->ny;
  L0.ncell = d->nx * d->ny;
  L0.dx = 1.0 / d->nx;
  L0.dy = 1.0 / d->ny;
  L0.f = d->f;
  bz_status s = bz::alloc_level(ctx, L0, false, cv->order == 2);
  cv->lv.push_back(L0);
  if (s == BZ_OK && hipMalloc((void**)&cv->d_stats, 4 * sizeof(unsigned long long)) != hipSuccess)
    s = set_err(ctx, BZ_ENOMEM, "cavity statistics");
  if (s != BZ_OK) {
    bz_cavity_destroy(cv);
    return s;
  }
  *out = cv;
  return BZ_OK;
}

void bz_cavity_destroy(bz_cavity* cv) {
  if (!cv) return;
  (void)hipDeviceSynchronize();
  for (size_t l = 0; l < cv->lv.size(); ++l) bz::free_level(cv->lv[l], l > 0);
  if (cv->d_stats) (void)hipFree(cv->d_stats);
  delete cv;
}

bz_status bz_cavity_sweep(bz_ctx* ctx, bz_cavity* cv, int n_iters, double* residual_out, bz_sweep_stats* stats,
                          void* stream) {
  if (!ctx || !cv || cv->ctx != ctx) return BZ_EINVAL;
  if (n_iters < 0) return set_err(ctx, BZ_EINVAL, "n_iters < 0");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  BZ_HIP(hipMemsetAsync(cv->d_stats, 0, 4 * sizeof(unsigned long long), st));
  for (int it = 0; it < n_iters; ++it) {
    bz_status s = bz::cav_sgs(ctx, cv, cv->lv[0], st);
    if (s == BZ_OK) s = bz::cav_rescale(ctx, cv, st);
    if (s != BZ_OK) return s;
  }
  if (residual_out) {
    bz_status s = bz::cav_residual(ctx, cv, cv->lv[0], nullptr, residual_out, st);
    if (s != BZ_OK) return s;
  }
  bz_status s = bz::read_stats(ctx, cv, stats, n_iters, st);
  return s != BZ_OK ? s : bz::strict_check(ctx, residual_out, residual_out ? 1 : 0);
}

bz_status bz_cavity_vcycle(bz_ctx* ctx, bz_cavity* cv, const bz_mg_opts* o, int n_cycles, double* residual_out,
                           bz_sweep_stats* stats, void* stream) {
  if (!ctx || !cv || cv->ctx != ctx || !o) return BZ_EINVAL;
  if (n_cycles < 0 || o->coarsest < 1 || o->nu1 < 0 || o->nu2 < 0 || o->coarse_iters < 0 || !(o->tol >= 0))
    return set_err(ctx, BZ_EINVAL, "bad multigrid options");
  if (o->fixed_cycle) return set_err(ctx, BZ_EUNSUPPORTED, "the cavity cycle keeps its residual-based exits");
  {
    int nx = cv->lv[0].nx, ny = cv->lv[0].ny;
    while ((cv->uy ? nx : (nx < ny ? nx : ny)) > o->coarsest) {
      if (nx % 2 || (!cv->uy && ny % 2))
        return set_err(ctx, BZ_EINVAL, "nx and ny must halve evenly down to the coarsest level");
      nx /= 2;
      if (!cv->uy) ny /= 2;
    }
  }
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  BZ_HIP(hipMemsetAsync(cv->d_stats, 0, 4 * sizeof(unsigned long long), st));
  for (int c = 0; c < n_cycles; ++c) {
    bz_status s = bz::cav_vcycle(ctx, cv, 0, *o, st);
    if (s == BZ_OK) s = bz::cav_rescale(ctx, cv, st);
    if (s != BZ_OK) return s;
  }
  if (residual_out) {
    bz_status s = bz::cav_residual(ctx, cv, cv->lv[0], nullptr, residual_out, st);
    if (s != BZ_OK) return s;
  }
  bz_status s = bz::read_stats(ctx, cv, stats, n_cycles, st);
  return s != BZ_OK ? s : bz::strict_check(ctx, residual_out, residual_out ? 1 : 0);
}

bz_status bz_cavity_inflow(bz_ctx* ctx, bz_cavity* cv, double* T_out, void* stream) {
  if (!ctx || !cv || cv->ctx != ctx || !T_out) return BZ_EINVAL;
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  return bz::cav_transport(ctx, cv, cv->lv[0], T_out, (hipStream_t)stream);
}

bz_status bz_cavity_ws_attach(bz_cavity* cv, bz_mlp* mlp) {
  if (!cv) return BZ_EINVAL;
  bz_ctx* ctx = cv->ctx;
  if (!mlp) {
    cv->ws = nullptr;
    return BZ_OK;
  }
  if (bz::ws_ctx(mlp) != ctx) return set_err(ctx, BZ_EINVAL, "the network belongs to another context");
  if (bz::ws_n_in(mlp) != ctx->K + 5 || bz::ws_n_out(mlp) != ctx->K)
    return set_err(ctx, BZ_EINVAL, "the 2D warm-start network must map K + 5 inputs to K outputs");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  bz_status e = bz::ws_prepare(mlp, cv->lv[0].ncell, nullptr);
  if (e != BZ_OK) return e;
  if (hipDeviceSynchronize() != hipSuccess) return set_err(ctx, BZ_EHIP, "hipDeviceSynchronize");
  cv->ws = mlp;
  return BZ_OK;
}

bz_status bz_cavity_residual(bz_ctx* ctx, bz_cavity* cv, double* residual_out, void* stream) {
  if (!ctx || !cv || cv->ctx != ctx || !residual_out) return BZ_EINVAL;
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  bz_status s = bz::cav_residual(ctx, cv, cv->lv[0], nullptr, residual_out, (hipStream_t)stream);
  return s != BZ_OK ? s : bz::strict_check(ctx, residual_out, 1);
}

}  // extern "C"
