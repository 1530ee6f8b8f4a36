// Symmetric Gauss-Seidel scans, outer residual, mass constraint and the FAS
// multigrid V-cycle on 1D slabs (Sections 3.1, 3.3 and 4), upwind finite
// volumes of first order or with the piecewise-linear reconstruction of
// eqs. reconstruction / slope (second order; the slopes are taken from the
// iterate before each scan and enter the static right-hand side).
//
// One scan of eq. SGS on every instance:
//   batched   Q, M[f], nu of every cell from the iterate before the scan
//             (P = Q - nu (M - f) is explicit, eq. Pf), the wall densities from
//             the zero-mass-flux condition (eq. boundary), and the static part
//             of the right-hand side r_j (eq. r): the not-yet-updated neighbour,
//             the ghost terms, -P_j/eps and the FAS source -b_j;
//   sequential one work-group per instance visits its cells in scan order;
//             each visit adds the freshly updated upwind neighbour to r and
//             solves eq. inner_eqn (solve_cell_block).
// After the backward scan every instance is rescaled uniformly to its total
// mass C (eq. mass_conserv).  Readings where the paper is silent: the wall
// density uses the discrete flux balance on the grid; ghost values use the
// latest value of the wall-adjacent cell; the inner solve starts from the
// cell's current value; the mass rescale happens after each SGS iteration on
// the finest level (after each V-cycle under multigrid), never inside coarse
// smoothing; restriction averages two children, prolongation injects the
// coarse correction; the coarsest level is smoothed until its residual falls
// 10x or coarse_iters iterations pass; a V-cycle stops descending once the
// level residual (max over instances) is below tol.
#include <cmath>
#include <vector>

#include "bz_cellsolve.hpp"
#include "bz_common.hpp"
#include "bz_internal.hpp"

namespace bz {

struct InstDev {
  int off;
  int nx;
  double dx;
  double eps;
  double mass;
};

struct WallDev {
  double T[2];
  double U[2][3];  // physical velocities
  int kind[2];     // bz_boundary
  double rho[2];   // inflow densities
};

struct Level {
  int ncell = 0;
  std::vector<InstDev> h_inst;
  InstDev* d_inst = nullptr;
  int* d_cell_inst = nullptr;
  double* f = nullptr;
  bool own_f = false;
  double* b = nullptr;  // FAS right-hand side (nullptr on the finest level)
  double* Q = nullptr;
  double* theta = nullptr;
  double* nu = nullptr;
  double* rs = nullptr;
  double* pre = nullptr;  // [cells][25] static moments of rs and f for the scan (see k_static_rhs)
  double* R = nullptr;  // residual field (transport - Q/eps), multigrid only
  double* fc0 = nullptr;  // restricted fine iterate (coarse levels)
  double* cellsum = nullptr;
  double* ghost = nullptr;  // [n_inst][2] wall densities
  double* S = nullptr;      // [cells][K] slopes of eq. slope (second order only)
  // learned warm start (allocated when a network is attached)
  double* T = nullptr;        // [cells][K] transport part of r, both neighbours old
  double* G = nullptr;        // [cells][K] learned candidates
  double* theta_l = nullptr;  // [cells][5] parameters of M[G]
  int32_t* it_l = nullptr;    // [cells] Newton iterations of M[G] (< 0: failed)
  double* eta0 = nullptr;     // [cells][5] Newton start of the visit's M[g0]
  double* cell_eps = nullptr, *cell_dx = nullptr;  // [cells] per-cell eps and dx
  bool q_valid = false;
};

}  // namespace bz

struct bz_slab {
  bz_ctx* ctx = nullptr;
  int n_inst = 0;
  std::vector<bz_slab_instance> inst;
  int collision = 0;
  double bgk_nu = 0.0;
  int order = 1;  // 1: first-order upwind; 2: linear reconstruction (eq. slope)
  int limiter = 0;  // second order: 0 none, 1 minmod (BZ_LIMITER_MINMOD)
  bz_solve_opts inner{};
  double* wallM = nullptr;    // [n_inst][2][K] unit-density wall Maxwellians
  double* wall_in = nullptr;  // [n_inst][2] incoming discrete flux of the unit wall Maxwellian
  double* bc_fixed = nullptr;  // [n_inst][2] inflow density, or 0 at a diffuse wall
  unsigned long long* d_stats = nullptr;  // inner iterations, visits, fallbacks, learned starts kept
  std::vector<bz::Level> levels;
  bool mg_built = false;
  bz_mlp* ws = nullptr;  // attached warm-start network (borrowed), or NULL
  bz::Slab1V* v1 = nullptr;  // one velocity dimension: the whole slab lives there
  double* f = nullptr;       // the caller's field (borrowed)
};

namespace bz {

// ------------------------------------------------------------------ kernels
template <int N>
__global__ __launch_bounds__(kCellThreads) void k_wall_init(const WallDev* __restrict__ walls, double* __restrict__ wallM,
                                                            double* __restrict__ wall_in, double* __restrict__ bc_fixed,
                                                            const double* __restrict__ nodes, double w, double u0) {
  constexpr int K = N * N * N;
  const int i = blockIdx.x / 2, side = blockIdx.x % 2;
  const WallDev wd = walls[i];
  const double T = wd.T[side];
  const double* U = wd.U[side];
  double* M = wallM + ((size_t)i * 2 + side) * K;
  __shared__ double s_red[kCellThreads / 64];
  double acc[1] = {0.0};
  const double norm = pow(2.0 * kPi * T, -1.5);
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double v0 = nodes[k / (N * N)] + u0, v1 = nodes[(k / N) % N], v2 = nodes[k % N];  // physical
    const double d0 = v0 - U[0], d1 = v1 - U[1], d2 = v2 - U[2];
    const double m = norm * exp(-(d0 * d0 + d1 * d1 + d2 * d2) / (2.0 * T));
    M[k] = m;
    // incoming half-space: v_1 > 0 at the left wall, v_1 < 0 at the right wall
    if (side == 0 ? v0 > 0.0 : v0 < 0.0) acc[0] += fabs(v0) * m;
  }
  block_sum<1>(acc, s_red);
  if (threadIdx.x == 0) {
    wall_in[i * 2 + side] = w * acc[0];
    bc_fixed[i * 2 + side] = wd.kind[side] == BZ_BC_INFLOW ? wd.rho[side] : 0.0;
  }
}

// wall density from the zero-mass-flux balance with the wall-adjacent face
// value: f_0 - s_0 / 2 at the left wall, f_{nx-1} + s_{nx-1} / 2 at the right
// (S = nullptr at first order)
template <int N>
__global__ __launch_bounds__(kCellThreads) void k_ghost_rho(const double* __restrict__ f, const double* __restrict__ S,
                                                            const InstDev* __restrict__ inst,
                                                            const double* __restrict__ wall_in,
                                                            const double* __restrict__ bc_fixed,
                                                            double* __restrict__ ghost, const double* __restrict__ nodes,
                                                            double w, double u0) {
  constexpr int K = N * N * N;
  const int i = blockIdx.x / 2, side = blockIdx.x % 2;
  if (bc_fixed[i * 2 + side] > 0.0) {  // inflow: the given density
    if (threadIdx.x == 0) ghost[i * 2 + side] = bc_fixed[i * 2 + side];
    return;
  }
  const InstDev id = inst[i];
  const size_t cell = (size_t)(id.off + (side == 0 ? 0 : id.nx - 1));
  const double* fc = f + cell * K;
  const double* sc = S ? S + cell * K : fc;
  const double hs = S ? (side == 0 ? -0.5 : 0.5) : 0.0;
  __shared__ double s_red[kCellThreads / 64];
  double acc[1] = {0.0};
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double v0 = nodes[k / (N * N)] + u0;  // physical v_1
    // outgoing half-space of the wall-adjacent cell's face value
    if (side == 0 ? v0 < 0.0 : v0 > 0.0) acc[0] += fabs(v0) * (fc[k] + hs * sc[k]);
  }
  block_sum<1>(acc, s_red);
  if (threadIdx.x == 0) ghost[i * 2 + side] = w * acc[0] / wall_in[i * 2 + side];
}

// eq. slope: centred differences inside, one-sided at the two ends, zero for
// a one-cell instance
template <int N>
__global__ __launch_bounds__(kCellThreads) void k_slopes(const double* __restrict__ f, double* __restrict__ S,
                                                         const InstDev* __restrict__ inst,
                                                         const int* __restrict__ cell_inst, int lim) {
  constexpr int K = N * N * N;
  const int c = blockIdx.x;
  const InstDev id = inst[cell_inst[c]];
  const int j = c - id.off;
  const int jp = j < id.nx - 1 ? j + 1 : j, jm = j > 0 ? j - 1 : j;
  const double wgt = (id.nx < 2) ? 0.0 : (jp - jm == 2 ? 0.5 : 1.0);
  const double* a = f + (size_t)(id.off + jp) * K;
  const double* b = f + (size_t)(id.off + jm) * K;
  double* out = S + (size_t)c * K;
  if (lim && jp - jm == 2) {  // minmod of the one-sided differences inside
    const double* m = f + (size_t)(id.off + j) * K;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
      const double d1 = a[k] - m[k], d0 = m[k] - b[k];
      out[k] = d1 * d0 > 0.0 ? copysign(fmin(fabs(d1), fabs(d0)), d1) : 0.0;
    }
    return;
  }
  for (int k = threadIdx.x; k < K; k += blockDim.x) out[k] = wgt * (a[k] - b[k]);
}

// theta -> (axis factors, e^alpha); returns 4 pi rho of the Gaussian in s_nu
template <int N>
__device__ __forceinline__ void gauss_tables(const double* th, const double* nodes, double w, double (*s_E)[N],
                                             double* s_rho) {
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
    *s_rho = w * exp(th[0]) * s[0] * s[1] * s[2];
  }
  __syncthreads();
}

// static right-hand side of one scan for every cell; also nu of every cell
template <int N>
__global__ __launch_bounds__(kCellThreads) void k_static_rhs(
    const double* __restrict__ f, const double* __restrict__ Q, const double* __restrict__ theta,
    const double* __restrict__ bsrc, double* __restrict__ rs, double* __restrict__ pre, double* __restrict__ nu_out,
    const InstDev* __restrict__ inst, const int* __restrict__ cell_inst, const double* __restrict__ ghost,
    const double* __restrict__ wallM, int forward, int bgk, double bgk_nu, const double* __restrict__ nodes, double w,
    double u0, const double* __restrict__ S, double gam, double gfac) {
  constexpr int K = N * N * N;
  const int c = blockIdx.x;
  const int i = cell_inst[c];
  const InstDev id = inst[i];
  const int j = c - id.off;
  __shared__ double s_E[3][N];
  __shared__ double s_rho;
  gauss_tables<N>(theta + (size_t)c * 5, nodes, w, s_E, &s_rho);
  // BGK model: its own frequency (4 pi rho unless given); binary: the penalty frequency
  const double nu = bgk ? (bgk_nu > 0.0 ? bgk_nu : 4.0 * kPi * s_rho)
                        : penalty_nu(s_rho, theta[(size_t)c * 5 + 4], gam, gfac);
  if (threadIdx.x == 0) nu_out[c] = nu;
  const double ea = exp(theta[(size_t)c * 5]);
  const double ie = 1.0 / id.eps, idx = 1.0 / id.dx;
  const double* fc = f + (size_t)c * K;
  const double* fR = (j < id.nx - 1) ? f + (size_t)(c + 1) * K : nullptr;
  const double* fL = (j > 0) ? f + (size_t)(c - 1) * K : nullptr;
  const double gL = ghost[i * 2], gR = ghost[i * 2 + 1];
  const double* ML = wallM + (size_t)i * 2 * K;
  const double* MR = ML + K;
  double* out = rs + (size_t)c * K;
  const double* bc = bsrc ? bsrc + (size_t)c * K : nullptr;
  // the scan visit needs, besides r = rs + (fresh upwind neighbour term), the
  // moments sum phi {1, 1/D, c/D} rs and sum phi {1, c} f of this cell; they are
  // summed here, in parallel over cells, instead of in the sequential scan
  __shared__ double s_c[N], s_dinv[N];
  __shared__ double s_red[25 * (kCellThreads / 64)];
  if (threadIdx.x < N) {
    const double cc = fabs(nodes[threadIdx.x] + u0) * idx;
    s_c[threadIdx.x] = cc;
    s_dinv[threadIdx.x] = 1.0 / (cc + nu * ie);
  }
  __syncthreads();
  // every source is read unconditionally (a valid pointer with weight 0 when a
  // term is absent), so that the loads of several points are in flight together:
  //   r = -wq (Q - nu (M - f)) - wb b + idx (v- sA A - v+ sB B)
  // forward scan: A = old downstream neighbour (or the right ghost), B = the
  // left ghost on the first cell; backward: B = the upstream neighbour from the
  // forward scan (or the left ghost), A = the right ghost on the last cell
  const double wq = bgk ? 0.0 : ie;
  const double* Qc = bgk ? fc : Q + (size_t)c * K;
  const double wb = bc ? 1.0 : 0.0;
  const double* bp = bc ? bc : fc;
  const double* A;
  const double* B;
  double sA, sB;
  if (forward) {
    A = fR ? fR : MR;
    sA = fR ? 1.0 : gR;
    B = ML;
    sB = (j == 0) ? gL : 0.0;
  } else {
    B = fL ? fL : ML;
    sB = fL ? 1.0 : gL;
    A = MR;
    sA = (j == id.nx - 1) ? gR : 0.0;
  }
  // second order: the reconstruction adds -(v+ s_{j-1} - v_1 s_j + v- s_{j+1}) / (2 dx),
  // with zero ghost slopes (weights 0 and a valid pointer when a slope is absent)
  const double* Sc = S ? S + (size_t)c * K : fc;
  const double* Sl = (S && j > 0) ? Sc - K : Sc;
  const double* Sr = (S && j < id.nx - 1) ? Sc + K : Sc;
  const double hsc = S ? 0.5 * idx : 0.0;
  const double wl = (S && j > 0) ? 1.0 : 0.0, wr = (S && j < id.nx - 1) ? 1.0 : 0.0;
  __shared__ double s_nodes[N];
  if (threadIdx.x < N) s_nodes[threadIdx.x] = nodes[threadIdx.x];
  __syncthreads();
  double acc[25];
#pragma unroll
  for (int q = 0; q < 25; ++q) acc[q] = 0.0;
#pragma unroll 4
  for (int k = threadIdx.x; k < K; k += kCellThreads) {
    const int a0 = k / (N * N), a1 = (k / N) % N, a2 = k % N;
    const double v0 = s_nodes[a0], v1 = s_nodes[a1], v2 = s_nodes[a2];
    const double vp = fmax(v0 + u0, 0.0), vm = fmin(v0 + u0, 0.0);  // physical v_1
    const double M = ea * s_E[0][a0] * s_E[1][a1] * s_E[2][a2];
    const double fk = fc[k];
    const double r = -wq * (Qc[k] - nu * (M - fk)) - wb * bp[k] + idx * (vm * sA * A[k] - vp * sB * B[k]) -
                     hsc * (vp * wl * Sl[k] - (vp + vm) * Sc[k] + vm * wr * Sr[k]);
    out[k] = r;
    const double phi[5] = {1.0, v0, v1, v2, v0 * v0 + v1 * v1 + v2 * v2};
    const double cc = s_c[a0], rd = r * s_dinv[a0];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      acc[q] += phi[q] * r;
      acc[5 + q] += phi[q] * rd;
      acc[10 + q] += phi[q] * cc * rd;
      acc[15 + q] += phi[q] * fk;
      acc[20 + q] += phi[q] * cc * fk;
    }
  }
  block_sum<25>(acc, s_red);
  if (threadIdx.x < 25) pre[(size_t)c * 25 + threadIdx.x] = w * acc[threadIdx.x];
}

template <int N>
struct RChain {
  const double* rs;
  const double* fn;     // freshly updated upwind neighbour (any valid array when idx == 0)
  const double* nodes;  // axis nodes (an LDS table in the scan kernel)
  double idx;           // 1/dx, or 0 for the first cell of the scan (no neighbour term)
  int forward;
  double u0;
  // branch-free, so that a batch of loads can be issued together
  __device__ __forceinline__ double operator()(int k) const {
    const double v0 = nodes[k / (N * N)] + u0;  // physical v_1
    const double coef = forward ? -fmax(v0, 0.0) : fmin(v0, 0.0);
    return rs[k] + coef * idx * fn[k];
  }
};

// Transport part of r for every cell with both neighbours (and the ghosts)
// from the current iterate: idx (v- E - v+ W) - (v+ s_W - v_1 s + v- s_E) / (2 dx),
// W / E the neighbours or the ghosts rho_w M_w, s the slopes (zero in the ghosts).
template <int N>
__global__ __launch_bounds__(kCellThreads) void k_slab_transport(
    const double* __restrict__ f, double* __restrict__ T, const InstDev* __restrict__ inst,
    const int* __restrict__ cell_inst, const double* __restrict__ ghost, const double* __restrict__ wallM,
    const double* __restrict__ nodes, double u0, const double* __restrict__ S) {
  constexpr int K = N * N * N;
  const int c = blockIdx.x;
  const int i = cell_inst[c];
  const InstDev id = inst[i];
  const int j = c - id.off;
  const double idx = 1.0 / id.dx;
  const double* fc = f + (size_t)c * K;
  const double* ML = wallM + (size_t)i * 2 * K;
  const double* Wp = j > 0 ? fc - K : ML;
  const double* Ep = j < id.nx - 1 ? fc + K : ML + K;
  const double sW = j > 0 ? 1.0 : ghost[i * 2], sE = j < id.nx - 1 ? 1.0 : ghost[i * 2 + 1];
  const double* Sc = S ? S + (size_t)c * K : fc;
  const double* Sl = (S && j > 0) ? Sc - K : Sc;
  const double* Sr = (S && j < id.nx - 1) ? Sc + K : Sc;
  const double hsc = S ? 0.5 * idx : 0.0;
  const double wl = (S && j > 0) ? 1.0 : 0.0, wr = (S && j < id.nx - 1) ? 1.0 : 0.0;
  double* out = T + (size_t)c * K;
#pragma unroll 4
  for (int k = threadIdx.x; k < K; k += kCellThreads) {
    const double v0 = nodes[k / (N * N)] + u0;  // physical v_1
    const double vp = fmax(v0, 0.0), vm = fmin(v0, 0.0);
    out[k] = idx * (vm * sE * Ep[k] - vp * sW * Wp[k]) - hsc * (vp * wl * Sl[k] - v0 * Sc[k] + vm * wr * Sr[k]);
  }
}

// Learned warm start: per cell, the inner residual |c g + r_old - lambda (M[g] - g)|
// of f_c and of the candidate G_c, with r_old the visit's right-hand side with the
// upwind neighbour from the iterate before the scan (rs plus that neighbour's
// term).  Where G_c's is smaller, M[G_c] exists and the preconditioned step 1
// from G_c is solvable (eq. existence for r_old), the visit starts from G_c:
// its moment sums replace those of f_c in pre, and eta0 gets M[G_c]'s
// parameters; elsewhere eta0 gets f_c's.
template <int N>
__global__ __launch_bounds__(kCellThreads) void k_ws_select(
    const double* __restrict__ f, const double* __restrict__ rs, const double* __restrict__ G,
    const double* __restrict__ theta, const double* __restrict__ theta_l, const int32_t* __restrict__ it_l,
    const double* __restrict__ nu, double* __restrict__ pre, double* __restrict__ eta0,
    const InstDev* __restrict__ inst, const int* __restrict__ cell_inst, int forward,
    const double* __restrict__ nodes, double w, double u0, unsigned long long* __restrict__ stats) {
  constexpr int K = N * N * N;
  const int c = blockIdx.x;
  const int i = cell_inst[c];
  const InstDev id = inst[i];
  const int j = c - id.off;
  const double idx = 1.0 / id.dx, lam = nu[c] / id.eps;
  const double* fc = f + (size_t)c * K;
  const double* Gc = G + (size_t)c * K;
  const double* rc = rs + (size_t)c * K;
  const bool has_up = forward ? j > 0 : j < id.nx - 1;
  const double* up = has_up ? (forward ? fc - K : fc + K) : fc;  // a valid pointer with weight 0 when absent
  const double wup = has_up ? idx : 0.0;
  __shared__ double s_Ea[3][N], s_Eb[3][N], s_v[N], s_c[N], s_coef[N];
  __shared__ double s_red[22 * (kCellThreads / 64)];
  const double* tha = theta + (size_t)c * 5;
  const double* thb = theta_l + (size_t)c * 5;
  if (threadIdx.x < N) {
    const double x = nodes[threadIdx.x], xp = x + u0;
    s_v[threadIdx.x] = x;
    s_c[threadIdx.x] = fabs(xp) * idx;
    s_coef[threadIdx.x] = forward ? -fmax(xp, 0.0) : fmin(xp, 0.0);
    for (int a = 0; a < 3; ++a) {
      s_Ea[a][threadIdx.x] = exp(tha[1 + a] * x - tha[4] * x * x);
      s_Eb[a][threadIdx.x] = exp(thb[1 + a] * x - thb[4] * x * x);
    }
  }
  __syncthreads();
  const double ea = exp(tha[0]), eb = exp(thb[0]);
  double acc[22];
#pragma unroll
  for (int q = 0; q < 22; ++q) acc[q] = 0.0;
#pragma unroll 4
  for (int k = threadIdx.x; k < K; k += kCellThreads) {
    const int a0 = k / (N * N), a1 = (k / N) % N, a2 = k % N;
    const double cc = s_c[a0];
    const double r = rc[k] + s_coef[a0] * wup * up[k];
    const double fk = fc[k], gk = Gc[k];
    const double Ma = ea * s_Ea[0][a0] * s_Ea[1][a1] * s_Ea[2][a2];
    const double Mb = eb * s_Eb[0][a0] * s_Eb[1][a1] * s_Eb[2][a2];
    const double ra = cc * fk + r - lam * (Ma - fk), rb = cc * gk + r - lam * (Mb - gk);
    acc[0] += ra * ra;
    acc[1] += rb * rb;
    const double v0 = s_v[a0], v1 = s_v[a1], v2 = s_v[a2];
    const double phi[5] = {1.0, v0, v1, v2, v0 * v0 + v1 * v1 + v2 * v2};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      acc[2 + q] += phi[q] * gk;
      acc[7 + q] += phi[q] * cc * gk;
      acc[12 + q] += phi[q] * cc * Mb;
      acc[17 + q] += phi[q] * r;
    }
  }
  block_sum<22>(acc, s_red);
  // step 1 of the preconditioned update from G (eq. step1) must be solvable:
  // s = sum w phi (c (M[G] - G) - r_old) satisfies eq. existence
  double sv[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) sv[q] = w * (acc[12 + q] - acc[7 + q] - acc[17 + q]);
  const bool exists = sv[0] > 0.0 && sv[0] * sv[4] > sv[1] * sv[1] + sv[2] * sv[2] + sv[3] * sv[3];
  // a candidate whose Maxwellian exists, from which step 1 is solvable, and whose
  // residual is the smaller
  const bool take = it_l[c] >= 0 && exists && isfinite(acc[1]) && acc[1] < acc[0];
  if (threadIdx.x < 10 && take) pre[(size_t)c * 25 + 15 + threadIdx.x] = w * acc[2 + threadIdx.x];
  if (threadIdx.x < 5) eta0[(size_t)c * 5 + threadIdx.x] = take ? thb[threadIdx.x] : tha[threadIdx.x];
  if (threadIdx.x == 0 && take) atomicAdd(&stats[3], 1ull);
}

// one work-group per instance: the cells of the scan in order.  A visit takes
// its fixed moments from pre (summed by k_static_rhs) plus the neighbour part
// accumulated by the previous visit's final write, so it touches memory only
// in that final write.
template <int N>
__global__ __launch_bounds__(kChainThreads) void k_chain(double* f, const double* __restrict__ rs,
                                                        const double* __restrict__ pre,
                                                        const double* __restrict__ eta0,
                                                        const double* __restrict__ nu, const InstDev* __restrict__ inst,
                                                        int forward, SolveArgs opt,
                                                        unsigned long long* __restrict__ stats,
                                                        const double* __restrict__ nodes, double w) {
  constexpr int K = N * N * N;
  const InstDev id = inst[blockIdx.x];
  __shared__ double s_nodes[N], s_c[N], s_dinv[N], s_coef[N], s_dinv_next[N];
  const double inv_dx = 1.0 / id.dx;
  unsigned long long it_sum = 0, fb_sum = 0;
  double nb[15];  // neighbour part of this visit's R0, R1, R2
#pragma unroll
  for (int q = 0; q < 15; ++q) nb[q] = 0.0;
  for (int step = 0; step < id.nx; ++step) {
    const int j = forward ? step : id.nx - 1 - step;
    const int c = id.off + j;
    const int jn = forward ? j + 1 : j - 1;
    const bool has_next = jn >= 0 && jn < id.nx;
    const double lam = nu[c] / id.eps;
    __syncthreads();  // the previous visit is done with the tables
    axis_tables<N>(nodes, inv_dx, lam, opt.u0, s_nodes, s_c, s_dinv);
    if (threadIdx.x < N) {
      const double x = nodes[threadIdx.x] + opt.u0;  // physical v_1
      s_coef[threadIdx.x] = forward ? -fmax(x, 0.0) * inv_dx : fmin(x, 0.0) * inv_dx;
      s_dinv_next[threadIdx.x] = has_next ? 1.0 / (fabs(x) * inv_dx + nu[id.off + jn] / id.eps) : 0.0;
    }
    __syncthreads();
    const double* fn = forward ? (j > 0 ? f + (size_t)(c - 1) * K : nullptr)
                               : (j < id.nx - 1 ? f + (size_t)(c + 1) * K : nullptr);
    const double* rsc = rs + (size_t)c * K;
    RChain<N> rf{rsc, fn ? fn : rsc, s_nodes, fn ? inv_dx : 0.0, forward, opt.u0};  // nodes from LDS
    double* fc = f + (size_t)c * K;
    VisitMoments vm;
    double eta[5];
    int nfail = 0;
    if (threadIdx.x < 64) {
      const double* p = pre + (size_t)c * 25;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        vm.R0[q] = p[q] + nb[q];
        vm.R1[q] = p[5 + q] + nb[5 + q];
        vm.R2[q] = p[10 + q] + nb[10 + q];
        vm.mg[q] = p[15 + q];
        vm.cg[q] = p[20 + q];
      }
      if (opt.mode == BZ_SOLVE_SI) {
        // source iteration: eta0[c] holds the parameters of M[f^n_c] from the
        // start of the iteration, which the one plain update takes as is
#pragma unroll
        for (int q = 0; q < 5; ++q) eta[q] = eta0[(size_t)c * 5 + q];
      } else {
        // eta0[c] holds the parameters of M[g0] known before the scan (of f_c,
        // still unchanged, or of the learned start): Newton only confirms them
        nfail = initial_eta<N>(s_nodes, w, vm.mg, inv_dx, lam, eta, eta0 + (size_t)c * 5);
      }
    }
    NextMoments nx{has_next ? s_coef : nullptr, s_dinv_next, {}};
    const SolveOut o = solve_core<N, kChainThreads>(rf, fc, fc, lam, inv_dx, opt, s_nodes, s_c, s_dinv, w, vm, eta,
                                                    nfail, opt.mode != BZ_SOLVE_PFP, 0, &nx);
#pragma unroll
    for (int q = 0; q < 15; ++q) nb[q] = has_next ? nx.out[q] : 0.0;
    it_sum += o.iterations;
    fb_sum += opt.mode == BZ_SOLVE_PFP ? o.fallback : 0;
  }
  if (threadIdx.x == 0) {
    atomicAdd(&stats[0], it_sum);
    atomicAdd(&stats[1], (unsigned long long)id.nx);
    atomicAdd(&stats[2], fb_sum);
  }
}

template <int N>
__global__ __launch_bounds__(kCellThreads) void k_cell_sum(const double* __restrict__ f, double* __restrict__ out) {
  constexpr int K = N * N * N;
  __shared__ double s_red[kCellThreads / 64];
  double acc[1] = {0.0};
  const double* fc = f + (size_t)blockIdx.x * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) acc[0] += fc[k];
  block_sum<1>(acc, s_red);
  if (threadIdx.x == 0) out[blockIdx.x] = acc[0];
}

template <int N>
__global__ __launch_bounds__(kCellThreads) void k_rescale(double* f, const double* __restrict__ cellsum,
                                                          const InstDev* __restrict__ inst,
                                                          const int* __restrict__ cell_inst, double w) {
  constexpr int K = N * N * N;
  const int c = blockIdx.x;
  const InstDev id = inst[cell_inst[c]];
  double tot = 0.0;
  for (int j = 0; j < id.nx; ++j) tot += cellsum[id.off + j];
  const double scale = id.mass / (id.dx * w * tot);
  double* fc = f + (size_t)c * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) fc[k] *= scale;
}

// residual field T = transport(f) - Q/eps; per-cell sum of w (T - b)^2
template <int N>
__global__ __launch_bounds__(kCellThreads) void k_residual(
    const double* __restrict__ f, const double* __restrict__ Q, const double* __restrict__ theta,
    const double* __restrict__ bsrc, double* __restrict__ Rout, double* __restrict__ cellres,
    const InstDev* __restrict__ inst, const int* __restrict__ cell_inst, const double* __restrict__ ghost,
    const double* __restrict__ wallM, int bgk, double bgk_nu, const double* __restrict__ nodes, double w, double u0,
    const double* __restrict__ S) {
  constexpr int K = N * N * N;
  const int c = blockIdx.x;
  const int i = cell_inst[c];
  const InstDev id = inst[i];
  const int j = c - id.off;
  __shared__ double s_E[3][N];
  __shared__ double s_rho;
  __shared__ double s_red[kCellThreads / 64];
  gauss_tables<N>(theta + (size_t)c * 5, nodes, w, s_E, &s_rho);
  const double nu = (bgk_nu > 0.0) ? bgk_nu : 4.0 * kPi * s_rho;
  const double ea = exp(theta[(size_t)c * 5]);
  const double ie = 1.0 / id.eps, idx = 1.0 / id.dx;
  const double* fc = f + (size_t)c * K;
  const double* fR = (j < id.nx - 1) ? fc + K : nullptr;
  const double* fL = (j > 0) ? fc - K : nullptr;
  const double gL = ghost[i * 2], gR = ghost[i * 2 + 1];
  const double* ML = wallM + (size_t)i * 2 * K;
  const double* MR = ML + K;
  // unconditional reads (valid pointers with weights), as in k_static_rhs
  const double* Lp = fL ? fL : ML;
  const double sL = fL ? 1.0 : gL;
  const double* Rp = fR ? fR : MR;
  const double sR = fR ? 1.0 : gR;
  const double* Qc = bgk ? fc : Q + (size_t)c * K;
  const double wq = bgk ? 0.0 : 1.0, wm = bgk ? 1.0 : 0.0;
  const double* bp = bsrc ? bsrc + (size_t)c * K : fc;
  const double wb = bsrc ? 1.0 : 0.0;
  // second order: (v+ (s_j - s_{j-1}) + v- (s_j - s_{j+1})) / (2 dx), zero ghost slopes
  const double* Sc = S ? S + (size_t)c * K : fc;
  const double* Sl = (S && j > 0) ? Sc - K : Sc;
  const double* Sr = (S && j < id.nx - 1) ? Sc + K : Sc;
  const double hsc = S ? 0.5 * idx : 0.0;
  const double wl = (S && j > 0) ? 1.0 : 0.0, wr = (S && j < id.nx - 1) ? 1.0 : 0.0;
  double acc[1] = {0.0};
#pragma unroll 4
  for (int k = threadIdx.x; k < K; k += kCellThreads) {
    const double v0 = nodes[k / (N * N)] + u0;  // physical v_1
    const double vp = fmax(v0, 0.0), vm = fmin(v0, 0.0);
    const double fk = fc[k];
    const double left = sL * Lp[k], right = sR * Rp[k];
    const double M = ea * s_E[0][k / (N * N)] * s_E[1][(k / N) % N] * s_E[2][k % N];
    const double q = wq * Qc[k] + wm * nu * (M - fk);
    const double T = (vp * (fk - left) + vm * (right - fk)) * idx - q * ie -
                     hsc * (vp * wl * Sl[k] - (vp + vm) * Sc[k] + vm * wr * Sr[k]);
    if (Rout) Rout[(size_t)c * K + k] = T;
    const double d = T - wb * bp[k];
    acc[0] += d * d;
  }
  block_sum<1>(acc, s_red);
  if (threadIdx.x == 0) cellres[c] = w * acc[0];
}

// coarse[J] = (a[2J] + a[2J+1]) / 2 - (b ? (b[2J] + b[2J+1]) / 2 : 0), K values per cell
__global__ void k_restrict(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out,
                           int64_t ncoarse, int K) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ncoarse * K) return;
  const int64_t J = g / K, k = g % K;
  const double* a0 = a + (2 * J) * K + k;
  double v = 0.5 * (a0[0] + a0[K]);
  if (b) {
    const double* b0 = b + (2 * J) * K + k;
    v -= 0.5 * (b0[0] + b0[K]);
  }
  out[g] = v;
}

// out = x + sign * y (elementwise)
__global__ void k_axpy(double* out, const double* __restrict__ x, const double* __restrict__ y, double sign, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) out[g] = x[g] + sign * y[g];
}

// f_fine[2J + s] += fc[J] - fc0[J]
__global__ void k_prolong_add(double* f, const double* __restrict__ fc, const double* __restrict__ fc0, int64_t nfine,
                              int K) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nfine * K) return;
  const int64_t jf = g / K, k = g % K;
  const int64_t J = jf / 2;
  f[g] += fc[J * K + k] - fc0[J * K + k];
}

// ------------------------------------------------------------------ host side
#define BZ_SLAB_N(NV, CALL)                                         \
  switch (NV) {                                                     \
    case 8: {                                                       \
      constexpr int NN_ = 8;                                        \
      CALL;                                                         \
    } break;                                                        \
    case 16: {                                                      \
      constexpr int NN_ = 16;                                       \
      CALL;                                                         \
    } break;                                                        \
    case 32: {                                                      \
      constexpr int NN_ = 32;                                       \
      CALL;                                                         \
    } break;                                                        \
    default:                                                        \
      return set_err(ctx, BZ_EUNSUPPORTED, "N must be 8, 16 or 32"); \
  }

static bz_status level_alloc(bz_ctx* ctx, Level& L, int n_inst, bool with_mg, bool with_slopes) {
  const size_t K = ctx->K;
  BZ_HIP(hipMalloc((void**)&L.d_inst, sizeof(InstDev) * L.h_inst.size()));
  BZ_HIP(hipMemcpy(L.d_inst, L.h_inst.data(), sizeof(InstDev) * L.h_inst.size(), hipMemcpyHostToDevice));
  std::vector<int> ci(L.ncell);
  for (size_t i = 0; i < L.h_inst.size(); ++i)
    for (int j = 0; j < L.h_inst[i].nx; ++j) ci[L.h_inst[i].off + j] = (int)i;
  BZ_HIP(hipMalloc((void**)&L.d_cell_inst, sizeof(int) * L.ncell));
  BZ_HIP(hipMemcpy(L.d_cell_inst, ci.data(), sizeof(int) * L.ncell, hipMemcpyHostToDevice));
  BZ_HIP(hipMalloc((void**)&L.Q, sizeof(double) * K * L.ncell));
  BZ_HIP(hipMalloc((void**)&L.rs, sizeof(double) * K * L.ncell));
  BZ_HIP(hipMalloc((void**)&L.pre, sizeof(double) * 25 * L.ncell));
  BZ_HIP(hipMalloc((void**)&L.theta, sizeof(double) * 5 * L.ncell));
  BZ_HIP(hipMalloc((void**)&L.nu, sizeof(double) * L.ncell));
  BZ_HIP(hipMalloc((void**)&L.cellsum, sizeof(double) * L.ncell));
  BZ_HIP(hipMalloc((void**)&L.ghost, sizeof(double) * 2 * n_inst));
  if (with_mg) BZ_HIP(hipMalloc((void**)&L.R, sizeof(double) * K * L.ncell));
  if (with_slopes) BZ_HIP(hipMalloc((void**)&L.S, sizeof(double) * K * L.ncell));
  std::vector<double> ce(L.ncell), cd(L.ncell);
  for (const InstDev& in : L.h_inst)
    for (int j = 0; j < in.nx; ++j) {
      ce[in.off + j] = in.eps;
      cd[in.off + j] = in.dx;
    }
  BZ_HIP(hipMalloc((void**)&L.cell_eps, sizeof(double) * L.ncell));
  BZ_HIP(hipMalloc((void**)&L.cell_dx, sizeof(double) * L.ncell));
  BZ_HIP(hipMemcpy(L.cell_eps, ce.data(), sizeof(double) * L.ncell, hipMemcpyHostToDevice));
  BZ_HIP(hipMemcpy(L.cell_dx, cd.data(), sizeof(double) * L.ncell, hipMemcpyHostToDevice));
  return BZ_OK;
}

// buffers of the learned warm start on one level (once)
static bz_status ws_alloc(bz_ctx* ctx, Level& L) {
  if (L.G) return BZ_OK;
  const size_t K = ctx->K;
  BZ_HIP(hipMalloc((void**)&L.T, sizeof(double) * K * L.ncell));
  BZ_HIP(hipMalloc((void**)&L.G, sizeof(double) * K * L.ncell));
  BZ_HIP(hipMalloc((void**)&L.theta_l, sizeof(double) * 5 * L.ncell));
  BZ_HIP(hipMalloc((void**)&L.it_l, sizeof(int32_t) * L.ncell));
  BZ_HIP(hipMalloc((void**)&L.eta0, sizeof(double) * 5 * L.ncell));
  return BZ_OK;
}

static void level_free(Level& L) {
  void* ptrs[] = {L.d_inst, L.d_cell_inst, L.Q, L.rs, L.pre, L.theta, L.nu, L.cellsum, L.ghost, L.R, L.b, L.fc0, L.S,
                  L.T, L.G, L.theta_l, L.it_l, L.eta0, L.cell_eps, L.cell_dx};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (L.own_f && L.f) (void)hipFree(L.f);
  L = Level();
}

static bz_status collide(bz_ctx* ctx, bz_slab* s, Level& L, hipStream_t st) {
  if (L.q_valid) return BZ_OK;
  bz_status e;
  if (s->collision != BZ_COLL_BGK) {
    e = eval_q(ctx, L.f, L.Q, L.ncell, true, L.theta, st);
    if (e == BZ_OK)
      e = s->collision == BZ_COLL_BINARY_CONSERVE ? conserve_project(ctx, L.Q, L.theta, L.ncell, st)
                                                  : mass_project(ctx, L.Q, L.theta, L.ncell, st);
  } else {
    e = maxwellian(ctx, L.f, L.theta, nullptr, nullptr, L.ncell, st);
  }
  if (e == BZ_OK) L.q_valid = true;
  return e;
}

// slopes of the current iterate (second order), then the wall densities
static bz_status ghosts(bz_ctx* ctx, bz_slab* s, Level& L, hipStream_t st) {
  if (s->order == 2)
    BZ_SLAB_N(ctx->N, hipLaunchKernelGGL((k_slopes<NN_>), dim3(L.ncell), dim3(kCellThreads), 0, st, L.f, L.S,
                                         L.d_inst, L.d_cell_inst, s->limiter));
  BZ_SLAB_N(ctx->N, hipLaunchKernelGGL((k_ghost_rho<NN_>), dim3(2 * s->n_inst), dim3(kCellThreads), 0, st, L.f,
                                       s->order == 2 ? L.S : nullptr, L.d_inst, s->wall_in, s->bc_fixed, L.ghost,
                                       ctx->d_nodes, ctx->w, ctx->p.v1_shift));
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

// One scan.  With the source iteration the Maxwellian parameters and nu of the
// iterate before the forward scan stay in force for the backward scan
// (L.q_valid is kept), and each visit makes one plain update from them.
static bz_status scan(bz_ctx* ctx, bz_slab* s, Level& L, bool forward, hipStream_t st) {
  const bool si = s->inner.mode == BZ_SOLVE_SI;
  bz_status e = collide(ctx, s, L, st);
  if (e != BZ_OK) return e;
  if ((e = ghosts(ctx, s, L, st)) != BZ_OK) return e;
  const int bgk = s->collision == BZ_COLL_BGK;
  BZ_SLAB_N(ctx->N, hipLaunchKernelGGL((k_static_rhs<NN_>), dim3(L.ncell), dim3(kCellThreads), 0, st, L.f, L.Q,
                                       L.theta, L.b, L.rs, L.pre, L.nu, L.d_inst, L.d_cell_inst, L.ghost, s->wallM,
                                       forward ? 1 : 0, bgk, s->bgk_nu, ctx->d_nodes, ctx->w, ctx->p.v1_shift,
                                       s->order == 2 ? L.S : nullptr, ctx->p.gamma, ctx->nu_gfac));
  if (s->ws) {
    // learned candidates from the iterate before the scan, then the choice per cell
    BZ_SLAB_N(ctx->N, hipLaunchKernelGGL((k_slab_transport<NN_>), dim3(L.ncell), dim3(kCellThreads), 0, st, L.f, L.T,
                                         L.d_inst, L.d_cell_inst, L.ghost, s->wallM, ctx->d_nodes, ctx->p.v1_shift,
                                         s->order == 2 ? L.S : nullptr));
    if ((e = ws_candidates(ctx, s->ws, L.T, L.theta, L.cell_eps, L.cell_dx, L.G, L.ncell, st)) != BZ_OK) return e;
    if ((e = maxwellian(ctx, L.G, L.theta_l, nullptr, L.it_l, L.ncell, st)) != BZ_OK) return e;
    BZ_SLAB_N(ctx->N, hipLaunchKernelGGL((k_ws_select<NN_>), dim3(L.ncell), dim3(kCellThreads), 0, st, L.f, L.rs, L.G,
                                         L.theta, L.theta_l, L.it_l, L.nu, L.pre, L.eta0, L.d_inst, L.d_cell_inst,
                                         forward ? 1 : 0, ctx->d_nodes, ctx->w, ctx->p.v1_shift, s->d_stats));
  }
  SolveArgs a{s->inner.mode, s->inner.tol, s->inner.max_iter, si ? 1 : s->inner.fixed_iters, ctx->p.v1_shift,
              s->inner.fallback == BZ_FALLBACK_RELAX ? 1 : 0};
  BZ_SLAB_N(ctx->N, hipLaunchKernelGGL((k_chain<NN_>), dim3(s->n_inst), dim3(kChainThreads), 0, st, L.f, L.rs, L.pre,
                                       s->ws ? L.eta0 : L.theta, L.nu,
                                       L.d_inst, forward ? 1 : 0, a, s->d_stats, ctx->d_nodes, ctx->w));
  BZ_HIP(hipGetLastError());
  L.q_valid = si && forward;
  return BZ_OK;
}

static bz_status rescale(bz_ctx* ctx, bz_slab* s, Level& L, hipStream_t st) {
  (void)s;
  BZ_SLAB_N(ctx->N, hipLaunchKernelGGL((k_cell_sum<NN_>), dim3(L.ncell), dim3(kCellThreads), 0, st, L.f, L.cellsum));
  BZ_SLAB_N(ctx->N, hipLaunchKernelGGL((k_rescale<NN_>), dim3(L.ncell), dim3(kCellThreads), 0, st, L.f, L.cellsum,
                                       L.d_inst, L.d_cell_inst, ctx->w));
  BZ_HIP(hipGetLastError());
  L.q_valid = false;
  return BZ_OK;
}

static bz_status sgs_iter(bz_ctx* ctx, bz_slab* s, Level& L, bool do_rescale, hipStream_t st) {
  bz_status e;
  if ((e = scan(ctx, s, L, true, st)) != BZ_OK) return e;
  if ((e = scan(ctx, s, L, false, st)) != BZ_OK) return e;
  if (do_rescale) return rescale(ctx, s, L, st);
  return BZ_OK;
}

// per-cell squared residual sums |T - b|^2 into L.cellsum (device work only);
// optionally keeps the field T in L.R
static bz_status residual_launch(bz_ctx* ctx, bz_slab* s, Level& L, bool keep_field, hipStream_t st) {
  bz_status e = collide(ctx, s, L, st);
  if (e != BZ_OK) return e;
  if ((e = ghosts(ctx, s, L, st)) != BZ_OK) return e;
  const int bgk = s->collision == BZ_COLL_BGK;
  BZ_SLAB_N(ctx->N, hipLaunchKernelGGL((k_residual<NN_>), dim3(L.ncell), dim3(kCellThreads), 0, st, L.f, L.Q,
                                       L.theta, L.b, keep_field ? L.R : nullptr, L.cellsum, L.d_inst, L.d_cell_inst,
                                       L.ghost, s->wallM, bgk, bgk ? s->bgk_nu : 0.0, ctx->d_nodes, ctx->w,
                                       ctx->p.v1_shift, s->order == 2 ? L.S : nullptr));
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

// per-instance norms from L.cellsum (one host synchronisation)
static bz_status residual_read(bz_ctx* ctx, Level& L, std::vector<double>& out, hipStream_t st) {
  std::vector<double> cs(L.ncell);
  BZ_HIP(hipMemcpyAsync(cs.data(), L.cellsum, sizeof(double) * L.ncell, hipMemcpyDeviceToHost, st));
  BZ_HIP(hipStreamSynchronize(st));
  out.assign(L.h_inst.size(), 0.0);
  for (size_t i = 0; i < L.h_inst.size(); ++i) {
    double t = 0.0;
    for (int j = 0; j < L.h_inst[i].nx; ++j) t += cs[L.h_inst[i].off + j];
    out[i] = std::sqrt(L.h_inst[i].dx * t);
  }
  return BZ_OK;
}

// per-instance residual norms |T - b| (host vector); optionally keeps the field T in L.R
static bz_status residual(bz_ctx* ctx, bz_slab* s, Level& L, bool keep_field, std::vector<double>& out,
                          hipStream_t st) {
  bz_status e = residual_launch(ctx, s, L, keep_field, st);
  if (e != BZ_OK) return e;
  return residual_read(ctx, L, out, st);
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

static double vmax(const std::vector<double>& v) {
  double m = 0.0;
  for (double x : v) m = std::fmax(m, x);
  return m;
}

static bz_status build_mg(bz_ctx* ctx, bz_slab* s, int coarsest) {
  if (s->mg_built) return BZ_OK;
  const int nx = s->inst[0].nx;
  for (const auto& in : s->inst)
    if (in.nx != nx) return set_err(ctx, BZ_EINVAL, "multigrid needs equal cell counts in every instance");
  int n = nx;
  while (n > coarsest && n % 2 == 0) n /= 2;
  if (n != coarsest) return set_err(ctx, BZ_EINVAL, "cell count must be coarsest * 2^k");
  const size_t K = ctx->K;
  // the finest level gets a residual field
  BZ_HIP(hipMalloc((void**)&s->levels[0].R, sizeof(double) * K * s->levels[0].ncell));
  int lev_nx = nx / 2;
  while (lev_nx >= coarsest) {
    Level L;
    const Level& F = s->levels.back();
    L.ncell = F.ncell / 2;
    for (const InstDev& fi : F.h_inst) L.h_inst.push_back(InstDev{fi.off / 2, fi.nx / 2, fi.dx * 2.0, fi.eps, fi.mass});
    bz_status e = level_alloc(ctx, L, s->n_inst, true, s->order == 2);
    if (e == BZ_OK && s->ws) e = ws_alloc(ctx, L);
    if (e != BZ_OK) return e;
    BZ_HIP(hipMalloc((void**)&L.f, sizeof(double) * K * L.ncell));
    L.own_f = true;
    BZ_HIP(hipMalloc((void**)&L.b, sizeof(double) * K * L.ncell));
    BZ_HIP(hipMalloc((void**)&L.fc0, sizeof(double) * K * L.ncell));
    s->levels.push_back(L);
    if (lev_nx == coarsest) break;
    lev_nx /= 2;
  }
  s->mg_built = true;
  return BZ_OK;
}

// One FAS V-cycle from level l.  With o->fixed_cycle the cycle reads nothing
// back: every level descends and the coarsest runs coarse_iters iterations.
static bz_status vcycle(bz_ctx* ctx, bz_slab* s, size_t l, const bz_mg_opts* o, hipStream_t st) {
  Level& L = s->levels[l];
  bz_status e;
  std::vector<double> rn;
  const bool fixed = o->fixed_cycle != 0;
  for (int i = 0; i < o->nu1; ++i)
    if ((e = sgs_iter(ctx, s, L, false, st)) != BZ_OK) return e;
  if (l + 1 == s->levels.size()) {
    if (fixed) {
      for (int it = 0; it < o->coarse_iters; ++it)
        if ((e = sgs_iter(ctx, s, L, false, st)) != BZ_OK) return e;
      return BZ_OK;
    }
    if ((e = residual(ctx, s, L, false, rn, st)) != BZ_OK) return e;
    const double r0 = vmax(rn);
    for (int it = 0; it < o->coarse_iters; ++it) {
      if (it > 0) {
        if ((e = residual(ctx, s, L, false, rn, st)) != BZ_OK) return e;
      }
      if (vmax(rn) <= 0.1 * r0) break;
      if ((e = sgs_iter(ctx, s, L, false, st)) != BZ_OK) return e;
    }
    return BZ_OK;
  }
  if (fixed) {
    if ((e = residual_launch(ctx, s, L, true, st)) != BZ_OK) return e;  // L.R = R_h(f)
  } else {
    if ((e = residual(ctx, s, L, true, rn, st)) != BZ_OK) return e;  // L.R = R_h(f)
    if (vmax(rn) < o->tol) return BZ_OK;
  }
  Level& C = s->levels[l + 1];
  const size_t K = ctx->K;
  const unsigned gc = (unsigned)(((int64_t)C.ncell * K + 255) / 256);
  // f_H = I f_h ; fc0 = f_H ; res_h = b_h - R_h(f_h) (b_h = 0 on the finest level)
  hipLaunchKernelGGL(k_restrict, dim3(gc), dim3(256), 0, st, L.f, (const double*)nullptr, C.f, (int64_t)C.ncell, (int)K);
  hipLaunchKernelGGL(k_axpy, dim3(gc), dim3(256), 0, st, C.fc0, (const double*)C.f, (const double*)C.f, 0.0,
                     (int64_t)C.ncell * K);
  C.q_valid = false;
  // b_H = R_H(f_H) + I (b_h - R_h(f_h)): first R_H(f_H) into C.R (C.b not yet used)
  double* saved_b = C.b;
  C.b = nullptr;
  e = residual_launch(ctx, s, C, true, st);
  C.b = saved_b;
  if (e != BZ_OK) return e;
  // C.b = I(b_h - R_h) computed as I(b_h) - I(R_h), then += R_H(f_H)
  if (L.b)
    hipLaunchKernelGGL(k_restrict, dim3(gc), dim3(256), 0, st, L.b, L.R, C.b, (int64_t)C.ncell, (int)K);
  else {
    hipLaunchKernelGGL(k_restrict, dim3(gc), dim3(256), 0, st, L.R, (const double*)nullptr, C.b, (int64_t)C.ncell,
                       (int)K);
    hipLaunchKernelGGL(k_axpy, dim3(gc), dim3(256), 0, st, C.b, (const double*)C.R, (const double*)C.b, -1.0,
                       (int64_t)C.ncell * K);
  }
  if (L.b) hipLaunchKernelGGL(k_axpy, dim3(gc), dim3(256), 0, st, C.b, (const double*)C.b, (const double*)C.R, 1.0,
                              (int64_t)C.ncell * K);
  BZ_HIP(hipGetLastError());
  if ((e = vcycle(ctx, s, l + 1, o, st)) != BZ_OK) return e;
  const unsigned gf = (unsigned)(((int64_t)L.ncell * K + 255) / 256);
  hipLaunchKernelGGL(k_prolong_add, dim3(gf), dim3(256), 0, st, L.f, (const double*)C.f, (const double*)C.fc0,
                     (int64_t)L.ncell, (int)K);
  BZ_HIP(hipGetLastError());
  L.q_valid = false;
  for (int i = 0; i < o->nu2; ++i)
    if ((e = sgs_iter(ctx, s, L, false, st)) != BZ_OK) return e;
  return BZ_OK;
}

static bz_status read_stats(bz_ctx* ctx, bz_slab* s, bz_sweep_stats* stats, int n_iters, hipStream_t st) {
  unsigned long long h[4] = {0, 0, 0, 0};
  BZ_HIP(hipMemcpyAsync(h, s->d_stats, sizeof(h), hipMemcpyDeviceToHost, st));
  BZ_HIP(hipStreamSynchronize(st));
  if (stats) {
    stats->n_iters = n_iters;
    stats->inner_iters = (int64_t)h[0];
    stats->visits = (int64_t)h[1];
    stats->fallbacks = (int64_t)h[2];
    stats->learned = (int64_t)h[3];
  }
  return BZ_OK;
}

}  // namespace bz

using bz::set_err;

extern "C" {

bz_status bz_slab_create(bz_ctx* ctx, const bz_slab_desc* d, bz_slab** out) {
  if (!ctx || !out) return BZ_EINVAL;
  *out = nullptr;
  if (ctx->d == 2) return set_err(ctx, BZ_EUNSUPPORTED, "the 1D slab needs d = 1 or 3 (use the bz_cavity_* calls)");
  if (!d || d->n_instances < 1 || !d->instances || !d->f) return set_err(ctx, BZ_EINVAL, "bad slab description");
  if (d->order < 0 || d->order > 2) return set_err(ctx, BZ_EINVAL, "order must be 1 or 2 (0 reads as 1)");
  if (d->limiter != BZ_LIMITER_NONE && d->limiter != BZ_LIMITER_MINMOD) return set_err(ctx, BZ_EINVAL, "bad limiter");
  if (d->collision != BZ_COLL_BINARY && d->collision != BZ_COLL_BGK && d->collision != BZ_COLL_BINARY_CONSERVE)
    return set_err(ctx, BZ_EINVAL, "bad collision");
  const bz_solve_opts& o = d->inner;
  if (o.mode != BZ_SOLVE_PFP && o.mode != BZ_SOLVE_FP && o.mode != BZ_SOLVE_SI)
    return set_err(ctx, BZ_EINVAL, "bad inner mode");
  if (o.mode == BZ_SOLVE_SI && d->collision != BZ_COLL_BGK)
    return set_err(ctx, BZ_EINVAL, "the source iteration needs BGK collisions");
  if (o.fallback != BZ_FALLBACK_FP && o.fallback != BZ_FALLBACK_RELAX) return set_err(ctx, BZ_EINVAL, "bad fallback");
  if (o.mode != BZ_SOLVE_SI &&
      (o.fixed_iters < 0 || (o.fixed_iters == 0 && (o.max_iter < 1 || o.max_iter > 100000)) || !(o.tol >= 0)))
    return set_err(ctx, BZ_EINVAL, "bad inner options");
  if (ctx->d == 1) {
    for (int i = 0; i < d->n_instances; ++i) {
      const bz_slab_instance& in = d->instances[i];
      if (in.nx < 1 || !(in.xR > in.xL) || !(in.eps > 0) || !(in.T_L > 0) || !(in.T_R > 0) || !(in.mass > 0))
        return set_err(ctx, BZ_EINVAL, "bad slab instance");
    }
    if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
    bz::Slab1V* v1 = nullptr;
    bz_status e = bz::slab1v_create(ctx, d, &v1);
    if (e != BZ_OK) return e;
    bz_slab* s = new bz_slab();
    s->ctx = ctx;
    s->n_inst = d->n_instances;
    s->inst.assign(d->instances, d->instances + d->n_instances);
    s->collision = d->collision;
    s->inner = o;
    s->v1 = v1;
    s->f = d->f;
    *out = s;
    return BZ_OK;
  }
  int off = 0;
  std::vector<bz::InstDev> hi;
  std::vector<bz::WallDev> walls;
  for (int i = 0; i < d->n_instances; ++i) {
    const bz_slab_instance& in = d->instances[i];
    if (in.nx < 1 || !(in.xR > in.xL) || !(in.eps > 0) || !(in.T_L > 0) || !(in.T_R > 0) || !(in.mass > 0))
      return set_err(ctx, BZ_EINVAL, "bad slab instance");
    if ((in.bc_L != BZ_BC_WALL && in.bc_L != BZ_BC_INFLOW) || (in.bc_R != BZ_BC_WALL && in.bc_R != BZ_BC_INFLOW))
      return set_err(ctx, BZ_EINVAL, "bad boundary kind");
    if ((in.bc_L == BZ_BC_WALL && in.U_L[0] != 0.0) || (in.bc_R == BZ_BC_WALL && in.U_R[0] != 0.0))
      return set_err(ctx, BZ_EINVAL, "wall velocity must be tangential");
    if ((in.bc_L == BZ_BC_INFLOW && !(in.rho_L > 0)) || (in.bc_R == BZ_BC_INFLOW && !(in.rho_R > 0)))
      return set_err(ctx, BZ_EINVAL, "inflow density must be > 0");
    hi.push_back(bz::InstDev{off, in.nx, (in.xR - in.xL) / in.nx, in.eps, in.mass});
    bz::WallDev wd{};
    wd.T[0] = in.T_L;
    wd.T[1] = in.T_R;
    for (int a = 0; a < 3; ++a) {
      wd.U[0][a] = in.U_L[a];
      wd.U[1][a] = in.U_R[a];
    }
    wd.kind[0] = in.bc_L;
    wd.kind[1] = in.bc_R;
    wd.rho[0] = in.rho_L;
    wd.rho[1] = in.rho_R;
    walls.push_back(wd);
    off += in.nx;
  }
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  bz_slab* s = new bz_slab();
  s->ctx = ctx;
  s->n_inst = d->n_instances;
  s->inst.assign(d->instances, d->instances + d->n_instances);
  s->collision = d->collision;
  s->bgk_nu = d->bgk_nu;
  s->order = d->order == 0 ? 1 : d->order;
  s->limiter = d->limiter;
  s->inner = d->inner;
  bz::Level L0;
  L0.ncell = off;
  L0.h_inst = hi;
  L0.f = d->f;
  bz_status e = bz::level_alloc(ctx, L0, s->n_inst, false, s->order == 2);
  s->levels.push_back(L0);
  auto fail = [&](bz_status st) {
    bz_slab_destroy(s);
    return st;
  };
  if (e != BZ_OK) return fail(e);
  const size_t K = ctx->K;
  bz::WallDev* d_walls = nullptr;
  if (hipMalloc((void**)&s->wallM, sizeof(double) * 2 * K * s->n_inst) != hipSuccess ||
      hipMalloc((void**)&s->wall_in, sizeof(double) * 2 * s->n_inst) != hipSuccess ||
      hipMalloc((void**)&s->bc_fixed, sizeof(double) * 2 * s->n_inst) != hipSuccess ||
      hipMalloc((void**)&s->d_stats, sizeof(unsigned long long) * 4) != hipSuccess ||
      hipMalloc((void**)&d_walls, sizeof(bz::WallDev) * s->n_inst) != hipSuccess)
    return fail(set_err(ctx, BZ_ENOMEM, "slab allocation"));
  if (hipMemcpy(d_walls, walls.data(), sizeof(bz::WallDev) * s->n_inst, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(s->d_stats, 0, sizeof(unsigned long long) * 4) != hipSuccess)
    return fail(set_err(ctx, BZ_EHIP, "slab upload"));
  switch (ctx->N) {
    case 8: hipLaunchKernelGGL((bz::k_wall_init<8>), dim3(2 * s->n_inst), dim3(bz::kCellThreads), 0, 0, d_walls, s->wallM, s->wall_in, s->bc_fixed, ctx->d_nodes, ctx->w, ctx->p.v1_shift); break;
    case 16: hipLaunchKernelGGL((bz::k_wall_init<16>), dim3(2 * s->n_inst), dim3(bz::kCellThreads), 0, 0, d_walls, s->wallM, s->wall_in, s->bc_fixed, ctx->d_nodes, ctx->w, ctx->p.v1_shift); break;
    case 32: hipLaunchKernelGGL((bz::k_wall_init<32>), dim3(2 * s->n_inst), dim3(bz::kCellThreads), 0, 0, d_walls, s->wallM, s->wall_in, s->bc_fixed, ctx->d_nodes, ctx->w, ctx->p.v1_shift); break;
  }
  if (hipDeviceSynchronize() != hipSuccess) return fail(set_err(ctx, BZ_EHIP, "wall init"));
  (void)hipFree(d_walls);
  *out = s;
  return BZ_OK;
}

void bz_slab_destroy(bz_slab* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  if (s->v1) bz::slab1v_destroy(s->v1);
  for (auto& L : s->levels) bz::level_free(L);
  if (s->wallM) (void)hipFree(s->wallM);
  if (s->wall_in) (void)hipFree(s->wall_in);
  if (s->bc_fixed) (void)hipFree(s->bc_fixed);
  if (s->d_stats) (void)hipFree(s->d_stats);
  delete s;
}

bz_status bz_sgs_sweep(bz_ctx* ctx, bz_slab* s, int n_iters, double* residual_out, bz_sweep_stats* stats,
                       void* stream) {
  if (!ctx || !s || s->ctx != ctx) return BZ_EINVAL;
  if (n_iters < 0) return set_err(ctx, BZ_EINVAL, "n_iters < 0");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (s->v1) {
    bz_status e = bz::slab1v_run(ctx, s->v1, s->f, 0, n_iters, nullptr, residual_out, stats, st);
    return e != BZ_OK ? e : bz::strict_check(ctx, residual_out, s->n_inst);
  }
  if (hipMemsetAsync(s->d_stats, 0, sizeof(unsigned long long) * 4, st) != hipSuccess)
    return set_err(ctx, BZ_EHIP, "stats reset");
  bz::Level& L = s->levels[0];
  L.q_valid = false;  // the caller may have changed f
  for (int it = 0; it < n_iters; ++it) {
    bz_status e = bz::sgs_iter(ctx, s, L, true, st);
    if (e != BZ_OK) return e;
  }
  if (residual_out) {
    std::vector<double> rn;
    bz_status e = bz::residual(ctx, s, L, false, rn, st);
    if (e != BZ_OK) return e;
    for (int i = 0; i < s->n_inst; ++i) residual_out[i] = rn[i];
  }
  bz_status e = bz::read_stats(ctx, s, stats, n_iters, st);
  return e != BZ_OK ? e : bz::strict_check(ctx, residual_out, s->n_inst);
}

bz_status bz_slab_inflow(bz_ctx* ctx, bz_slab* s, double* out, void* stream) {
  if (!ctx || !s || s->ctx != ctx || !out) return BZ_EINVAL;
  if (s->v1) return set_err(ctx, BZ_EUNSUPPORTED, "one velocity dimension: no learned start");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  bz::Level& L = s->levels[0];
  bz_status e = bz::ghosts(ctx, s, L, st);
  if (e != BZ_OK) return e;
  BZ_SLAB_N(ctx->N, hipLaunchKernelGGL((bz::k_slab_transport<NN_>), dim3(L.ncell), dim3(bz::kCellThreads), 0, st, L.f,
                                       out, L.d_inst, L.d_cell_inst, L.ghost, s->wallM, ctx->d_nodes, ctx->p.v1_shift,
                                       s->order == 2 ? L.S : nullptr));
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

bz_status bz_ws_attach(bz_slab* s, bz_mlp* mlp) {
  if (!s) return BZ_EINVAL;
  bz_ctx* ctx = s->ctx;
  if (!mlp) {
    s->ws = nullptr;
    return BZ_OK;
  }
  if (s->v1) return set_err(ctx, BZ_EUNSUPPORTED, "one velocity dimension: no learned start");
  if (s->inner.mode == BZ_SOLVE_SI)
    return set_err(ctx, BZ_EUNSUPPORTED, "the source iteration has no inner iteration to start");
  if (bz::ws_ctx(mlp) != ctx) return set_err(ctx, BZ_EINVAL, "the network belongs to another context");
  if (bz::ws_n_in(mlp) != ctx->K + 6 || bz::ws_n_out(mlp) != ctx->K)
    return set_err(ctx, BZ_EINVAL, "the warm-start network must map K + 6 inputs to K outputs");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  for (auto& L : s->levels) {
    bz_status e = bz::ws_alloc(ctx, L);
    if (e != BZ_OK) return e;
  }
  bz_status e = bz::ws_prepare(mlp, s->levels[0].ncell, nullptr);
  if (e != BZ_OK) return e;
  if (hipDeviceSynchronize() != hipSuccess) return set_err(ctx, BZ_EHIP, "hipDeviceSynchronize");
  s->ws = mlp;
  return BZ_OK;
}

bz_status bz_outer_residual(bz_ctx* ctx, bz_slab* s, double* residual_out, void* stream) {
  if (!ctx || !s || s->ctx != ctx || !residual_out) return BZ_EINVAL;
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  if (s->v1) {
    bz_status e = bz::slab1v_run(ctx, s->v1, s->f, 2, 0, nullptr, residual_out, nullptr, (hipStream_t)stream);
    return e != BZ_OK ? e : bz::strict_check(ctx, residual_out, s->n_inst);
  }
  bz::Level& L = s->levels[0];
  L.q_valid = false;
  std::vector<double> rn;
  bz_status e = bz::residual(ctx, s, L, false, rn, (hipStream_t)stream);
  if (e != BZ_OK) return e;
  for (int i = 0; i < s->n_inst; ++i) residual_out[i] = rn[i];
  return bz::strict_check(ctx, residual_out, s->n_inst);
}

bz_status bz_multigrid_vcycle(bz_ctx* ctx, bz_slab* s, const bz_mg_opts* o, int n_cycles, double* residual_out,
                              bz_sweep_stats* stats, void* stream) {
  if (!ctx || !s || s->ctx != ctx || !o) return BZ_EINVAL;
  if (n_cycles < 0 || o->coarsest < 1 || o->nu1 < 0 || o->nu2 < 0 || o->coarse_iters < 0 || !(o->tol >= 0))
    return set_err(ctx, BZ_EINVAL, "bad multigrid options");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (s->v1) {
    bz_status e1 = bz::slab1v_run(ctx, s->v1, s->f, 1, n_cycles, o, residual_out, stats, st);
    return e1 != BZ_OK ? e1 : bz::strict_check(ctx, residual_out, s->n_inst);
  }
  bz_status e = bz::build_mg(ctx, s, o->coarsest);
  if (e != BZ_OK) return e;
  if (hipMemsetAsync(s->d_stats, 0, sizeof(unsigned long long) * 4, st) != hipSuccess)
    return set_err(ctx, BZ_EHIP, "stats reset");
  bz::Level& L = s->levels[0];
  L.q_valid = false;
  for (int c = 0; c < n_cycles; ++c) {
    if ((e = bz::vcycle(ctx, s, 0, o, st)) != BZ_OK) return e;
    if ((e = bz::rescale(ctx, s, L, st)) != BZ_OK) return e;
  }
  if (residual_out) {
    std::vector<double> rn;
    if ((e = bz::residual(ctx, s, L, false, rn, st)) != BZ_OK) return e;
    for (int i = 0; i < s->n_inst; ++i) residual_out[i] = rn[i];
  }
  e = bz::read_stats(ctx, s, stats, n_cycles, st);
  return e != BZ_OK ? e : bz::strict_check(ctx, residual_out, s->n_inst);
}

}  // extern "C"

/* ------------------------------------------------------------ graph replay */
struct bz_graph {
  bz_ctx* ctx = nullptr;
  bz_slab* slab = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int iters = 0;
  bool with_residual = false;
};

namespace {

// Records body(stream) (plus a stats reset and, optionally, the outer
// residual) into a graph; segments is what the statistics count per replay.
template <typename Body>
bz_status capture_graph(bz_ctx* ctx, bz_slab* s, int segments, int with_residual, void* stream, bz_graph** out,
                        Body body) {
  hipStream_t st = (hipStream_t)stream;
  bz::Level& L = s->levels[0];
  // everything that allocates or sets attributes happens before the capture
  if (s->collision != BZ_COLL_BGK) {
    bz_status e = bz::eval_q_prepare(ctx, L.ncell, true);
    if (e != BZ_OK) return e;
  }
  if (hipStreamSynchronize(st) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipStreamSynchronize");
  const bool prof = ctx->prof;
  ctx->prof = false;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    ctx->prof = prof;
    return set_err(ctx, BZ_EHIP, "hipStreamBeginCapture");
  }
  for (auto& lv : s->levels) lv.q_valid = false;
  hipLaunchKernelGGL(bz::k_zero_u64, dim3(1), dim3(64), 0, st, s->d_stats, 4);  // a kernel, not a memset node
  bz_status e = body(st);
  if (e == BZ_OK && with_residual) e = bz::residual_launch(ctx, s, L, false, st);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(st, &g);
  ctx->prof = prof;
  for (auto& lv : s->levels) lv.q_valid = false;
  if (e != BZ_OK || ce != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return e != BZ_OK ? e : set_err(ctx, BZ_EHIP, "hipStreamEndCapture");
  }
  bz_graph* gr = new bz_graph();
  gr->ctx = ctx;
  gr->slab = s;
  gr->graph = g;
  gr->iters = segments;
  gr->with_residual = with_residual != 0;
  if (hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    bz_graph_destroy(gr);
    return set_err(ctx, BZ_EHIP, "hipGraphInstantiate");
  }
  *out = gr;
  return BZ_OK;
}

bz_status capture_checks(bz_ctx* ctx, bz_slab* s, int n, void* stream, bz_graph** out) {
  if (!out) return BZ_EINVAL;
  *out = nullptr;
  if (!ctx || !s || s->ctx != ctx) return BZ_EINVAL;
  if (n < 1) return set_err(ctx, BZ_EINVAL, "at least one iteration or cycle per replay");
  if (!stream) return set_err(ctx, BZ_EINVAL, "capture needs a non-default stream");
  if (s->ws) return set_err(ctx, BZ_EUNSUPPORTED, "a slab with a warm-start network attached is not captured");
  if (s->v1)
    return set_err(ctx, BZ_EUNSUPPORTED, "one velocity dimension: a call already runs whole iterations in one launch");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  return BZ_OK;
}

}  // namespace

extern "C" {

bz_status bz_graph_capture_sweeps(bz_ctx* ctx, bz_slab* s, int iters_per_replay, int with_residual, void* stream,
                                  bz_graph** out) {
  bz_status e = capture_checks(ctx, s, iters_per_replay, stream, out);
  if (e != BZ_OK) return e;
  bz::Level& L = s->levels[0];
  return capture_graph(ctx, s, iters_per_replay, with_residual, stream, out, [&](hipStream_t st) {
    bz_status r = BZ_OK;
    for (int it = 0; it < iters_per_replay && r == BZ_OK; ++it) r = bz::sgs_iter(ctx, s, L, true, st);
    return r;
  });
}

bz_status bz_graph_capture_vcycles(bz_ctx* ctx, bz_slab* s, const bz_mg_opts* opts, int cycles_per_replay,
                                   int with_residual, void* stream, bz_graph** out) {
  bz_status e = capture_checks(ctx, s, cycles_per_replay, stream, out);
  if (e != BZ_OK) return e;
  if (!opts || opts->coarsest < 1 || opts->nu1 < 0 || opts->nu2 < 0 || opts->coarse_iters < 0)
    return set_err(ctx, BZ_EINVAL, "bad multigrid options");
  if ((e = bz::build_mg(ctx, s, opts->coarsest)) != BZ_OK) return e;
  bz_mg_opts o = *opts;
  o.fixed_cycle = 1;
  bz::Level& L = s->levels[0];
  return capture_graph(ctx, s, cycles_per_replay, with_residual, stream, out, [&](hipStream_t st) {
    bz_status r = BZ_OK;
    for (int c = 0; c < cycles_per_replay && r == BZ_OK; ++c) {
      r = bz::vcycle(ctx, s, 0, &o, st);
      if (r == BZ_OK) r = bz::rescale(ctx, s, L, st);
    }
    return r;
  });
}

bz_status bz_graph_launch(bz_graph* g, double* residual_out, bz_sweep_stats* stats, void* stream) {
  if (!g || !g->exec) return BZ_EINVAL;
  bz_ctx* ctx = g->ctx;
  if (residual_out && !g->with_residual) return set_err(ctx, BZ_EINVAL, "graph captured without the residual");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (hipGraphLaunch(g->exec, st) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipGraphLaunch");
  bz::Level& L = g->slab->levels[0];
  L.q_valid = false;
  if (residual_out) {
    std::vector<double> rn;
    bz_status e = bz::residual_read(ctx, L, rn, st);
    if (e != BZ_OK) return e;
    for (int i = 0; i < g->slab->n_inst; ++i) residual_out[i] = rn[i];
  }
  return bz::read_stats(ctx, g->slab, stats, g->iters, st);
}

void bz_graph_destroy(bz_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"
