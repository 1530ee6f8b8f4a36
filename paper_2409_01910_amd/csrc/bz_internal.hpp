// Internal declarations of the bz library: context, tables, workspace and
// the launchers each translation unit provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bz.h"

struct bz_ctx {
  bz_params p{};
  int N = 0, K = 0;
  int n_theta = 0, n_phi = 0, n_rho = 0, n_pairs = 0;
  double dv = 0, w = 0, R = 0, Rg = 0;
  double nu_gfac = 1.0;  // 4^{gamma/2} Gamma((3 + gamma)/2) / Gamma(3/2), for the penalty frequency
  int d = 3;             // velocity dimension (1, 2 or 3)
  bool strict = false;   // bz_set_strict
  std::string err;

  // host copies of the tables (FP64)
  std::vector<double> h_nodes;  // [N] axis node coordinates
  std::vector<double> h_pair_w; // [n_pairs] weight of one direction of each antipodal pair

  // device tables (FP64 masters; FP32 copies where the FP32 path reads them)
  double* d_nodes = nullptr;   // [N]
  double* d_ph1 = nullptr;     // [n_rho][n_theta][N] complex: exp(i xi_l rho c_t / 2)
  double* d_ph23 = nullptr;    // [n_rho][n_pairs][2][N] complex: exp(i xi_l s_2), exp(i xi_l s_3)
  double* d_pairw = nullptr;   // [n_pairs]
  double* d_pairsw = nullptr;  // [n_pairs] sqrt of d_pairw
  double* d_W = nullptr;       // [n_rho][K] gain radial weights / K
  double* d_Gm = nullptr;      // [K] loss weight
  // Carleman form (BZ_METHOD_CARLEMAN): n_dir half-sphere directions
  int n_dir = 0;
  double* d_cw = nullptr;      // [n_dir][2][K] A_p, B_p on the spectrum grid
  double* d_cbeta = nullptr;   // [K] loss weight sum_p A_p B_p
  // two-dimensional velocity (d = 2): N x N grid, M = n_phi circle directions
  int v2_npass = 0;             // radix passes of one length-N transform
  int v2_rad[4] = {0, 0, 0, 0};  // their radices (4, 3 or 2)
  double* d_v2tw = nullptr;     // [N] complex exp(2 pi i j / N)
  double* d_v2xi = nullptr;     // [N] xi_l = pi l / L, l in transform order
  double* d_v2dir = nullptr;    // [n_phi / 2][2] sigma_p of the antipodal pairs
  double* d_v2rho = nullptr;    // [n_rho] radial nodes
  double* d_v2ph = nullptr;     // [n_rho][n_phi / 2][2][N] (cos, sin)(xi_l rho_r sigma_p,a / 2)
  float* d_ph1_f = nullptr;
  float* d_ph23_f = nullptr;
  float* d_pairw_f = nullptr;
  float* d_pairsw_f = nullptr;
  float* d_W_f = nullptr;
  float* d_Gm_f = nullptr;
  float* d_cw_f = nullptr;
  float* d_cbeta_f = nullptr;

  // profiling of the direction-pair kernel (events recorded around launches)
  bool prof = false;
  std::vector<hipEvent_t> prof_ev;  // start/stop pairs
  size_t prof_used = 0;             // events used
  double prof_flops = 0.0;

  // launch plan of the collision pipeline (bz_plan; 0 = default): waves per
  // block of the N = 32 direction-pair kernel (8), the cells of a chunk (as
  // many as the 8 GiB workspace budget holds) and the radial nodes whose
  // accumulated planes are held for one column pass (all); set by bz_tune
  // (measured and cached per discretisation) or bz_set_plan
  int pair_waves = 0;
  int chunk_cap = 0;
  int acc_nodes = 0;

  // workspace (grown on demand, never shrunk until destroy)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // device address of the static scratch array of the allocation-free entry
  // point on this context's device (resolved at create)
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
};

namespace bz {

bz_status set_err(bz_ctx* c, bz_status s, const std::string& msg);
bz_status hip_err(bz_ctx* c, hipError_t e, const char* what);
bz_status ensure_ws(bz_ctx* c, size_t bytes);
// record the start (stop = false) or stop event of a profiled launch
bz_status prof_mark(bz_ctx* c, hipStream_t st, bool stop, double flops);

#define BZ_HIP(call)                                         \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return bz::hip_err(ctx, e_, #call); \
  } while (0)

// host tables (bz_tables.cpp)
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
bz_status build_tables(bz_ctx* ctx);
void free_tables(bz_ctx* ctx);

// collision pipeline (bz_q.hip).  Writes Q (FP64).  When rho_out / theta_out are
// non-null (corrected mode), the discrete Maxwellian parameters and density of
// each cell are returned too.
// With ws_ext non-null the pipeline runs in that caller-provided workspace of
// ws_ext_bytes (chunks sized to it; BZ_EINVAL if one cell does not fit) and
// allocates nothing.
bz_status eval_q(bz_ctx* ctx, const double* f, double* Q, int64_t batch, bool corrected, double* theta_out,
                 hipStream_t st, void* ws_ext = nullptr, size_t ws_ext_bytes = 0);
size_t eval_q_ws_per_cell(const bz_ctx* ctx, bool corrected);
// sizes the workspace and sets kernel attributes for eval_q on `batch` cells,
// so that a later eval_q makes no allocation (needed under stream capture)
bz_status eval_q_prepare(bz_ctx* ctx, int64_t batch, bool corrected);

// two-dimensional velocity (bz_v2.hip, tables in bz_tables.cpp)
bz_status build_tables_v2(bz_ctx* ctx);
bz_status v2_maxwellian(bz_ctx* ctx, const double* f, double* theta, double* M, int32_t* iters, int64_t batch,
                        hipStream_t st);
// Q (FP64) of each cell; corrected: Q_s(f - M, f + M) with M from theta (computed
// here, written to theta_out [batch][4] when non-null); mass: the projection of
// mass_project on the corrected form
// ws_ext as for eval_q: the [batch][4] parameters of the corrected form go there
// when theta_out is NULL (BZ_EINVAL if they do not fit)
bz_status v2_eval_q(bz_ctx* ctx, const double* f, double* Q, int64_t batch, bool corrected, bool mass,
                    double* theta_out, hipStream_t st, void* ws_ext = nullptr, size_t ws_ext_bytes = 0);
// allocation-free collision evaluation (bz_noalloc.hip): resolves, once per
// device, the device address of the library's static scratch array
bz_status scratch_attach(bz_ctx* ctx);
// the tuned launch plan cached for this context's discretisation, if any (bz_tune.cpp)
void apply_cached_plan(bz_ctx* ctx);
// argument checks shared by bz_eval_Q and bz_eval_Q_noalloc (bz_api.cpp)
bz_status check_eval_q_args(bz_ctx* ctx, const double* f, const double* Q, int64_t batch, uint32_t flags,
                            const double* theta);

// cell kernels (bz_cell.hip)
bz_status maxwellian(bz_ctx* ctx, const double* f, double* theta, double* M, int32_t* iters, int64_t batch,
                     hipStream_t st);
bz_status cell_solve(bz_ctx* ctx, const double* r, const double* nu, const double* eps, double dx, const double* g0,
                     double* g, int64_t batch, const bz_solve_opts* opts, bz_cell_stats* stats, hipStream_t st,
                     const double* g0b = nullptr, const double* dxs = nullptr);
// learned initial guesses g0 [batch][K] (bz_mlp.hip)
bz_status learned_guess(bz_ctx* ctx, bz_mlp* mp, const double* inflow_r, const double* theta, const double* eps,
                        double dx, double* g0, int64_t batch, hipStream_t st);
// learned warm start inside the scans (bz_mlp.hip): candidates
// G = M_theta + scale MLP(features) of a batch with per-cell eps and dx (BF16
// inference), and the sizing of the network's scratch and BF16 weights
bz_status ws_candidates(bz_ctx* ctx, bz_mlp* mp, const double* inflow, const double* theta, const double* eps,
                        const double* dxs, double* G, int64_t batch, hipStream_t st);
bz_status ws_candidates2(bz_ctx* ctx, bz_mlp* mp, const double* inflow, const double* theta, double eps, double dx,
                         double* G, int64_t batch, hipStream_t st);
bz_status ws_prepare(bz_mlp* mp, int64_t batch, hipStream_t st);

// the slab with one velocity dimension (csrc/bz_slab1v.hip); op 0: SGS
// iterations, 1: V-cycles, 2: residual only
struct Slab1V;
bz_status slab1v_create(bz_ctx* ctx, const bz_slab_desc* d, Slab1V** out);
void slab1v_destroy(Slab1V* s);
bz_status slab1v_run(bz_ctx* ctx, Slab1V* s, double* f, int op, int n, const bz_mg_opts* mg, double* residual_out,
                     bz_sweep_stats* stats, hipStream_t st);
bz_ctx* ws_ctx(bz_mlp* mp);
int ws_n_in(bz_mlp* mp);
int ws_n_out(bz_mlp* mp);
// Q <- Q - M_theta sum(Q) / sum(M_theta) per cell (mass-conserving projection)
bz_status mass_project(bz_ctx* ctx, double* Q, const double* theta, int64_t batch, hipStream_t st);
// Q <- Q - M_theta (a . phi): mass, momentum and energy conserved per cell
bz_status conserve_project(bz_ctx* ctx, double* Q, const double* theta, int64_t batch, hipStream_t st);
// r = inflow - (Q - nu (M_theta - f)) / eps, nu = 4 pi rho(theta); writes nu
bz_status penalty_rhs(bz_ctx* ctx, const double* f, const double* Q, const double* theta, const double* inflow,
                      const double* eps, double* r, double* nu, int64_t batch, hipStream_t st,
                      const double* nu_in = nullptr);
// strict mode: BZ_ENUMERIC when one of the n returned values is not finite
bz_status strict_check(bz_ctx* ctx, const double* vals, int64_t n);

}  // namespace bz
