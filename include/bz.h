/*
 * bz.h - C ABI of the MI355X (gfx950) steady-state Boltzmann hot path.
 *
 * Method: Cai, Dong, Hu, "Symmetric Gauss-Seidel Method with a Preconditioned
 * Fixed-Point Iteration for the Steady-State Boltzmann Equation".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Velocity grid (Section 2.2): d = 3, N points per axis, nodes k*dv with
 *    k = -N/2+1 .. N/2 and dv = 2L/N, periodic box [-L, L)^3, equal weights
 *    w = dv^3.  A distribution of one cell is K = N^3 doubles in C order
 *    [i1][i2][i3]; velocity axis i1 is v_1, the transport direction.
 *  - Field buffers are caller-owned DEVICE pointers (hipMalloc / torch), FP64,
 *    contiguous: a batch of B cells is [B][K].  The library never frees or
 *    reallocates caller memory.  The context owns its tables and workspace.
 *  - All work is asynchronous and stream-ordered on `stream` (a hipStream_t,
 *    NULL = the default stream).  Results are valid once the stream is
 *    synchronised.  A context is not thread-safe: one context per host thread.
 *  - Argument and shape errors are detected synchronously and returned as a
 *    bz_status; nothing is launched then.  No C++ exception crosses the ABI.
 *    bz_last_error() gives the message of the last failure on a context.
 *  - Numerical events (existence test failed and the fixed-point fallback was
 *    taken, Newton not converged, non-finite values) never fail a call; they
 *    are reported per cell in device-side statistics.
 */
#ifndef BZ_H
#define BZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BZ_OK = 0,
  BZ_EINVAL = 1,       /* bad argument or shape */
  BZ_ENOMEM = 2,       /* device allocation of workspace failed */
  BZ_EHIP = 3,         /* a HIP runtime call failed */
  BZ_EUNSUPPORTED = 4, /* valid request this build does not implement */
  BZ_ENUMERIC = 5      /* strict mode (bz_set_strict): the call finished and filled its
                          outputs, but a result it returns is not finite */
} bz_status;

typedef enum { BZ_FP64 = 0, BZ_FP32 = 1, BZ_FP32_DIFF = 2 } bz_precision;

typedef struct bz_ctx bz_ctx;

/* Discretisation of one velocity cell.
 *   N        points per axis: 8, 16 or 32
 *   L        half-width of the periodic velocity box (> 0)
 *   gamma    VHS exponent of B = |v - v_*|^gamma (0: Maxwell molecules, B = 1;
 *            1: hard spheres), Section 4.2 and eq. collision
 *   n_theta  Gauss-Legendre nodes in cos(theta) of the sphere rule (even >= 2)
 *   n_phi    uniform azimuth nodes (even >= 2); M = n_theta * n_phi directions
 *   n_rho    Gauss-Legendre nodes of the radial rule for |g| in [0, 2R]
 *   R        support radius; <= 0 selects L = (3 sqrt 2 + 1) R / 2 (Section 4.2)
 *   precision  arithmetic of the spectral stage (FFTs, shifted products and
 *            their accumulation).  Moments, Newton solves, the steady-state
 *            correction, the cell solve and residuals are always FP64.
 *            BZ_FP64 evaluates the corrected form (eq. discrete_Q) of the 3D
 *            sigma form as the difference Q[f,f] - Q[M,M] (one field through
 *            the direction pairs, the Maxwellian's gain from separable FP64 1D
 *            transforms); BZ_FP32, and the 2D and Carleman forms in either
 *            precision, as the symmetric bilinear form Q_s(f - M, f + M) (two
 *            fields through the pairs, f - M scaled by a power of two to the
 *            magnitude of f + M), whose FP32 rounding error scales with
 *            |f - M|, so it stays small against Q near equilibrium;
 *            BZ_FP32_DIFF as the difference with an FP32 stage (d = 3, sigma
 *            form): half the pair work of BZ_FP32, but its rounding error
 *            scales with the loss term Q^- itself, so near equilibrium it
 *            bounds the residual an FP32 stage can reach.
 *   device   HIP device ordinal the context works on.
 *   v1_shift physical v_1 of the grid origin: the nodes sample v' = v - v1_shift e_1.
 *            Fields, moments, Maxwellian parameters (theta) and the collision
 *            operator (translation invariant) are all in v'; transport uses the
 *            physical v_1 = v'_1 + v1_shift (c = |v_1|/dx, upwind split, wall
 *            fluxes).  0 for a grid centred on rest.
 *   method   evaluation of the Fourier spectral operator:
 *            BZ_METHOD_SIGMA: the sigma form described at bz_eval_Q (any gamma).
 *            BZ_METHOD_CARLEMAN: the fast form for kernels that separate in the
 *            Carleman representation (Section 2.2 cites this family of fast
 *            spectral methods); here hard spheres in 3D, gamma = 1, whose
 *            Carleman kernel is the constant 4.  x and y are truncated to the
 *            ball of radius Rc = sqrt(2) R, the truncation that the cited fast
 *            spectral construction keeps free of aliasing when
 *            L = (3 sqrt 2 + 1) R / 2 (Section 4.2).  The spectral weight then
 *            separates per direction e of the half sphere into
 *            psi1(xi.e) Phi2(|P_e xi|),
 *              psi1(s) = 2 int_0^{Rc} rho cos(rho s) drho,
 *              Phi2(t) = 2 pi Rc J1(Rc t) / t,
 *            P_e the projection perpendicular to e.  The M/2 directions of the
 *            sphere rule with cos(theta) > 0 give the gain
 *              Q+ = sum_p IDFT(A_p fh) IDFT(B_p fh),
 *              A_p = 4 w_p psi1(xi.e_p),  B_p = Phi2(|P_{e_p} xi|),
 *            and the loss f IDFT(beta fh) with beta = sum_p A_p B_p, so the
 *            plain form conserves mass exactly.  n_rho is not used.  A context
 *            with this method and gamma != 1 is refused (BZ_EUNSUPPORTED).
 *            With d = 2 the method is the Carleman form of Maxwell molecules
 *            (gamma = 0; other gamma are refused): the weight is the constant
 *            2, x runs over the half circle (the circle rule's M/2 nodes with
 *            p < M/2, weights 2 pi / M) and y along e_perp, both truncated at
 *            Rc = sqrt(2) R, psi2(s) = 2 Rc sinc(Rc s), and
 *              Q+ = sum_p IDFT(A_p fh) IDFT(B_p fh),
 *              A_p = 2 w_p psi2(xi.e_p),  B_p = psi2(xi.e_p_perp),
 *            with the loss f IDFT(beta fh), beta = sum_p A_p B_p.
 *   d        velocity dimension: 3 (or 0, the default) or 2.  Section 4.2 runs
 *            its binary-collision examples with two-dimensional velocities.
 *            With d = 2 the grid is N x N (N in {8, 12, 16, 24, 32, 48}, point
 *            k = i_1 N + i_2), fields are [batch][N^2], moments and Maxwellian
 *            parameters have 4 entries (1, v_1, v_2, |v|^2), and the sigma
 *            form runs over the circle: M = n_phi directions
 *            theta_p = 2 pi p / n_phi with weights 2 pi / n_phi (n_theta is not
 *            used), S_2(z) = 2 pi J0(z) in place of 4 pi sin(z)/z, radial
 *            measure rho^{gamma+1}.  d = 2 supports BZ_FP64 and BZ_FP32 (the
 *            transform stage; the rest stays FP64), BZ_METHOD_SIGMA and
 *            BZ_METHOD_CARLEMAN (gamma = 0),
 *            v1_shift = 0, and the calls bz_eval_Q (flags BZ_Q_CORRECTED and
 *            BZ_Q_MASS), bz_maxwellian and the bz_cavity_* scans; the other calls
 *            return BZ_EUNSUPPORTED on such a context.
 *            With d = 1 the grid is N nodes (N even, 2 <= N <= 64) and the
 *            context serves the BGK slab of Section 4.1's 1D1V model only
 *            (bz_slab_create with BZ_COLL_BGK and diffuse walls at rest, modes
 *            PFP, FP and SI, first or second order; bz_sgs_sweep,
 *            bz_multigrid_vcycle, bz_outer_residual): BZ_FP64, BZ_METHOD_SIGMA,
 *            v1_shift = 0; the collision rule sizes are not used.  Moments and
 *            Maxwellian parameters have 3 entries (1, v, v^2), the BGK
 *            frequency is |S^0| rho = 2 rho unless bgk_nu is given, and one
 *            wave runs each instance's whole call (iterations or V-cycles) in
 *            one launch, with the V-cycle's exits decided per instance.  Graph
 *            capture, the learned start and the other calls return
 *            BZ_EUNSUPPORTED. */
typedef enum { BZ_METHOD_SIGMA = 0, BZ_METHOD_CARLEMAN = 1 } bz_method;

typedef struct {
  int N;
  double L;
  double gamma;
  int n_theta;
  int n_phi;
  int n_rho;
  double R;
  int precision;
  int device;
  double v1_shift;
  int method;
  int d;
} bz_params;

/* Create / destroy a context: host-built quadrature, phase and weight tables
 * are uploaded to the device.  Returns BZ_EINVAL for unsupported N or rule
 * sizes, BZ_EHIP / BZ_ENOMEM on runtime failures.  *out is NULL on error. */
bz_status bz_create(const bz_params* p, bz_ctx** out);
void bz_destroy(bz_ctx* ctx);

const char* bz_status_str(bz_status s);
/* Copies the last error message of ctx (NUL-terminated, truncated to n). */
bz_status bz_last_error(bz_ctx* ctx, char* buf, size_t n);
/* Workspace bytes the context currently holds on the device. */
size_t bz_workspace_bytes(bz_ctx* ctx);

/* ---------------------------------------------------------------- collision
 * bz_eval_Q: collision term of `batch` independent cells.
 *   f  [batch][K] FP64 device, read only;  Q  [batch][K] FP64 device, written.
 *   flags & BZ_Q_CORRECTED: the steady-state preserving form of eq. discrete_Q,
 *       Q = Q^FSM[f,f] - Q^FSM[M[f], M[f]], with M[f] the discrete Maxwellian of
 *       eqs. discrete_conservation / discrete_Gaussian.  It is evaluated as
 *       the symmetric bilinear form Q_s(f - M, f + M), which is equal up to
 *       rounding and avoids cancellation.
 *   otherwise Q = Q^FSM[f,f]: the Fourier spectral operator (Section 2.2,
 *       eq. collision truncated to |v - v_*| <= 2R on the periodic box) with an
 *       M-direction sphere rule and an n_rho-node radial rule.
 *   flags & BZ_Q_MASS (with BZ_Q_CORRECTED): afterwards Q <- Q - M[f] s, with
 *       s = sum_k Q_k / sum_k M[f]_k, so that sum_k w Q_k = 0 to rounding.  The
 *       sigma quadrature of the gain term conserves mass only approximately;
 *       with diffuse walls the steady problem is solvable only if the summed
 *       collision term vanishes, so the slab solver and bz_cell_fixed_point
 *       use this form by default.  Allocates a [batch][5] stream-ordered
 *       temporary when theta is NULL.
 *   flags & BZ_Q_CONSERVE (with BZ_Q_CORRECTED, not with BZ_Q_MASS): afterwards
 *       Q <- Q - M[f] (a . phi), phi = (1, v, |v|^2), with a from the 5x5 system
 *       sum_k phi_i M phi_j a_j = sum_k phi_i Q_k, so that mass, momentum and
 *       energy are conserved to rounding (the least change in sum dQ^2 / M).
 *       The spectral operator conserves momentum and energy only up to its
 *       truncation error; problems with inflow at both ends of a slab need all
 *       five invariants balanced (BZ_COLL_BINARY_CONSERVE).
 *   theta (nullable, BZ_Q_CORRECTED only) receives [batch][5] parameters
 *       (alpha, beta_1..3, gamma) of M[f] = exp(alpha + beta.v - gamma |v|^2).
 * Returns BZ_EINVAL for batch < 0 or NULL buffers with batch > 0. */
#define BZ_Q_CORRECTED 1u
#define BZ_Q_MASS 2u
#define BZ_Q_CONSERVE 4u
bz_status bz_eval_Q(bz_ctx* ctx, const double* f, double* Q, int64_t batch, uint32_t flags,
                    double* theta, void* stream);

/* bz_eval_Q_noalloc: bz_eval_Q for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, flags, layouts, results and errors as
 * bz_eval_Q, but no allocating call (no hipMalloc, hipMallocAsync or hipFree)
 * is made.  The collision workspace, and the Maxwellian parameters the flags
 * need when theta is NULL, live in a static device array of 64 MiB per device,
 * held by the library until the process ends; cells are processed in chunks
 * that fit it.  Returns BZ_EINVAL, with a message, when one cell's workspace
 * exceeds the array.  With d = 3 the corrected form needs, per cell,
 * N^3 (104 + 16 n_theta) + 8 n_rho n_theta N (N + 1) + 40 bytes in FP64
 * (8.7 MB at 32^3 with n_theta = 8, n_rho = 16: 7 cells per chunk; 32^3 with
 * n_theta = 64, n_rho = 64 is refused) and N^3 (64 + 16 n_theta) bytes with an
 * FP32 spectral stage; d = 2 needs 32 bytes per
 * cell.  All calls on one device share that device's array and leave it
 * holding the last call's contents: calls that overlap on one device (other
 * streams, other host threads) race, and the caller must serialise them. */
bz_status bz_eval_Q_noalloc(bz_ctx* ctx, const double* f, double* Q, int64_t batch, uint32_t flags,
                            double* theta, void* stream);

/* ---------------------------------------------------------------- launch plans
 * How the collision pipeline is launched, without changing what it computes:
 *   pair_waves   waves per block of the N = 32 direction-pair kernel: 8 (one
 *                block per CU), 4 or 2 (two or four blocks per CU, so that one
 *                block's loads and final reduction overlap another's
 *                transforms); 0 = the default, 8
 *   chunk_cells  cells of one chunk of the pipeline's workspace (fewer when a
 *                caller-provided workspace holds fewer); a small chunk keeps a
 *                radial node's z-stage planes in the last-level cache between
 *                the z-stage and the pair kernel, a large one fills the GPU with
 *                fewer launches; 0 = as many as an 8 GiB workspace budget holds
 *   acc_nodes    radial nodes whose accumulated direction-pair planes are held
 *                in the workspace before one pass applies their axis-0
 *                transforms and radial weights to the gain spectrum (the sum
 *                runs in node order either way, so the result does not
 *                change); more nodes read and write the gain spectrum fewer
 *                times and take 16 bytes per cell and velocity each; 0 = all
 *                n_rho nodes (at most n_rho are used)
 * bz_set_plan / bz_get_plan set and read a context's plan (BZ_EINVAL for other
 * values).  bz_tune is the project's autotuner: it times bz_eval_Q(f, batch,
 * flags), reps times after a warm-up, under every candidate plan of the
 * context (pair_waves in {8, 4, 2} for the N = 32 sigma form, chunk_cells in
 * {0, 64, 24} with d = 3), reports each candidate's mean time in `report`,
 * keeps the fastest in the context and caches it for the discretisation
 * (device, d, N, precision, method, rule sizes, BZ_Q_CORRECTED): contexts
 * created later with the same discretisation start with it.  bz_tune
 * synchronises the stream and allocates a [batch][K] output buffer. */
#define BZ_TUNE_MAX 16
typedef struct {
  int pair_waves;
  int chunk_cells;
  int acc_nodes;
} bz_plan;

typedef struct {
  int n;                      /* candidates timed */
  bz_plan plan[BZ_TUNE_MAX];  /* the candidates */
  double ms[BZ_TUNE_MAX];     /* mean time of one bz_eval_Q under each */
  int best;                   /* index of the plan kept */
} bz_tune_report;

bz_status bz_set_plan(bz_ctx* ctx, const bz_plan* plan);
bz_status bz_get_plan(bz_ctx* ctx, bz_plan* plan);
bz_status bz_tune(bz_ctx* ctx, const double* f, int64_t batch, uint32_t flags, int reps, bz_tune_report* report,
                  void* stream);

/* bz_eval_Q_strided: bz_eval_Q on fields whose rows are ldf (input) and ldq
 * (output) doubles apart (ldf, ldq >= K; a row holds one cell's K values): a
 * batch that is a view into a larger array.  Rows of other strides are packed
 * into and unpacked from contiguous device buffers (stream-ordered
 * allocations), one extra pass each way; with ldf = ldq = K it is bz_eval_Q. */
bz_status bz_eval_Q_strided(bz_ctx* ctx, const double* f, int64_t ldf, double* Q, int64_t ldq, int64_t batch,
                            uint32_t flags, double* theta, void* stream);

/* bz_maxwellian: discrete Maxwellian of each cell (eqs. discrete_conservation,
 * discrete_Gaussian; Newton's method, Section 2.2).
 *   f [batch][K] in;  theta [batch][5] out (alpha, beta, gamma);
 *   M [batch][K] out, nullable;  newton_iters [batch] int32 out, nullable
 *   (negative when Newton did not converge). */
bz_status bz_maxwellian(bz_ctx* ctx, const double* f, double* theta, double* M, int32_t* newton_iters,
                        int64_t batch, void* stream);

/* ---------------------------------------------------------------- cell solve
 * Inner problem of one cell visit, eq. inner_eqn:
 *     (|v_1|/dx) g + r = (nu/eps) (M[g] - g).
 * mode BZ_SOLVE_PFP: preconditioned fixed point, eqs. step1 / step2, with the
 *     existence test of eq. existence; on failure (or when the step-1 Newton
 *     does not converge) the visit continues with the plain iteration.
 * mode BZ_SOLVE_FP: plain fixed point, eq. fix_point.
 * mode BZ_SOLVE_SI (slab scans with BGK collisions only): source iteration,
 *     eq. SI.  The Maxwellian and nu of the iterate at the start of an SGS
 *     iteration are kept through both of its scans, and each visit makes the
 *     single update g = D^{-1}(nu/eps M^n_j - r); tol, max_iter and
 *     fixed_iters are ignored.  The cell-solve calls, the cavity and a slab
 *     with a learned start attached reject it (BZ_EINVAL / BZ_EUNSUPPORTED).
 * The residual |(|v_1|/dx) g + r - (nu/eps)(M[g] - g)|_{L2(R^3)} is evaluated
 * after every update; iteration stops when it is <= tol or after max_iter
 * updates.  fixed_iters > 0 makes exactly that many updates (for one-to-one
 * comparisons of iterates). */
typedef enum { BZ_SOLVE_PFP = 0, BZ_SOLVE_FP = 1, BZ_SOLVE_SI = 2 } bz_solve_mode;

/* What a PFP update does when eq. existence fails for step 1's right-hand side s:
 * BZ_FALLBACK_FP continues the visit with the plain iteration (Section 3.2);
 * BZ_FALLBACK_RELAX takes the relaxed step 1 of the remark in Section 3.2,
 * s_tau = (s + tau sum w phi c M[g]) / (1 + tau), with the smallest tau in
 * {1, 2, 4, ..., 2^20} that satisfies eq. existence, and stays preconditioned
 * (falling back to the plain iteration only if that Newton solve fails). */
typedef enum { BZ_FALLBACK_FP = 0, BZ_FALLBACK_RELAX = 1 } bz_fallback;

typedef struct {
  int mode;        /* bz_solve_mode */
  double tol;      /* inner residual tolerance (1e-8 in Section 4) */
  int max_iter;    /* cap on updates per visit */
  int fixed_iters; /* > 0: exactly this many updates */
  int fallback;    /* bz_fallback (0: the plain iteration) */
} bz_solve_opts;

/* Per-cell statistics (device memory, written by the solve). */
typedef struct {
  int32_t iterations;  /* updates made */
  int32_t fallback;    /* 1 if the visit fell back to the plain iteration */
  int32_t newton_fail; /* Newton failures met during the visit */
  int32_t status;      /* 0 ok, 1 residual not below tol, 2 non-finite */
  double residual;     /* last inner residual */
  int32_t learned;     /* 1 if the learned initial guess was kept (learned path) */
  int32_t relaxed;     /* updates whose step 1 used the relaxation factor (BZ_FALLBACK_RELAX) */
} bz_cell_stats;

/* bz_cell_solve: `batch` independent inner problems.
 *   r  [batch][K] right-hand sides;  g0 [batch][K] initial guesses (may equal g);
 *   nu, eps [batch] per-cell collision frequency and Knudsen number (device);
 *   dx > 0 cell width;  g [batch][K] out;  stats [batch] device, nullable. */
bz_status bz_cell_solve(bz_ctx* ctx, const double* r, const double* nu, const double* eps, double dx,
                        const double* g0, double* g, int64_t batch, const bz_solve_opts* opts,
                        bz_cell_stats* stats, void* stream);

/* bz_cell_fixed_point: the data-parallel cell update of the SGS scan with the
 * binary collision operator (Section 3.3, eq. SGS): from the previous iterate
 * f_old of each cell it computes Q[f_old] (BZ_Q_CORRECTED | BZ_Q_MASS form), nu = 4 pi rho,
 * the BGK-penalty part P = Q - nu (M[f_old] - f_old) (eq. Pf), the right-hand
 * side r = inflow_r - P / eps, and solves eq. inner_eqn from g0 = f_old.
 *   f_old, inflow_r [batch][K];  eps [batch];  g [batch][K] out;
 *   inflow_r is the transport part of eq. r (neighbour and slope terms). */
bz_status bz_cell_fixed_point(bz_ctx* ctx, const double* f_old, const double* inflow_r, const double* eps,
                              double dx, double* g, int64_t batch, const bz_solve_opts* opts,
                              bz_cell_stats* stats, void* stream);

/* ---------------------------------------------------------------- learned warm start
 * A three-layer MLP  y = W3^T tanh(W2^T tanh(W1^T x + b1) + b2) + b3  that
 * predicts the correction g^0 - M[f_old] of a cell's initial guess (not part of
 * the paper's method: an addition whose only effect is the starting point of
 * the inner iteration, which still converges to the same fixed point).
 * Parameters are FP32 on the device; flat layout W1 [in][H], b1 [H],
 * W2 [H][H], b2 [H], W3 [H][out], b3 [out], row-major.  Inference uses BF16
 * matrix-core products with FP32 accumulation, training FP32 products.
 * bz_mlp_create: Glorot-uniform weights from `seed`, zero biases.
 * bz_mlp_forward: X [batch][in] FP32 device -> Y [batch][out] FP32 device;
 *   bf16 != 0 rounds X and the weights to BF16 for the products.
 * bz_mlp_grad: loss = mean((y - T)^2) (returned on the host when loss != NULL,
 *   which synchronises) and its gradient [num_params] FP32 device (nullable).
 * bz_mlp_train_step: one Adam step (beta 0.9 / 0.999, eps 1e-8) on that loss.
 * bz_mlp_features: the model input of each cell, width K + 6: inflow_r * dx
 *   (K values), rho, U_1..3, T of the Maxwellian theta, log10(eps); on a context
 *   with d = 2, width K + 5: inflow_r * dx, rho, U_1, U_2, T of theta [batch][4],
 *   log10(eps).
 * bz_mlp_set_output_scale: y is multiplied by this before it is added to
 *   M[f_old]. */
typedef struct bz_mlp bz_mlp;

bz_status bz_mlp_create(bz_ctx* ctx, int n_in, int hidden, int n_out, uint64_t seed, bz_mlp** out);
void bz_mlp_destroy(bz_mlp* mlp);
int64_t bz_mlp_num_params(bz_mlp* mlp);
bz_status bz_mlp_get_params(bz_mlp* mlp, float* host, int64_t n);
bz_status bz_mlp_set_params(bz_mlp* mlp, const float* host, int64_t n);
bz_status bz_mlp_set_output_scale(bz_mlp* mlp, double y_scale);
bz_status bz_mlp_forward(bz_mlp* mlp, const float* X, float* Y, int64_t batch, int bf16, void* stream);
bz_status bz_mlp_grad(bz_mlp* mlp, const float* X, const float* T, int64_t batch, float* grad, double* loss,
                      void* stream);
bz_status bz_mlp_train_step(bz_mlp* mlp, const float* X, const float* T, int64_t batch, double lr, double* loss,
                            void* stream);
bz_status bz_mlp_features(bz_ctx* ctx, const double* inflow_r, const double* theta, const double* eps, double dx,
                          float* X, int64_t batch, void* stream);

/* bz_cell_fixed_point_ex: bz_cell_fixed_point with the cell update's
 * remaining inputs given per cell:
 *   nu  [batch] device, nullable: the penalty frequency of eq. Pf used both in
 *       P = Q - nu (M - f_old) and in the visit (NULL: the matched frequency of
 *       the Maxwellian, as bz_cell_fixed_point);
 *   dxs [batch] device, nullable: each cell's width (NULL: dx for every cell);
 *   g0  [batch][K] device, nullable: the initial guesses (NULL: f_old); g may
 *       alias g0 but not f_old. */
bz_status bz_cell_fixed_point_ex(bz_ctx* ctx, const double* f_old, const double* inflow_r, const double* eps,
                                 const double* nu, double dx, const double* dxs, const double* g0, double* g,
                                 int64_t batch, const bz_solve_opts* opts, bz_cell_stats* stats, void* stream);

/* Strict mode (off by default).  Numerical events never fail a call by
 * themselves; with strict != 0, a call that synchronises with the host and
 * returns residuals (bz_sgs_sweep, bz_multigrid_vcycle, bz_outer_residual and
 * the bz_cavity_* sweeps, V-cycles and residual) returns BZ_ENUMERIC after
 * filling its outputs when one of them is not finite.  bz_cell_check
 * synchronises on `stream`, counts the cells of a cell call's statistics
 * (device [batch]) whose visit ended non-finite (status 2) into *n_bad (host,
 * nullable), and in strict mode returns BZ_ENUMERIC when there is one. */
bz_status bz_set_strict(bz_ctx* ctx, int strict);
bz_status bz_cell_check(bz_ctx* ctx, const bz_cell_stats* stats, int64_t batch, int64_t* n_bad, void* stream);

/* bz_cell_fixed_point_learned: bz_cell_fixed_point with a second candidate
 * initial guess g^0 = M[f_old] + scale * MLP(features) (BF16 inference); each
 * cell keeps the candidate (f_old or learned) with the smaller initial residual
 * of eq. inner_eqn, recorded in stats.learned.  mlp must have n_in = K + 6 and
 * n_out = K. */
bz_status bz_cell_fixed_point_learned(bz_ctx* ctx, bz_mlp* mlp, const double* f_old, const double* inflow_r,
                                      const double* eps, double dx, double* g, int64_t batch,
                                      const bz_solve_opts* opts, bz_cell_stats* stats, void* stream);

/* ---------------------------------------------------------------- 1D slabs
 * A set of independent 1D slab problems (instances) on x in [xL, xR] with
 * nx cells each, a diffuse wall (eq. boundary) or an inflow boundary at each
 * end, Knudsen number eps, and the total-mass constraint of eq. mass_conserv
 * (which also fixes the position of a shock between two inflow states).  Instances may
 * have different cell counts; their cells are stored back to back in the
 * caller's field buffer f [sum_i nx_i][K] (borrowed for the slab lifetime).
 * collision: BZ_COLL_BINARY (Q of eq. discrete_Q with the BZ_Q_MASS projection,
 * nu = 4 pi rho), BZ_COLL_BINARY_CONSERVE (the same with the BZ_Q_CONSERVE
 * projection instead), or BZ_COLL_BGK (P == 0, nu = bgk_nu if > 0 else 4 pi rho). */
typedef enum { BZ_COLL_BINARY = 0, BZ_COLL_BGK = 1, BZ_COLL_BINARY_CONSERVE = 2 } bz_collision;

typedef enum { BZ_BC_WALL = 0, BZ_BC_INFLOW = 1 } bz_boundary;

/* Slopes of the second-order scheme: BZ_LIMITER_NONE takes eq. slope (centred
 * inside); BZ_LIMITER_MINMOD takes minmod(f_{j+1} - f_j, f_j - f_{j-1}) inside
 * (a nonlinear limiter, which the explicit slopes of eq. SGS allow, Section
 * 3.1).  Both keep the one-sided differences at the first and last cell. */
typedef enum { BZ_LIMITER_NONE = 0, BZ_LIMITER_MINMOD = 1 } bz_limiter;

typedef struct {
  double xL, xR;
  int nx;
  double eps;
  double T_L, T_R;      /* wall / inflow temperatures */
  double U_L[3], U_R[3];/* physical velocities: of a wall (tangential, U[0] = 0)
                           or the bulk velocity of an inflow Maxwellian */
  double mass;          /* C in eq. mass_conserv */
  int bc_L, bc_R;       /* bz_boundary: BZ_BC_WALL, or BZ_BC_INFLOW for a ghost
                           cell holding rho M(T, U) on the incoming half-space */
  double rho_L, rho_R;  /* inflow densities (> 0; unused at walls) */
} bz_slab_instance;

typedef struct {
  int n_instances;
  const bz_slab_instance* instances; /* host array [n_instances] */
  int collision;                     /* bz_collision */
  double bgk_nu;                     /* BGK only; <= 0: 4 pi rho */
  bz_solve_opts inner;               /* inner solve options */
  double* f;                         /* device [sum nx][K], borrowed */
  int order;                         /* spatial order of eq. upwind: 1 (zero slopes) or 2
                                        (piecewise-linear reconstruction with the slopes of
                                        eq. slope: centred inside, one-sided at the two end
                                        cells, zero ghost slopes; taken from the iterate
                                        before each scan, so they enter the static part of
                                        r, Section 3.1).  The wall density then balances the
                                        flux of the face value f_0 - s_0/2 (left) or
                                        f_{nx-1} + s_{nx-1}/2 (right).  0 reads as 1. */
  int limiter;                       /* bz_limiter for second order (0: none) */
} bz_slab_desc;

typedef struct bz_slab bz_slab;

bz_status bz_slab_create(bz_ctx* ctx, const bz_slab_desc* desc, bz_slab** out);
void bz_slab_destroy(bz_slab* slab);

/* Statistics of the last sweep / V-cycle call (host memory, filled on return;
 * these calls synchronise the stream once at the end). */
typedef struct {
  int n_iters;           /* SGS iterations (or V-cycles) made */
  int64_t inner_iters;   /* total inner updates over all visits */
  int64_t visits;        /* cell visits */
  int64_t fallbacks;     /* visits that fell back to the plain iteration */
  int64_t learned;       /* visits that started from the learned guess (bz_ws_attach) */
} bz_sweep_stats;

/* bz_sgs_sweep: n_iters full SGS iterations (forward then backward scan,
 * eq. SGS, at the desc's spatial order), each followed by the uniform mass rescale of
 * Section 4.  P and nu of every cell are computed in one batched collision
 * evaluation before each scan (P is explicit); the cells of a scan are
 * then visited in order, one visit per instance at a time.
 * residual_out (host, nullable) [n_instances] receives each instance's outer
 * residual AFTER the last iteration. */
bz_status bz_sgs_sweep(bz_ctx* ctx, bz_slab* slab, int n_iters, double* residual_out, bz_sweep_stats* stats,
                       void* stream);

/* bz_slab_inflow: the transport part of eq. r for every cell of the slab's
 * current iterate, with both neighbours and the boundary ghosts (eq. boundary,
 * or the inflow Maxwellians) taken from that iterate:
 *   (v1- E - v1+ W) / dx - (v1+ s_W - v1 s + v1- s_E) / (2 dx),
 * W / E the left / right neighbour or ghost, s the slopes of eq. slope at
 * second order (zero in the ghosts), v1 the physical velocity.  It is what a
 * visit's r holds, less -P/eps, before any neighbour has been updated in the
 * scan: the input of the learned warm start, and of the cell problems that
 * train it.  out [sum nx][K] device. */
bz_status bz_slab_inflow(bz_ctx* ctx, bz_slab* slab, double* out, void* stream);

/* bz_ws_attach: use a warm-start network (bz_mlp with n_in = K + 6, n_out = K,
 * on the slab's context) in the slab's scans; NULL detaches.  Before each scan
 * every cell gets a second initial guess G = M[f_j] + scale * MLP(features of
 * bz_slab_inflow's row), BF16 inference with FP32 accumulation, computed for
 * all cells at once.  A visit starts from G instead of f_j when M[G] exists,
 * step 1 of the preconditioned update from G is solvable (eq. existence for
 * r_old), and G's inner residual |c g + r_old - (nu/eps)(M[g] - g)|_{L2} is the
 * smaller, r_old being
 * the visit's right-hand side with its upwind neighbour taken from the iterate
 * before the scan (the fresh value is not known then); the plain iteration of
 * the visit is unchanged, so the result is again the visit's inner solution,
 * to the inner tolerance.  bz_sweep_stats.learned counts the visits that
 * started from G.  The slab borrows the network; it must outlive the
 * attachment.  A slab with a network attached cannot be graph-captured
 * (BZ_EUNSUPPORTED).  Not part of the paper's method. */
bz_status bz_ws_attach(bz_slab* slab, bz_mlp* mlp);

/* bz_outer_residual: sqrt(sum_j dx sum_k w (v.grad f - Q/eps)^2) per instance
 * (Section 4 stopping rule), into residual_out (host) [n_instances]. */
bz_status bz_outer_residual(bz_ctx* ctx, bz_slab* slab, double* residual_out, void* stream);

/* ---------------------------------------------------------- 2D cavities
 * The lid-driven cavity family of Section 4.2: the unit square [0, 1]^2 with
 * nx x ny uniform cells, a diffuse wall (eq. boundary) on each side, two-
 * dimensional velocities (a context with d = 2), Knudsen number eps and the
 * total-mass constraint of eq. mass_conserv.  Upwind finite volumes (first
 * order shown; second order uses the face values, see `order`): for cell (i, j),
 *   [v1+ (f_ij - f_{i-1,j}) + v1- (f_{i+1,j} - f_ij)] / dx
 *     + [v2+ (f_ij - f_{i,j-1}) + v2- (f_{i,j+1} - f_ij)] / dy = Q[f_ij] / eps.
 * Cell (i, j) is stored at f + (i ny + j) K (borrowed for the cavity lifetime).
 * walls[0..3] are the sides x = 0, x = 1, y = 0, y = 1: temperature T and
 * velocity U (tangential: U[0] = 0 on x = 0 and x = 1, U[1] = 0 on y = 0 and
 * y = 1).  collision: BZ_COLL_BINARY (Q of eq. discrete_Q with the BZ_Q_MASS
 * projection, nu = 2 pi rho <|g|^gamma>) or BZ_COLL_BGK (P == 0, nu = bgk_nu if
 * > 0 else 2 pi rho). */
typedef struct {
  double T;
  double U[2];
} bz_wall;

typedef struct {
  int nx, ny;          /* cells along x and y (1 .. 4096 each) */
  double eps;          /* Knudsen number (> 0) */
  bz_wall walls[4];    /* x = 0, x = 1, y = 0, y = 1 */
  double mass;         /* C in eq. mass_conserv (> 0) */
  int collision;       /* BZ_COLL_BINARY or BZ_COLL_BGK */
  double bgk_nu;       /* BGK only; <= 0: 2 pi rho */
  bz_solve_opts inner; /* inner solve options */
  double* f;           /* device [nx ny][K], borrowed */
  int order;           /* 1 (0 reads as 1) or 2: the linear reconstruction of
                          eqs. reconstruction and slope along x and y, slopes
                          centred inside and one-sided at the ends of each line,
                          zero in the ghosts, taken from the iterate before each
                          scan; a wall then balances the flux of the adjacent
                          face value f -+ s/2 */
  int uniform_y;       /* != 0: the problem does not vary along y (ny must be 1):
                          no y transport and no y walls (walls[2], walls[3] are
                          ignored), two scans (+x, -x) per iteration, multigrid
                          coarsening along x only.  This is the 1D slab between
                          two plates with 2D velocities (Section 4.2). */
  int limiter;         /* bz_limiter for second order, along each axis (0: none) */
} bz_cavity_desc;

typedef struct bz_cavity bz_cavity;

bz_status bz_cavity_create(bz_ctx* ctx, const bz_cavity_desc* desc, bz_cavity** out);
void bz_cavity_destroy(bz_cavity* cav);

/* bz_cavity_sweep: n_iters SGS iterations, each four scans visiting the cells
 * in lexicographic order along (+x, +y), (-x, -y), (-x, +y), (+x, -y), then the
 * uniform mass rescale of Section 4.  Before each scan, P and nu of every cell
 * come from one batched collision evaluation (P is explicit, as in eq. SGS).
 * A visit uses the latest values of its four neighbours, so the cells of one
 * anti-diagonal (i + j constant in scan order) are independent: each
 * anti-diagonal is one launch with one workgroup per cell, which gives exactly
 * the lexicographic result.  At a wall the ghost value is rho_w M_w on the
 * incoming half-space, rho_w from the discrete zero-mass-flux balance with the
 * adjacent cell's latest value.  Each visit solves eq. inner_eqn with the
 * upwind diagonal c = |v1|/dx + |v2|/dy by the desc's inner options.
 * residual_out (host, nullable) receives the outer residual after the last
 * iteration. */
bz_status bz_cavity_sweep(bz_ctx* ctx, bz_cavity* cav, int n_iters, double* residual_out, bz_sweep_stats* stats,
                          void* stream);

/* bz_cavity_residual: sqrt(dx dy sum_ij sum_k w (v.grad f - Q/eps)^2), the
 * Section 4 stopping norm, into residual_out (host). */
bz_status bz_cavity_residual(bz_ctx* ctx, bz_cavity* cav, double* residual_out, void* stream);

/* bz_cavity_inflow: the transport part of every cell's visit right-hand side
 * (eq. r in two space dimensions) with all four neighbours and the wall ghosts
 * taken from the current field, plus the static reconstruction terms of its
 * slopes at second order: what a visit's r would be, less -P/eps, if no
 * neighbour had been updated yet.  out [nx * ny][K] device, cell (i, j) at row
 * i * ny + j. */
bz_status bz_cavity_inflow(bz_ctx* ctx, bz_cavity* cav, double* out, void* stream);

/* bz_cavity_ws_attach: use a warm-start network (bz_mlp with n_in = K + 5,
 * n_out = K, on the cavity's context) in the cavity's scans; NULL detaches.
 * Before each scan every cell gets a candidate G = M[f_ij] + scale *
 * MLP(features of bz_cavity_inflow's row, theta of f_ij, eps, dx), BF16
 * inference with FP32 accumulation.  The visit itself knows its right-hand
 * side r (the fresh neighbours of the wavefront included) and starts from G
 * instead of f_ij when M[G] exists, step 1 of the preconditioned update from G
 * satisfies eq. existence for r, and G's inner residual
 * |c g + r - (nu/eps)(M[g] - g)|_{L2} is the smaller.  The visit's iteration is
 * unchanged, so its result is again the inner solution to the inner tolerance.
 * bz_sweep_stats.learned counts the visits that started from G.  The cavity
 * borrows the network; it must outlive the attachment.  Not part of the
 * paper's method. */
bz_status bz_cavity_ws_attach(bz_cavity* cav, bz_mlp* mlp);

/* bz_multigrid_vcycle: n_cycles nonlinear multigrid V-cycles (eq. coarse,
 * H = 2h) with SGS-PFP smoothing (nu1 pre-, nu2 post-steps, tab. mg), a
 * coarsest level of `coarsest` cells smoothed until its residual falls 10x or
 * coarse_iters iterations pass, and a mass rescale after each cycle.  Every
 * instance's cell count must be coarsest * 2^k.  A cycle stops descending
 * once a level's residual is below `tol`.  With fixed_cycle != 0 the cycle has
 * no data-dependent exit: every level descends (tol is not consulted) and the
 * coarsest level runs exactly coarse_iters iterations, so the cycle makes no
 * host synchronisation; this is the cycle bz_graph_capture_vcycles records
 * (the cavity rejects it with BZ_EUNSUPPORTED). */
typedef struct {
  int coarsest;
  int nu1, nu2;
  int coarse_iters;
  double tol;
  int fixed_cycle;
} bz_mg_opts;

bz_status bz_multigrid_vcycle(bz_ctx* ctx, bz_slab* slab, const bz_mg_opts* opts, int n_cycles,
                              double* residual_out, bz_sweep_stats* stats, void* stream);

/* bz_cavity_vcycle: n_cycles nonlinear multigrid V-cycles (eq. coarse) on a
 * 2D cavity, with H = 2h in both directions.  Each level runs nu1 pre- and nu2
 * post-smoothing SGS iterations (four scans each) with its FAS source.
 * Restriction averages the four children; prolongation adds the coarse
 * correction to each child.  Levels halve nx and ny until min(nx, ny) <=
 * coarsest, so nx and ny must halve evenly down to there.  That level is
 * smoothed until its residual falls 10x or coarse_iters iterations pass.  A
 * cycle stops descending once a level's residual is below tol, and the mass
 * rescale follows each cycle.  Coarse levels are allocated on the first call.
 * residual_out (host, nullable) receives the outer residual after the last
 * cycle. */
bz_status bz_cavity_vcycle(bz_ctx* ctx, bz_cavity* cav, const bz_mg_opts* opts, int n_cycles, double* residual_out,
                           bz_sweep_stats* stats, void* stream);

/* ---------------------------------------------------------------- graph replay
 * For callers that run many SGS iterations and want one host synchronisation
 * per segment instead of one per iteration (launch-bound small slabs, serving
 * loops): bz_graph_capture_sweeps records iters_per_replay SGS iterations of
 * bz_sgs_sweep (two scans and the mass rescale each), and with with_residual
 * != 0 the outer residual of the result, into a HIP graph; bz_graph_launch
 * replays it on `stream` and, when requested, returns the per-instance
 * residuals (host, [n_instances], needs with_residual) and the statistics of
 * the replay, synchronising once.  Capture needs a non-default stream; the
 * collision workspace is sized before the capture, and the graph holds no
 * allocation and no memset node.  The graph borrows the slab and its field f:
 * replays read and update f in place, and the slab must outlive the graph.
 * Graphs of one slab must not be replayed concurrently.  Returns BZ_EINVAL for
 * iters_per_replay < 1, a NULL stream, or a residual request on a graph
 * captured without it. */
typedef struct bz_graph bz_graph;
bz_status bz_graph_capture_sweeps(bz_ctx* ctx, bz_slab* slab, int iters_per_replay, int with_residual,
                                  void* stream, bz_graph** out);
/* bz_graph_capture_vcycles: the same for cycles_per_replay FAS V-cycles (eq.
 * coarse) of bz_multigrid_vcycle with opts->fixed_cycle forced on (no early
 * exit, so the replay is one fixed launch sequence), each followed by the mass
 * rescale.  The coarse levels are allocated before the capture.  A slab with a
 * learned start attached is refused (BZ_EUNSUPPORTED). */
bz_status bz_graph_capture_vcycles(bz_ctx* ctx, bz_slab* slab, const bz_mg_opts* opts, int cycles_per_replay,
                                   int with_residual, void* stream, bz_graph** out);
bz_status bz_graph_launch(bz_graph* graph, double* residual_out, bz_sweep_stats* stats, void* stream);
void bz_graph_destroy(bz_graph* graph);

/* ---------------------------------------------------------------- profiling
 * bz_profile_enable(ctx, 1) makes the library record a pair of HIP events
 * around every launch of the direction-pair kernel (the dominant kernel of
 * bz_eval_Q), on the stream it is launched on; 0 disables and clears.
 * bz_profile_get synchronises the device and returns, since enabling, the
 * number of launches, their summed duration (ms) and the algorithmic FLOPs
 * they performed: per launch, cells * N * pairs * fields *
 * (10 N^2 log2 N + 17 N^2) - one N x N complex inverse transform per
 * (plane, pair, field combination), the two phase products, the combination
 * into one complex field and the weighted product accumulation. */
typedef struct {
  int64_t launches;
  double total_ms;
  double flops;
} bz_profile_info;

bz_status bz_profile_enable(bz_ctx* ctx, int enable);
bz_status bz_profile_get(bz_ctx* ctx, bz_profile_info* out);

#ifdef __cplusplus
}
#endif
#endif /* BZ_H */
