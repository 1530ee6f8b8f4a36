// C ABI entry points: validation, context lifetime, workspace.
#include <cmath>
#include <cstring>
#include <vector>
#include <string>

#include "bz_internal.hpp"

namespace bz {

bz_status set_err(bz_ctx* c, bz_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

bz_status hip_err(bz_ctx* c, hipError_t e, const char* what) {
  return set_err(c, e == hipErrorOutOfMemory ? BZ_ENOMEM : BZ_EHIP,
                 std::string(what) + ": " + hipGetErrorString(e));
}

bz_status ensure_ws(bz_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return BZ_OK;
  if (ctx->ws) {
    // the workspace may still be in use by queued work on any stream
    BZ_HIP(hipDeviceSynchronize());
    BZ_HIP(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  BZ_HIP(hipMalloc(&ctx->ws, bytes));
  ctx->ws_bytes = bytes;
  return BZ_OK;
}

bz_status prof_mark(bz_ctx* ctx, hipStream_t st, bool stop, double flops) {
  if (!ctx->prof) return BZ_OK;
  if (ctx->prof_used == ctx->prof_ev.size()) {
    hipEvent_t e;
    BZ_HIP(hipEventCreate(&e));
    ctx->prof_ev.push_back(e);
  }
  BZ_HIP(hipEventRecord(ctx->prof_ev[ctx->prof_used++], st));
  if (stop) ctx->prof_flops += flops;
  return BZ_OK;
}

}  // namespace bz

using bz::set_err;

extern "C" {

const char* bz_status_str(bz_status s) {
  switch (s) {
    case BZ_OK: return "ok";
    case BZ_EINVAL: return "invalid argument";
    case BZ_ENOMEM: return "out of device memory";
    case BZ_EHIP: return "HIP runtime error";
    case BZ_EUNSUPPORTED: return "unsupported";
    case BZ_ENUMERIC: return "non-finite result (strict mode)";
  }
  return "unknown status";
}

bz_status bz_last_error(bz_ctx* ctx, char* buf, size_t n) {
  if (!ctx || !buf || n == 0) return BZ_EINVAL;
  std::strncpy(buf, ctx->err.c_str(), n - 1);
  buf[n - 1] = '\0';
  return BZ_OK;
}

size_t bz_workspace_bytes(bz_ctx* ctx) { return ctx ? ctx->ws_bytes : 0; }

bz_status bz_create(const bz_params* p, bz_ctx** out) {
  if (!out) return BZ_EINVAL;
  *out = nullptr;
  if (!p) return BZ_EINVAL;
  const int d = p->d == 0 ? 3 : p->d;
  if (d != 1 && d != 2 && d != 3) return BZ_EINVAL;
  // one velocity dimension serves the BGK slab only: up to 64 nodes, FP64, no shift
  if (d == 1 && (p->N < 2 || p->N > 64 || p->N % 2 || p->precision != BZ_FP64 || p->v1_shift != 0.0 ||
                 p->method != BZ_METHOD_SIGMA))
    return BZ_EINVAL;
  if (d == 3 && !(p->N == 8 || p->N == 16 || p->N == 32)) return BZ_EINVAL;
  if (d == 2 && !(p->N == 8 || p->N == 12 || p->N == 16 || p->N == 24 || p->N == 32 || p->N == 48))
    return BZ_EINVAL;
  if (!(p->L > 0) || !std::isfinite(p->L)) return BZ_EINVAL;
  if (d == 3 && (p->n_theta < 2 || p->n_theta % 2 || p->n_theta > 64)) return BZ_EINVAL;
  if (d > 1 && (p->n_phi < 2 || p->n_phi % 2 || p->n_phi > 256)) return BZ_EINVAL;
  if (d > 1 && (p->n_rho < 1 || p->n_rho > 256)) return BZ_EINVAL;
  if (p->precision != BZ_FP64 && p->precision != BZ_FP32 && p->precision != BZ_FP32_DIFF) return BZ_EINVAL;
  // the FP32 difference form: 3D velocities, sigma form (its Maxwellian part is separable)
  if (p->precision == BZ_FP32_DIFF && (d != 3 || p->method != BZ_METHOD_SIGMA)) return BZ_EUNSUPPORTED;
  if (!(p->gamma > -3.0) || p->gamma > 2.0) return BZ_EINVAL;
  if (!std::isfinite(p->v1_shift) || std::fabs(p->v1_shift) > 1e6) return BZ_EINVAL;
  if (p->method != BZ_METHOD_SIGMA && p->method != BZ_METHOD_CARLEMAN) return BZ_EINVAL;
  // Carleman form: hard spheres in 3D, Maxwell molecules in 2D (the kernels whose
  // Carleman weight is constant)
  if (p->method == BZ_METHOD_CARLEMAN && p->gamma != (d == 3 ? 1.0 : 0.0)) return BZ_EUNSUPPORTED;
  if (d == 2 && p->v1_shift != 0.0) return BZ_EUNSUPPORTED;
  bz_ctx* ctx = new bz_ctx();
  ctx->p = *p;
  ctx->p.d = d;
  ctx->d = d;
  ctx->N = p->N;
  ctx->K = d == 3 ? p->N * p->N * p->N : d == 2 ? p->N * p->N : p->N;
  ctx->n_theta = p->n_theta;
  ctx->n_phi = p->n_phi;
  ctx->n_rho = p->n_rho;
  ctx->dv = 2.0 * p->L / p->N;
  ctx->w = d == 3 ? ctx->dv * ctx->dv * ctx->dv : d == 2 ? ctx->dv * ctx->dv : ctx->dv;
  ctx->R = p->R > 0 ? p->R : 2.0 * p->L / (3.0 * std::sqrt(2.0) + 1.0);
  ctx->Rg = 2.0 * ctx->R;
  // <|g|^gamma> = (4T)^{gamma/2} Gamma((d + gamma)/2) / Gamma(d/2): the T-independent factor
  ctx->nu_gfac = std::pow(4.0, 0.5 * p->gamma) * std::tgamma(0.5 * (d + p->gamma)) / std::tgamma(0.5 * d);
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) {
    delete ctx;
    return BZ_EHIP;
  }
  bz_status s = bz::build_tables(ctx);
  if (s == BZ_OK) s = bz::scratch_attach(ctx);
  if (s == BZ_OK) bz::apply_cached_plan(ctx);
  if (s != BZ_OK) {
    bz::free_tables(ctx);
    delete ctx;
    return s;
  }
  *out = ctx;
  return BZ_OK;
}

void bz_destroy(bz_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->p.device);
  (void)hipDeviceSynchronize();
  bz::free_tables(ctx);
  if (ctx->ws) (void)hipFree(ctx->ws);
  for (hipEvent_t e : ctx->prof_ev) (void)hipEventDestroy(e);
  delete ctx;
}

bz_status bz_profile_enable(bz_ctx* ctx, int enable) {
  if (!ctx) return BZ_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return set_err(ctx, BZ_EHIP, "hipDeviceSynchronize");
  ctx->prof = enable != 0;
  ctx->prof_used = 0;
  ctx->prof_flops = 0.0;
  return BZ_OK;
}

bz_status bz_profile_get(bz_ctx* ctx, bz_profile_info* out) {
  if (!ctx || !out) return BZ_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return set_err(ctx, BZ_EHIP, "hipDeviceSynchronize");
  double ms = 0.0;
  for (size_t i = 0; i + 1 < ctx->prof_used; i += 2) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, ctx->prof_ev[i], ctx->prof_ev[i + 1]) != hipSuccess)
      return set_err(ctx, BZ_EHIP, "hipEventElapsedTime");
    ms += t;
  }
  out->launches = (int64_t)(ctx->prof_used / 2);
  out->total_ms = ms;
  out->flops = ctx->prof_flops;
  return BZ_OK;
}

}  // extern "C"

namespace bz {

bz_status check_eval_q_args(bz_ctx* ctx, const double* f, const double* Q, int64_t batch, uint32_t flags,
                            const double* theta) {
  if (!ctx) return BZ_EINVAL;
  if (batch < 0) return set_err(ctx, BZ_EINVAL, "batch < 0");
  if (batch > 0 && (!f || !Q)) return set_err(ctx, BZ_EINVAL, "NULL field buffer");
  if (flags & ~(BZ_Q_CORRECTED | BZ_Q_MASS | BZ_Q_CONSERVE)) return set_err(ctx, BZ_EINVAL, "unknown flag");
  if ((flags & BZ_Q_MASS) && (flags & BZ_Q_CONSERVE)) return set_err(ctx, BZ_EINVAL, "BZ_Q_MASS with BZ_Q_CONSERVE");
  if ((flags & BZ_Q_CONSERVE) && !(flags & BZ_Q_CORRECTED))
    return set_err(ctx, BZ_EINVAL, "BZ_Q_CONSERVE requires BZ_Q_CORRECTED");
  if (theta && !(flags & BZ_Q_CORRECTED)) return set_err(ctx, BZ_EINVAL, "theta requires BZ_Q_CORRECTED");
  if ((flags & BZ_Q_MASS) && !(flags & BZ_Q_CORRECTED)) return set_err(ctx, BZ_EINVAL, "BZ_Q_MASS requires BZ_Q_CORRECTED");
  if (ctx->d == 2 && (flags & BZ_Q_CONSERVE)) return set_err(ctx, BZ_EUNSUPPORTED, "BZ_Q_CONSERVE with d = 2");
  if (ctx->d == 1) return set_err(ctx, BZ_EUNSUPPORTED, "a context with d = 1 serves the BGK slab only");
  return BZ_OK;
}

bz_status strict_check(bz_ctx* ctx, const double* vals, int64_t n) {
  if (!ctx->strict || !vals) return BZ_OK;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(vals[i])) return set_err(ctx, BZ_ENUMERIC, "a returned residual is not finite");
  return BZ_OK;
}

}  // namespace bz

extern "C" {

bz_status bz_eval_Q(bz_ctx* ctx, const double* f, double* Q, int64_t batch, uint32_t flags, double* theta,
                    void* stream) {
  bz_status cs = bz::check_eval_q_args(ctx, f, Q, batch, flags, theta);
  if (cs != BZ_OK) return cs;
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (ctx->d == 2)
    return bz::v2_eval_q(ctx, f, Q, batch, (flags & BZ_Q_CORRECTED) != 0, (flags & BZ_Q_MASS) != 0, theta, st);
  if (!(flags & (BZ_Q_MASS | BZ_Q_CONSERVE)) || batch == 0)
    return bz::eval_q(ctx, f, Q, batch, (flags & BZ_Q_CORRECTED) != 0, theta, st);
  double* th = theta;
  if (!th) {
    hipError_t e = hipMallocAsync((void**)&th, (size_t)batch * 5 * sizeof(double), st);
    if (e != hipSuccess) return bz::hip_err(ctx, e, "hipMallocAsync");
  }
  bz_status s = bz::eval_q(ctx, f, Q, batch, true, th, st);
  if (s == BZ_OK)
    s = (flags & BZ_Q_CONSERVE) ? bz::conserve_project(ctx, Q, th, batch, st) : bz::mass_project(ctx, Q, th, batch, st);
  if (!theta) (void)hipFreeAsync(th, st);
  return s;
}

bz_status bz_eval_Q_strided(bz_ctx* ctx, const double* f, int64_t ldf, double* Q, int64_t ldq, int64_t batch,
                            uint32_t flags, double* theta, void* stream) {
  bz_status cs = bz::check_eval_q_args(ctx, f, Q, batch, flags, theta);
  if (cs != BZ_OK) return cs;
  const int64_t K = ctx->K;
  if (ldf < K || ldq < K) return set_err(ctx, BZ_EINVAL, "row strides must be >= K");
  if (ldf == K && ldq == K) return bz_eval_Q(ctx, f, Q, batch, flags, theta, stream);
  if (batch == 0) return BZ_OK;
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const size_t row = (size_t)K * sizeof(double), bytes = row * (size_t)batch;
  double *fp = const_cast<double*>(f), *qp = Q;
  hipError_t e = hipSuccess;
  if (ldf != K && (e = hipMallocAsync((void**)&fp, bytes, st)) != hipSuccess) return bz::hip_err(ctx, e, "hipMallocAsync");
  if (ldq != K && (e = hipMallocAsync((void**)&qp, bytes, st)) != hipSuccess) {
    if (fp != f) (void)hipFreeAsync(fp, st);
    return bz::hip_err(ctx, e, "hipMallocAsync");
  }
  bz_status s = BZ_OK;
  if (fp != f && (e = hipMemcpy2DAsync(fp, row, f, (size_t)ldf * sizeof(double), row, (size_t)batch,
                                       hipMemcpyDeviceToDevice, st)) != hipSuccess)
    s = bz::hip_err(ctx, e, "pack f");
  if (s == BZ_OK) s = bz_eval_Q(ctx, fp, qp, batch, flags, theta, stream);
  if (s == BZ_OK && qp != Q &&
      (e = hipMemcpy2DAsync(Q, (size_t)ldq * sizeof(double), qp, row, row, (size_t)batch, hipMemcpyDeviceToDevice,
                            st)) != hipSuccess)
    s = bz::hip_err(ctx, e, "unpack Q");
  if (fp != f) (void)hipFreeAsync(fp, st);
  if (qp != Q) (void)hipFreeAsync(qp, st);
  return s;
}

bz_status bz_maxwellian(bz_ctx* ctx, const double* f, double* theta, double* M, int32_t* newton_iters, int64_t batch,
                        void* stream) {
  if (!ctx) return BZ_EINVAL;
  if (batch < 0) return set_err(ctx, BZ_EINVAL, "batch < 0");
  if (batch > 0 && (!f || !theta)) return set_err(ctx, BZ_EINVAL, "NULL buffer");
  if (ctx->d == 1) return set_err(ctx, BZ_EUNSUPPORTED, "a context with d = 1 serves the BGK slab only");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  if (ctx->d == 2) return bz::v2_maxwellian(ctx, f, theta, M, newton_iters, batch, (hipStream_t)stream);
  return bz::maxwellian(ctx, f, theta, M, newton_iters, batch, (hipStream_t)stream);
}

static bz_status check_opts(bz_ctx* ctx, const bz_solve_opts* o) {
  if (!o) return set_err(ctx, BZ_EINVAL, "NULL solve options");
  if (o->mode != BZ_SOLVE_PFP && o->mode != BZ_SOLVE_FP) return set_err(ctx, BZ_EINVAL, "bad solve mode");
  if (o->fixed_iters < 0 || o->fixed_iters > 100000) return set_err(ctx, BZ_EINVAL, "bad fixed_iters");
  if (o->fixed_iters == 0 && (o->max_iter < 1 || o->max_iter > 100000))
    return set_err(ctx, BZ_EINVAL, "max_iter must be in [1, 100000]");
  if (!(o->tol >= 0) || !std::isfinite(o->tol)) return set_err(ctx, BZ_EINVAL, "bad tol");
  if (o->fallback != BZ_FALLBACK_FP && o->fallback != BZ_FALLBACK_RELAX) return set_err(ctx, BZ_EINVAL, "bad fallback");
  return BZ_OK;
}

bz_status bz_cell_solve(bz_ctx* ctx, const double* r, const double* nu, const double* eps, double dx, const double* g0,
                        double* g, int64_t batch, const bz_solve_opts* opts, bz_cell_stats* stats, void* stream) {
  if (!ctx) return BZ_EINVAL;
  if (ctx->d != 3) return set_err(ctx, BZ_EUNSUPPORTED, "this call needs d = 3");
  if (batch < 0) return set_err(ctx, BZ_EINVAL, "batch < 0");
  bz_status s = check_opts(ctx, opts);
  if (s != BZ_OK) return s;
  if (!(dx > 0) || !std::isfinite(dx)) return set_err(ctx, BZ_EINVAL, "dx must be > 0");
  if (batch > 0 && (!r || !nu || !eps || !g0 || !g)) return set_err(ctx, BZ_EINVAL, "NULL buffer");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  return bz::cell_solve(ctx, r, nu, eps, dx, g0, g, batch, opts, stats, (hipStream_t)stream);
}

bz_status bz_cell_fixed_point(bz_ctx* ctx, const double* f_old, const double* inflow_r, const double* eps, double dx,
                              double* g, int64_t batch, const bz_solve_opts* opts, bz_cell_stats* stats,
                              void* stream) {
  if (!ctx) return BZ_EINVAL;
  if (ctx->d != 3) return set_err(ctx, BZ_EUNSUPPORTED, "this call needs d = 3");
  if (batch < 0) return set_err(ctx, BZ_EINVAL, "batch < 0");
  bz_status s = check_opts(ctx, opts);
  if (s != BZ_OK) return s;
  if (!(dx > 0) || !std::isfinite(dx)) return set_err(ctx, BZ_EINVAL, "dx must be > 0");
  if (batch == 0) return BZ_OK;
  if (!f_old || !inflow_r || !eps || !g) return set_err(ctx, BZ_EINVAL, "NULL buffer");
  if (g == f_old) return set_err(ctx, BZ_EINVAL, "g must not alias f_old");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  // scratch: Q, r [batch][K], theta [batch][5], nu [batch] (separate from the
  // collision workspace, which eval_q sizes itself)
  const size_t K = (size_t)ctx->K;
  double* buf = nullptr;
  const size_t bytes = (size_t)batch * (2 * K + 6) * sizeof(double);
  hipError_t e = hipMallocAsync((void**)&buf, bytes, st);
  if (e != hipSuccess) return bz::hip_err(ctx, e, "hipMallocAsync");
  double* Q = buf;
  double* r = Q + batch * K;
  double* theta = r + batch * K;
  double* nu = theta + batch * 5;
  s = bz::eval_q(ctx, f_old, Q, batch, true, theta, st);
  if (s == BZ_OK) s = bz::mass_project(ctx, Q, theta, batch, st);
  if (s == BZ_OK) s = bz::penalty_rhs(ctx, f_old, Q, theta, inflow_r, eps, r, nu, batch, st);
  if (s == BZ_OK) s = bz::cell_solve(ctx, r, nu, eps, dx, f_old, g, batch, opts, stats, st);
  (void)hipFreeAsync(buf, st);
  return s;
}

bz_status bz_cell_fixed_point_ex(bz_ctx* ctx, const double* f_old, const double* inflow_r, const double* eps,
                                 const double* nu_in, double dx, const double* dxs, const double* g0, double* g,
                                 int64_t batch, const bz_solve_opts* opts, bz_cell_stats* stats, void* stream) {
  if (!ctx) return BZ_EINVAL;
  if (ctx->d != 3) return set_err(ctx, BZ_EUNSUPPORTED, "this call needs d = 3");
  if (batch < 0) return set_err(ctx, BZ_EINVAL, "batch < 0");
  bz_status s = check_opts(ctx, opts);
  if (s != BZ_OK) return s;
  if (!dxs && (!(dx > 0) || !std::isfinite(dx))) return set_err(ctx, BZ_EINVAL, "dx must be > 0");
  if (batch == 0) return BZ_OK;
  if (!f_old || !inflow_r || !eps || !g) return set_err(ctx, BZ_EINVAL, "NULL buffer");
  if (g == f_old) return set_err(ctx, BZ_EINVAL, "g must not alias f_old");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const size_t K = (size_t)ctx->K;
  double* buf = nullptr;
  const size_t bytes = (size_t)batch * (2 * K + 6) * sizeof(double);
  hipError_t e = hipMallocAsync((void**)&buf, bytes, st);
  if (e != hipSuccess) return bz::hip_err(ctx, e, "hipMallocAsync");
  double* Q = buf;
  double* r = Q + batch * K;
  double* theta = r + batch * K;
  double* nu = theta + batch * 5;
  s = bz::eval_q(ctx, f_old, Q, batch, true, theta, st);
  if (s == BZ_OK) s = bz::mass_project(ctx, Q, theta, batch, st);
  if (s == BZ_OK) s = bz::penalty_rhs(ctx, f_old, Q, theta, inflow_r, eps, r, nu, batch, st, nu_in);
  if (s == BZ_OK) s = bz::cell_solve(ctx, r, nu, eps, dx, g0 ? g0 : f_old, g, batch, opts, stats, st, nullptr, dxs);
  (void)hipFreeAsync(buf, st);
  return s;
}

bz_status bz_set_strict(bz_ctx* ctx, int strict) {
  if (!ctx) return BZ_EINVAL;
  ctx->strict = strict != 0;
  return BZ_OK;
}

bz_status bz_cell_check(bz_ctx* ctx, const bz_cell_stats* stats, int64_t batch, int64_t* n_bad, void* stream) {
  if (!ctx || batch < 0 || (batch > 0 && !stats)) return BZ_EINVAL;
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  std::vector<bz_cell_stats> h((size_t)batch);
  if (batch > 0) {
    hipError_t e = hipMemcpyAsync(h.data(), stats, sizeof(bz_cell_stats) * (size_t)batch, hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return bz::hip_err(ctx, e, "reading cell statistics");
  }
  int64_t bad = 0;
  for (const bz_cell_stats& c : h) bad += c.status == 2 ? 1 : 0;
  if (n_bad) *n_bad = bad;
  if (ctx->strict && bad > 0) return set_err(ctx, BZ_ENUMERIC, std::to_string(bad) + " cells ended non-finite");
  return BZ_OK;
}

bz_status bz_cell_fixed_point_learned(bz_ctx* ctx, bz_mlp* mlp, const double* f_old, const double* inflow_r,
                                      const double* eps, double dx, double* g, int64_t batch,
                                      const bz_solve_opts* opts, bz_cell_stats* stats, void* stream) {
  if (!ctx || !mlp) return BZ_EINVAL;
  if (ctx->d != 3) return set_err(ctx, BZ_EUNSUPPORTED, "this call needs d = 3");
  if (batch < 0) return set_err(ctx, BZ_EINVAL, "batch < 0");
  bz_status s = check_opts(ctx, opts);
  if (s != BZ_OK) return s;
  if (!(dx > 0) || !std::isfinite(dx)) return set_err(ctx, BZ_EINVAL, "dx must be > 0");
  if (batch == 0) return BZ_OK;
  if (!f_old || !inflow_r || !eps || !g) return set_err(ctx, BZ_EINVAL, "NULL buffer");
  if (g == f_old) return set_err(ctx, BZ_EINVAL, "g must not alias f_old");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const size_t K = (size_t)ctx->K;
  double* buf = nullptr;
  const size_t bytes = (size_t)batch * (3 * K + 6) * sizeof(double);
  hipError_t e = hipMallocAsync((void**)&buf, bytes, st);
  if (e != hipSuccess) return bz::hip_err(ctx, e, "hipMallocAsync");
  double* Q = buf;
  double* r = Q + batch * K;
  double* g0l = r + batch * K;
  double* theta = g0l + batch * K;
  double* nu = theta + batch * 5;
  s = bz::eval_q(ctx, f_old, Q, batch, true, theta, st);
  if (s == BZ_OK) s = bz::mass_project(ctx, Q, theta, batch, st);
  if (s == BZ_OK) s = bz::penalty_rhs(ctx, f_old, Q, theta, inflow_r, eps, r, nu, batch, st);
  if (s == BZ_OK) s = bz::learned_guess(ctx, mlp, inflow_r, theta, eps, dx, g0l, batch, st);
  if (s == BZ_OK) s = bz::cell_solve(ctx, r, nu, eps, dx, f_old, g, batch, opts, stats, st, g0l);
  (void)hipFreeAsync(buf, st);
  return s;
}

}  // extern "C"
