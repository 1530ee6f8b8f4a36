// Launch-plan tuner of the collision pipeline: the waves per block of the
// N = 32 direction-pair kernel (8, 4 or 2: one, two or four blocks per CU) and
// the cells per chunk of the pipeline's workspace (the 8 GiB budget, 64 or 24
// cells: a smaller chunk keeps a radial node's z-stage planes in the 256 MB
// last-level cache between the z-stage and the pair kernel); the radial nodes
// held per column pass stay the context's.  Every candidate
// computes the same operator; the tuner times bz_eval_Q on the caller's batch
// under each and keeps the fastest, in the context and in a process-wide cache
// keyed by the discretisation, which bz_create consults.
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "bz_internal.hpp"

namespace {

using Key = std::tuple<int, int, int, int, int, int, int, int, int>;

std::mutex g_mu;
std::map<Key, bz_plan> g_cache;

Key key_of(const bz_ctx* ctx, uint32_t flags) {
  return Key{ctx->p.device, ctx->d, ctx->N, ctx->p.precision, ctx->p.method, ctx->n_theta, ctx->n_phi, ctx->n_rho,
             (int)(flags & BZ_Q_CORRECTED)};
}

bool plan_ok(const bz_plan* p) {
  const bool w_ok = p->pair_waves == 0 || p->pair_waves == 2 || p->pair_waves == 4 || p->pair_waves == 8;
  return w_ok && p->chunk_cells >= 0 && p->acc_nodes >= 0;
}

}  // namespace

namespace bz {

void apply_cached_plan(bz_ctx* ctx) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_cache.find(key_of(ctx, BZ_Q_CORRECTED));
  if (it != g_cache.end()) {
    ctx->pair_waves = it->second.pair_waves;
    ctx->chunk_cap = it->second.chunk_cells;
    ctx->acc_nodes = it->second.acc_nodes;
  }
}

}  // namespace bz

using bz::set_err;

extern "C" {

bz_status bz_set_plan(bz_ctx* ctx, const bz_plan* plan) {
  if (!ctx || !plan) return BZ_EINVAL;
  if (!plan_ok(plan))
    return set_err(ctx, BZ_EINVAL, "pair_waves must be 0, 2, 4 or 8, chunk_cells and acc_nodes >= 0");
  ctx->pair_waves = plan->pair_waves;
  ctx->chunk_cap = plan->chunk_cells;
  ctx->acc_nodes = plan->acc_nodes;
  return BZ_OK;
}

bz_status bz_get_plan(bz_ctx* ctx, bz_plan* plan) {
  if (!ctx || !plan) return BZ_EINVAL;
  plan->pair_waves = ctx->pair_waves;
  plan->chunk_cells = ctx->chunk_cap;
  plan->acc_nodes = ctx->acc_nodes;
  return BZ_OK;
}

bz_status bz_tune(bz_ctx* ctx, const double* f, int64_t batch, uint32_t flags, int reps, bz_tune_report* report,
                  void* stream) {
  if (!ctx || !report) return BZ_EINVAL;
  if (batch < 1 || !f) return set_err(ctx, BZ_EINVAL, "bz_tune needs a non-empty batch");
  if (reps < 1 || reps > 100) return set_err(ctx, BZ_EINVAL, "reps must be in [1, 100]");
  if (flags & ~(BZ_Q_CORRECTED | BZ_Q_MASS | BZ_Q_CONSERVE)) return set_err(ctx, BZ_EINVAL, "unknown flag");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  std::memset(report, 0, sizeof(*report));
  std::vector<bz_plan> cand;
  const bool pairs32 = ctx->d == 3 && ctx->N == 32 && ctx->p.method == BZ_METHOD_SIGMA;
  const int waves[3] = {8, 4, 2};
  const int chunks[3] = {0, 64, 24};
  for (int w = 0; w < (pairs32 ? 3 : 1); ++w)
    for (int c = 0; c < (ctx->d == 3 ? 3 : 1); ++c)
      cand.push_back(bz_plan{pairs32 ? waves[w] : 0, chunks[c], ctx->acc_nodes});
  if ((int)cand.size() > BZ_TUNE_MAX) cand.resize(BZ_TUNE_MAX);
  double* Q = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bz_status s = BZ_OK;
  const bz_plan saved{ctx->pair_waves, ctx->chunk_cap, ctx->acc_nodes};
  if (hipMalloc((void**)&Q, sizeof(double) * (size_t)ctx->K * batch) != hipSuccess)
    return set_err(ctx, BZ_ENOMEM, "tuner output buffer");
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) s = set_err(ctx, BZ_EHIP, "event");
  int best = -1;
  for (size_t i = 0; i < cand.size() && s == BZ_OK; ++i) {
    ctx->pair_waves = cand[i].pair_waves;
    ctx->chunk_cap = cand[i].chunk_cells;
    ctx->acc_nodes = cand[i].acc_nodes;
    s = bz_eval_Q(ctx, f, Q, batch, flags, nullptr, stream);  // warm-up (sizes the workspace)
    if (s == BZ_OK && hipStreamSynchronize(st) != hipSuccess) s = set_err(ctx, BZ_EHIP, "sync");
    if (s == BZ_OK && hipEventRecord(e0, st) != hipSuccess) s = set_err(ctx, BZ_EHIP, "event record");
    for (int r = 0; r < reps && s == BZ_OK; ++r) s = bz_eval_Q(ctx, f, Q, batch, flags, nullptr, stream);
    if (s == BZ_OK && hipEventRecord(e1, st) != hipSuccess) s = set_err(ctx, BZ_EHIP, "event record");
    float ms = 0.f;
    if (s == BZ_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      s = set_err(ctx, BZ_EHIP, "event timing");
    report->plan[i] = cand[i];
    report->ms[i] = ms / reps;
    if (s == BZ_OK && (best < 0 || report->ms[i] < report->ms[best])) best = (int)i;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(Q);
  if (s != BZ_OK || best < 0) {
    ctx->pair_waves = saved.pair_waves;
    ctx->chunk_cap = saved.chunk_cells;
    ctx->acc_nodes = saved.acc_nodes;
    return s != BZ_OK ? s : set_err(ctx, BZ_EHIP, "no candidate ran");
  }
  report->n = (int)cand.size();
  report->best = best;
  ctx->pair_waves = cand[best].pair_waves;
  ctx->chunk_cap = cand[best].chunk_cells;
  ctx->acc_nodes = cand[best].acc_nodes;
  std::lock_guard<std::mutex> lock(g_mu);
  g_cache[key_of(ctx, flags)] = cand[best];
  return BZ_OK;
}

}  // extern "C"
