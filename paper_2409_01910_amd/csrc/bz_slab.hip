// 1D slab sweeps (placeholder until the SGS driver lands).
#include "bz_internal.hpp"

extern "C" {
struct bz_slab {
  int dummy;
};
bz_status bz_slab_create(bz_ctx* ctx, const bz_slab_desc*, bz_slab** out) {
  if (out) *out = nullptr;
  return bz::set_err(ctx, BZ_EUNSUPPORTED, "slab sweeps not built yet");
}
void bz_slab_destroy(bz_slab*) {}
bz_status bz_sgs_sweep(bz_ctx* ctx, bz_slab*, int, double*, bz_sweep_stats*, void*) {
  return bz::set_err(ctx, BZ_EUNSUPPORTED, "slab sweeps not built yet");
}
bz_status bz_outer_residual(bz_ctx* ctx, bz_slab*, double*, void*) {
  return bz::set_err(ctx, BZ_EUNSUPPORTED, "slab sweeps not built yet");
}
bz_status bz_multigrid_vcycle(bz_ctx* ctx, bz_slab*, const bz_mg_opts*, int, double*, bz_sweep_stats*, void*) {
  return bz::set_err(ctx, BZ_EUNSUPPORTED, "slab sweeps not built yet");
}
}
