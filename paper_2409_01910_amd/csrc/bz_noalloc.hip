// Allocation-free evaluation of the collision term, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The collision pipeline's workspace (spectra, loss transforms, z-stage planes,
// accumulators) and the per-cell Maxwellian parameters of the projections live
// in one file-scope device array of kScratchBytes per device.  Its device
// address is resolved once per device, when the first context on that device
// is created (hipGetSymbolAddress with the device current), and kept per
// device; host code uses only that address, never the array's name.  Cells are
// processed in chunks sized to the array, so any batch works as long as one
// cell's workspace fits.  Every call on a device shares that device's array:
// calls that overlap on one device (two streams, two host threads) race.
#include <mutex>

#include "bz_internal.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

namespace bz {

bz_status scratch_attach(bz_ctx* ctx) {
  const int dev = ctx->p.device;
  if (dev < 0 || dev >= kMaxDevices) return set_err(ctx, BZ_EUNSUPPORTED, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_err(ctx, e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress");
    g_ptr[dev] = p;
  }
  ctx->scratch = g_ptr[dev];
  ctx->scratch_bytes = kScratchBytes;
  return BZ_OK;
}

}  // namespace bz

extern "C" bz_status bz_eval_Q_noalloc(bz_ctx* ctx, const double* f, double* Q, int64_t batch, uint32_t flags,
                                       double* theta, void* stream) {
  bz_status s = bz::check_eval_q_args(ctx, f, Q, batch, flags, theta);
  if (s != BZ_OK || batch == 0) return s;
  if (!ctx->scratch) return bz::set_err(ctx, BZ_EHIP, "scratch address not resolved for this device");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return bz::set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const bool corrected = (flags & BZ_Q_CORRECTED) != 0;
  const bool mass = (flags & BZ_Q_MASS) != 0, conserve = (flags & BZ_Q_CONSERVE) != 0;
  const int d = ctx->d, np = d + 2;
  const size_t K = (size_t)ctx->K;
  // scratch per cell: the collision workspace (d = 3; the 2D kernels work in
  // LDS) and, when the caller passes no theta but the call needs it, the
  // Maxwellian parameters
  const bool need_th = !theta && ((d == 3 && (mass || conserve)) || (d == 2 && corrected));
  const size_t per_th = need_th ? (size_t)np * sizeof(double) : 0;
  const size_t per_ws = d == 3 ? bz::eval_q_ws_per_cell(ctx, corrected) : 0;
  const size_t per = per_th + per_ws;
  const size_t room = ctx->scratch_bytes - 256;
  if (per > room)
    return bz::set_err(ctx, BZ_EINVAL,
                       "one cell needs " + std::to_string(per) + " bytes of scratch; the allocation-free entry point "
                       "holds " + std::to_string(ctx->scratch_bytes) + " (use bz_eval_Q)");
  const int64_t chunk = per == 0 ? batch : (int64_t)(room / per);
  unsigned char* base = (unsigned char*)ctx->scratch;
  for (int64_t c0 = 0; c0 < batch; c0 += chunk) {
    const int64_t B = (batch - c0) < chunk ? (batch - c0) : chunk;
    double* th = theta ? theta + c0 * np : (need_th ? (double*)base : nullptr);
    unsigned char* ws = base + align256((size_t)B * per_th);
    const size_t ws_bytes = ctx->scratch_bytes - align256((size_t)B * per_th);
    const double* fb = f + c0 * K;
    double* Qb = Q + c0 * K;
    if (d == 2) {
      s = bz::v2_eval_q(ctx, fb, Qb, B, corrected, mass, th, st, ws, ws_bytes);
    } else {
      s = bz::eval_q(ctx, fb, Qb, B, corrected, th, st, ws, ws_bytes);
      if (s == BZ_OK && mass) s = bz::mass_project(ctx, Qb, th, B, st);
      if (s == BZ_OK && conserve) s = bz::conserve_project(ctx, Qb, th, B, st);
    }
    if (s != BZ_OK) return s;
  }
  return BZ_OK;
}
