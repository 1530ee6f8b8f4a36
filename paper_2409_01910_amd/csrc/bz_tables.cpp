// Host-built quadrature, phase and spectral weight tables (FP64), uploaded
// once per context.
//
// Fourier spectral collision operator (Section 2.2, eq. collision with the
// relative speed truncated at R_g = 2R, Section 4.2): with f periodic on
// [-L, L)^3, f(v) = sum_l fh_l exp(i xi_l.v), xi_l = pi l / L, and B = |g|^gamma,
//   gain  Qh+_k = sum_r W_r(|xi_k|) DFT_k[ sum_sigma w_sigma f(v + s) f(v - s) ],
//         s = rho_r sigma / 2,  W_r(z) = w_r rho_r^{gamma+2} 4 pi sinc(rho_r z / 2),
//   loss  Q- = f * IDFT[ Gm(|xi|) fh ],  Gm(z) = 4 pi sum_r w_r rho_r^{gamma+2} 4 pi sinc(rho_r z),
// with a Gauss-Legendre x uniform-azimuth sphere rule and a Gauss-Legendre
// radial rule on [0, R_g].  The shift f(v + s) is a phase exp(i xi.s) on fh;
// it separates over the three axes, which the kernels exploit.
#include <algorithm>
#include <cmath>
#include <vector>

#include "bz_internal.hpp"

namespace bz {

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  // Newton's method on P_n from the Tricomi-type initial guess; nodes ascending.
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) {
        p1 = z;
        p0 = 1.0;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  // enforce exact antipodal symmetry of the rule
  for (int i = 0; i < n / 2; ++i) {
    const double a = 0.5 * (x[n - 1 - i] - x[i]);
    const double b = 0.5 * (w[n - 1 - i] + w[i]);
    x[i] = -a;
    x[n - 1 - i] = a;
    w[i] = w[n - 1 - i] = b;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

static double sinc(double z) { return z == 0.0 ? 1.0 : std::sin(z) / z; }

template <typename D, typename S>
static bz_status upload(bz_ctx* ctx, D** dst, const std::vector<S>& src) {
  std::vector<D> tmp(src.begin(), src.end());
  BZ_HIP(hipMalloc((void**)dst, tmp.size() * sizeof(D)));
  BZ_HIP(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(D), hipMemcpyHostToDevice));
  return BZ_OK;
}

// Carleman form of the hard-sphere operator: per direction e_p of the half
// sphere (the sigma rule's nodes with cos(theta) > 0, weight w_p), the tables
//   A_p(xi) = 4 w_p psi1(xi.e_p),  psi1(s) = 2 int_0^Rc rho cos(rho s) drho,
//   B_p(xi) = Phi2(|P_{e_p} xi|),  Phi2(t) = 2 pi Rc J1(Rc t) / t,
// with Rc = sqrt(2) R (R the support radius: the truncation of x and y that the
// cited fast spectral construction keeps free of aliasing on [-L, L]^3 when
// L = (3 sqrt 2 + 1) R / 2), and the loss weight beta = sum_p A_p B_p.
static double carleman_psi1(double Rc, double s) {
  const double x = Rc * s;
  double v;
  if (std::fabs(x) < 0.5) {
    // (x sin x + cos x - 1) / x^2 = sum_n (-1)^n x^{2n} (2n + 1) / (2n + 2)!
    double fact = 2.0, xp = 1.0;
    v = 0.0;
    for (int n = 0; n < 12; ++n) {
      if (n > 0) {
        fact *= (2.0 * n + 1.0) * (2.0 * n + 2.0);
        xp *= -x * x;
      }
      v += xp * (2.0 * n + 1.0) / fact;
    }
  } else {
    v = (x * std::sin(x) + std::cos(x) - 1.0) / (x * x);
  }
  return 2.0 * Rc * Rc * v;
}

static double carleman_phi2(double Rc, double t) {
  const double x = Rc * t;
  const double v = x > 1e-12 ? std::cyl_bessel_j(1.0, x) / x : 0.5;
  return 2.0 * M_PI * Rc * Rc * v;
}

static bz_status build_carleman_tables(bz_ctx* ctx, const std::vector<double>& ct, const std::vector<double>& wt,
                                       const std::vector<double>& xi) {
  const int N = ctx->N, K = ctx->K, nt = ctx->n_theta, np = ctx->n_phi;
  const double Rc = std::sqrt(2.0) * ctx->R;
  const int nd = (nt / 2) * np;
  std::vector<double> cw((size_t)nd * 2 * K), beta(K, 0.0);
  int p = 0;
  for (int t = nt / 2; t < nt; ++t) {  // Gauss-Legendre nodes ascending: cos(theta) > 0
    const double c = ct[t], st = std::sqrt(std::max(0.0, 1.0 - c * c));
    for (int j = 0; j < np; ++j, ++p) {
      const double ph = 2.0 * M_PI * j / np;
      const double e0 = c, e1 = st * std::cos(ph), e2 = st * std::sin(ph);
      const double wp = wt[t] * 2.0 * M_PI / np;
      double* A = cw.data() + (size_t)p * 2 * K;
      double* B = A + K;
      for (int l1 = 0; l1 < N; ++l1)
        for (int l2 = 0; l2 < N; ++l2)
          for (int l3 = 0; l3 < N; ++l3) {
            const size_t k = ((size_t)l1 * N + l2) * N + l3;
            const double s = xi[l1] * e0 + xi[l2] * e1 + xi[l3] * e2;
            const double x2 = xi[l1] * xi[l1] + xi[l2] * xi[l2] + xi[l3] * xi[l3];
            A[k] = 4.0 * wp * carleman_psi1(Rc, s);
            B[k] = carleman_phi2(Rc, std::sqrt(std::max(0.0, x2 - s * s)));
            beta[k] += A[k] * B[k];
          }
    }
  }
  bz_status s;
  if ((s = upload(ctx, &ctx->d_cw, cw)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_cbeta, beta)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_cw_f, cw)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_cbeta_f, beta)) != BZ_OK) return s;
  ctx->n_dir = nd;
  return BZ_OK;
}

bz_status build_tables(bz_ctx* ctx) {
  if (ctx->d == 2) return build_tables_v2(ctx);
  if (ctx->d == 1) {  // the BGK slab needs the nodes only
    ctx->h_nodes.resize(ctx->N);
    for (int i = 0; i < ctx->N; ++i) ctx->h_nodes[i] = (i - ctx->N / 2 + 1) * ctx->dv;
    return upload(ctx, &ctx->d_nodes, ctx->h_nodes);
  }
  const int N = ctx->N, K = ctx->K, nt = ctx->n_theta, np = ctx->n_phi, nr = ctx->n_rho;
  const double L = ctx->p.L, gam = ctx->p.gamma;
  std::vector<double> ct, wt, rr, wr;
  gauss_legendre(nt, ct, wt);
  gauss_legendre(nr, rr, wr);
  for (int i = 0; i < nr; ++i) {  // map [-1, 1] -> [0, R_g]
    rr[i] = 0.5 * ctx->Rg * (rr[i] + 1.0);
    wr[i] = 0.5 * ctx->Rg * wr[i];
  }
  std::vector<double> xi(N);
  for (int l = 0; l < N; ++l) xi[l] = M_PI * (l < N / 2 ? l : l - N) / L;
  ctx->h_nodes.resize(N);
  for (int i = 0; i < N; ++i) ctx->h_nodes[i] = (i - N / 2 + 1) * ctx->dv;

  // z-stage phases exp(i xi_l rho_r c_t / 2)
  std::vector<double> ph1((size_t)nr * nt * N * 2);
  for (int r = 0; r < nr; ++r)
    for (int t = 0; t < nt; ++t)
      for (int l = 0; l < N; ++l) {
        const double a = xi[l] * rr[r] * ct[t] / 2.0;
        const size_t o = (((size_t)r * nt + t) * N + l) * 2;
        ph1[o] = std::cos(a);
        ph1[o + 1] = std::sin(a);
      }
  // pair q = tp * n_phi + j: theta node t = nt/2 + tp (c_t > 0), azimuth 2 pi j / n_phi;
  // its antipode is (nt - 1 - t, j + n_phi / 2).
  const int npairs = (nt / 2) * np;
  ctx->h_pair_w.resize(npairs);
  std::vector<double> ph23((size_t)nr * npairs * 2 * N * 2);
  for (int tp = 0; tp < nt / 2; ++tp) {
    const int t = nt / 2 + tp;
    const double st = std::sqrt(std::max(0.0, 1.0 - ct[t] * ct[t]));
    for (int j = 0; j < np; ++j) {
      const int q = tp * np + j;
      const double ph = 2.0 * M_PI * j / np;
      ctx->h_pair_w[q] = wt[t] * 2.0 * M_PI / np;
      const double s2 = st * std::cos(ph), s3 = st * std::sin(ph);
      for (int r = 0; r < nr; ++r)
        for (int l = 0; l < N; ++l) {
          const double a2 = xi[l] * rr[r] * s2 / 2.0, a3 = xi[l] * rr[r] * s3 / 2.0;
          const size_t o = ((((size_t)r * npairs + q) * 2 + 0) * N + l) * 2;
          const size_t o3 = ((((size_t)r * npairs + q) * 2 + 1) * N + l) * 2;
          ph23[o] = std::cos(a2);
          ph23[o + 1] = std::sin(a2);
          ph23[o3] = std::cos(a3);
          ph23[o3 + 1] = std::sin(a3);
        }
    }
  }
  // radial gain weights (with the 1/K of the forward transform) and loss weight
  std::vector<double> W((size_t)nr * K), Gm(K, 0.0);
  for (int l1 = 0; l1 < N; ++l1)
    for (int l2 = 0; l2 < N; ++l2)
      for (int l3 = 0; l3 < N; ++l3) {
        const size_t k = ((size_t)l1 * N + l2) * N + l3;
        const double z = std::sqrt(xi[l1] * xi[l1] + xi[l2] * xi[l2] + xi[l3] * xi[l3]);
        double g = 0.0;
        for (int r = 0; r < nr; ++r) {
          const double rad = wr[r] * std::pow(rr[r], gam + 2.0);
          W[(size_t)r * K + k] = rad * 4.0 * M_PI * sinc(rr[r] * z / 2.0) / K;
          g += rad * 4.0 * M_PI * sinc(rr[r] * z);
        }
        Gm[k] = 4.0 * M_PI * g;
      }
  bz_status s;
  if ((s = upload(ctx, &ctx->d_nodes, ctx->h_nodes)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_ph1, ph1)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_ph23, ph23)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_pairw, ctx->h_pair_w)) != BZ_OK) return s;
  std::vector<double> pair_sw(npairs);
  for (int q = 0; q < npairs; ++q) pair_sw[q] = std::sqrt(ctx->h_pair_w[q]);
  if ((s = upload(ctx, &ctx->d_pairsw, pair_sw)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_W, W)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_Gm, Gm)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_ph1_f, ph1)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_ph23_f, ph23)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_pairw_f, ctx->h_pair_w)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_pairsw_f, pair_sw)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_W_f, W)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_Gm_f, Gm)) != BZ_OK) return s;
  ctx->n_pairs = npairs;
  if (ctx->p.method == BZ_METHOD_CARLEMAN) return build_carleman_tables(ctx, ct, wt, xi);
  return BZ_OK;
}

// Two-dimensional velocity (d = 2, the velocity space of the paper's binary
// runs, Section 4.2): the same sigma form on the circle, with
//   W_r(z) = w_r rho_r^{gamma+1} 2 pi J0(rho_r z / 2),
//   Gm(z)  = 2 pi sum_r w_r rho_r^{gamma+1} 2 pi J0(rho_r z),
// the circle rule theta_p = 2 pi p / M with equal weights 2 pi / M (antipodal
// pairs p, p + M/2), and transforms of length N = 2^a 3^b by radix-4/3/2 passes.
bz_status build_tables_v2(bz_ctx* ctx) {
  const int N = ctx->N, K = ctx->K, nr = ctx->n_rho, M = ctx->n_phi;
  const double L = ctx->p.L, gam = ctx->p.gamma;
  int n = N, np = 0;
  while (n % 4 == 0 && np < 4) ctx->v2_rad[np++] = 4, n /= 4;
  while (n % 3 == 0 && np < 4) ctx->v2_rad[np++] = 3, n /= 3;
  while (n % 2 == 0 && np < 4) ctx->v2_rad[np++] = 2, n /= 2;
  if (n != 1) return set_err(ctx, BZ_EINVAL, "d = 2 needs N = 2^a 3^b with at most four radix-4/3/2 passes");
  ctx->v2_npass = np;
  std::vector<double> rr, wr;
  gauss_legendre(nr, rr, wr);
  for (int i = 0; i < nr; ++i) {
    rr[i] = 0.5 * ctx->Rg * (rr[i] + 1.0);
    wr[i] = 0.5 * ctx->Rg * wr[i];
  }
  std::vector<double> xi(N), tw(2 * N), dir(M), W((size_t)nr * K), Gm(K);
  for (int l = 0; l < N; ++l) xi[l] = M_PI * (l < N / 2 ? l : l - N) / L;
  for (int j = 0; j < N; ++j) {
    tw[2 * j] = std::cos(2.0 * M_PI * j / N);
    tw[2 * j + 1] = std::sin(2.0 * M_PI * j / N);
  }
  for (int p = 0; p < M / 2; ++p) {
    dir[2 * p] = std::cos(2.0 * M_PI * p / M);
    dir[2 * p + 1] = std::sin(2.0 * M_PI * p / M);
  }
  ctx->h_nodes.resize(N);
  for (int i = 0; i < N; ++i) ctx->h_nodes[i] = (i - N / 2 + 1) * ctx->dv;
  for (int l1 = 0; l1 < N; ++l1)
    for (int l2 = 0; l2 < N; ++l2) {
      const size_t k = (size_t)l1 * N + l2;
      const double z = std::sqrt(xi[l1] * xi[l1] + xi[l2] * xi[l2]);
      double g = 0.0;
      for (int r = 0; r < nr; ++r) {
        const double rad = wr[r] * std::pow(rr[r], gam + 1.0);
        W[(size_t)r * K + k] = rad * 2.0 * M_PI * std::cyl_bessel_j(0.0, rr[r] * z / 2.0) / K;
        g += rad * 2.0 * M_PI * std::cyl_bessel_j(0.0, rr[r] * z);
      }
      Gm[k] = 2.0 * M_PI * g;
    }
  bz_status s;
  if ((s = upload(ctx, &ctx->d_nodes, ctx->h_nodes)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_v2xi, xi)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_v2tw, tw)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_v2dir, dir)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_v2rho, rr)) != BZ_OK) return s;
  // axis phases (cos, sin)(xi_l s_a), s = rho_r sigma_p / 2, per (radial node,
  // pair, axis a, l)
  std::vector<double> ph((size_t)nr * (M / 2) * 2 * N * 2);
  for (int r = 0; r < nr; ++r)
    for (int p = 0; p < M / 2; ++p)
      for (int a = 0; a < 2; ++a)
        for (int l = 0; l < N; ++l) {
          const double t = xi[l] * (0.5 * rr[r] * dir[2 * p + a]);
          const size_t i = ((((size_t)r * (M / 2) + p) * 2 + a) * N + l) * 2;
          ph[i] = std::cos(t);
          ph[i + 1] = std::sin(t);
        }
  if ((s = upload(ctx, &ctx->d_v2ph, ph)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_W, W)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_Gm, Gm)) != BZ_OK) return s;
  if (ctx->p.method != BZ_METHOD_CARLEMAN) return BZ_OK;
  // Carleman form for Maxwell molecules: x = rho e over the half circle, y along
  // e_perp, both truncated at Rc = sqrt(2) R; psi2(s) = 2 Rc sinc(Rc s) and
  // A_p = 2 w_p psi2(xi.e_p), B_p = psi2(xi.e_p_perp), beta = sum_p A_p B_p
  const double Rc = std::sqrt(2.0) * ctx->R;
  const int nd = M / 2;
  std::vector<double> cw((size_t)nd * 2 * K), beta(K, 0.0);
  auto psi2 = [&](double t) { const double z = Rc * t; return 2.0 * Rc * (z == 0.0 ? 1.0 : std::sin(z) / z); };
  for (int p = 0; p < nd; ++p) {
    const double c = std::cos(2.0 * M_PI * p / M), sn = std::sin(2.0 * M_PI * p / M), wp = 2.0 * M_PI / M;
    for (int l1 = 0; l1 < N; ++l1)
      for (int l2 = 0; l2 < N; ++l2) {
        const size_t k = (size_t)l1 * N + l2;
        const double a = 2.0 * wp * psi2(xi[l1] * c + xi[l2] * sn);
        const double b = psi2(-xi[l1] * sn + xi[l2] * c);
        cw[((size_t)p * 2 + 0) * K + k] = a;
        cw[((size_t)p * 2 + 1) * K + k] = b;
        beta[k] += a * b;
      }
  }
  ctx->n_dir = nd;
  if ((s = upload(ctx, &ctx->d_cw, cw)) != BZ_OK) return s;
  if ((s = upload(ctx, &ctx->d_cbeta, beta)) != BZ_OK) return s;
  return BZ_OK;
}

void free_tables(bz_ctx* ctx) {
  void* ptrs[] = {ctx->d_nodes,  ctx->d_ph1,   ctx->d_ph23,     ctx->d_pairw,      ctx->d_pairsw, ctx->d_W,
                  ctx->d_Gm,     ctx->d_ph1_f, ctx->d_ph23_f,   ctx->d_pairw_f,    ctx->d_pairsw_f,
                  ctx->d_W_f,    ctx->d_Gm_f,   ctx->d_cw,       ctx->d_cbeta,      ctx->d_cw_f,   ctx->d_cbeta_f,
                  ctx->d_v2tw,   ctx->d_v2xi,   ctx->d_v2dir,    ctx->d_v2rho,      ctx->d_v2ph};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
}

}  // namespace bz
