// Batched Fourier-spectral collision operator on gfx950.
//
// Pipeline for a chunk of cells (T = double or float for the spectral stage):
//   prep      moments + discrete Maxwellian (FP64 Newton) ; fields g = f - M,
//             h = f + M (corrected form) or f (plain form)
//   fft3      forward transform of the fields, 1/K scaling, Nyquist modes zeroed
//   loss      L[u] = IDFT(Gm * DFT u)                   (loss term of the operator)
//   per radial node r:
//     zstage  axis-0 inverse transform with the phase exp(i xi_1 s_1) for every
//             polar node: shared by all azimuths of that node (at N = 32 only
//             the half of each Hermitian plane with l2 < N/2 is stored)
//     pairs   for every antipodal direction pair (sigma, -sigma): axis-1/axis-2
//             inverse transforms with the remaining phases, giving
//             c = A(v + s) + i B(v - s) in one complex transform; accumulate
//             w Re(c) Im(c) in physical space; then 2D forward transform of the
//             accumulated plane, held with those of the other radial nodes
//   colw      per group of held radial nodes: axis-0 forward transform of each
//             node's planes, multiply by W_r(|xi|), add into Qh+
//   final     inverse transform of Qh+, Q = Q+ - loss (FP64 combine)
// The corrected form (eq. discrete_Q), Q^FSM[f,f] - Q^FSM[M,M], is evaluated
//   * with an FP32 spectral stage as the symmetric bilinear form Q_s(g, h),
//     g = f - M, h = f + M: gain pairs g(v+s) h(v-s) + g(v-s) h(v+s), loss
//     (g L[h] + h L[g]) / 2, equal up to rounding and free of the cancellation
//     that FP32 would not survive;
//   * in FP64 as the difference itself: Q^FSM[f,f] through the pipeline above
//     (one field, half the direction-pair work of the bilinear form) minus
//     Q^FSM[M,M], whose gain is computed from 1D transforms: M is a sampled
//     Gaussian, so its spectrum, every shifted copy M(v +- s) and their
//     products factorise over the three axes (k_max_sep1, k_max_sep2); its
//     loss goes through the same loss transform as f's.
#include "bz_common.hpp"
#include "bz_internal.hpp"
#include "bz_newton.hpp"

namespace bz {

template <typename T>
struct V2;
template <>
struct V2<double> {
  using type = double2;
};
template <>
struct V2<float> {
  using type = float2;
};

constexpr int kPrepThreads = 256;

// ------------------------------------------------------------------ prep
template <typename T, int N>
__global__ __launch_bounds__(kPrepThreads) void k_prep(const double* __restrict__ f, double* __restrict__ GH,
                                                       typename V2<T>::type* __restrict__ Fc,
                                                       double* __restrict__ theta_out, const double* __restrict__ nodes,
                                                       double w, int corrected, double* __restrict__ scale) {
  using C = typename V2<T>::type;
  constexpr int K = N * N * N;
  const int b = blockIdx.x;
  const double* fb = f + (size_t)b * K;
  __shared__ double s_red[5 * (kPrepThreads / 64)];
  __shared__ double s_nodes[N];
  __shared__ double s_E[3][N];
  __shared__ double s_th[5];
  if (threadIdx.x < N) s_nodes[threadIdx.x] = nodes[threadIdx.x];
  __syncthreads();
  if (!corrected) {
    C* out = Fc + (size_t)b * K;
    for (int k = threadIdx.x; k < K; k += blockDim.x) out[k] = C{T(fb[k]), T(0)};
    return;
  }
  double m[5] = {0, 0, 0, 0, 0};
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double v0 = s_nodes[k / (N * N)], v1 = s_nodes[(k / N) % N], v2 = s_nodes[k % N];
    const double fk = fb[k];
    m[0] += fk;
    m[1] += fk * v0;
    m[2] += fk * v1;
    m[3] += fk * v2;
    m[4] += fk * (v0 * v0 + v1 * v1 + v2 * v2);
  }
  block_sum<5>(m, s_red);
  if (threadIdx.x < 64) {
    double tgt[5], th[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) tgt[i] = w * m[i];
    theta_from_moments(tgt, w, th);
    AxisW aw{W_ONE, 0.0, 0.0, 0.0};
    newton_gauss(s_nodes, N, w, tgt, th, aw, 1e-13, 60);
    if (threadIdx.x < 5) s_th[threadIdx.x] = th[threadIdx.x];
  }
  __syncthreads();
  if (threadIdx.x < 3 * N) {
    const int a = threadIdx.x / N, i = threadIdx.x % N;
    const double x = s_nodes[i];
    s_E[a][i] = exp(s_th[1 + a] * x - s_th[4] * x * x);
  }
  if (theta_out && threadIdx.x < 5) theta_out[(size_t)b * 5 + threadIdx.x] = s_th[threadIdx.x];
  __syncthreads();
  const double ea = exp(s_th[0]);
  if (corrected == 2) {
    // difference form: f and M packed as f + i M in volume b (both real, so one
    // complex transform carries both spectra); GH keeps M
    double* Mb = GH + (size_t)b * K;
    C* Ff = Fc + (size_t)b * K;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
      const double M = ea * s_E[0][k / (N * N)] * s_E[1][(k / N) % N] * s_E[2][k % N];
      Mb[k] = M;
      Ff[k] = C{T(fb[k]), T(M)};
    }
    return;
  }
  // bilinear form: g = f - M and h = f + M.  The direction stage carries g and h
  // as the two parts of one complex transform, whose rounding is relative to
  // the larger part; g enters the transforms scaled by the power of two that
  // brings it to h's magnitude (exact in any precision), so that its rounding
  // error scales with g itself.  The combine divides the scale out again.
  double* g = GH + (size_t)b * 2 * K;
  double* h = g + K;
  C* Fg = Fc + (size_t)b * 2 * K;
  C* Fh = Fg + K;
  // (the first pass only finds the maxima; the second recomputes M, which
  // costs less than reading back stored fields)
  double gm = 0.0, hm = 0.0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double M = ea * s_E[0][k / (N * N)] * s_E[1][(k / N) % N] * s_E[2][k % N];
    gm = fmax(gm, fabs(fb[k] - M));
    hm = fmax(hm, fabs(fb[k] + M));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    gm = fmax(gm, __shfl_xor(gm, off, 64));
    hm = fmax(hm, __shfl_xor(hm, off, 64));
  }
  const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_red[wid] = gm;
    s_red[nw + wid] = hm;
  }
  __syncthreads();
  gm = 0.0;
  hm = 0.0;
  for (int i = 0; i < nw; ++i) {
    gm = fmax(gm, s_red[i]);
    hm = fmax(hm, s_red[nw + i]);
  }
  int e = (gm > 0.0 && hm > gm) ? ilogb(hm) - ilogb(gm) : 0;
  e = e < 60 ? e : 60;
  const double sc = ldexp(1.0, e);
  if (threadIdx.x == 0) scale[b] = sc;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double M = ea * s_E[0][k / (N * N)] * s_E[1][(k / N) % N] * s_E[2][k % N];
    const double gk = fb[k] - M, hk = fb[k] + M;
    g[k] = gk;
    h[k] = hk;
    Fg[k] = C{T(sc * gk), T(0)};
    Fh[k] = C{T(hk), T(0)};
  }
}

// ------------------------------------------------------------------ plane FFT (axes 1, 2)
template <typename T, int N>
constexpr int plane_ppb() {
  return (N >= 32) ? (sizeof(T) == 8 ? 4 : 8) : (N == 16 ? 8 : 16);
}

template <typename T, int N, int SIGN>
__global__ __launch_bounds__((N * plane_ppb<T, N>())) void k_plane(const typename V2<T>::type* __restrict__ in,
                                                                typename V2<T>::type* __restrict__ out,
                                                                int64_t nplanes) {
  using C = typename V2<T>::type;
  constexpr int PPB = plane_ppb<T, N>();
  constexpr int NT = N * PPB;
  constexpr int LD = N + 1;
  __shared__ C s[PPB * N * LD];
  const int64_t p0 = (int64_t)blockIdx.x * PPB;
  const int np = (int)((nplanes - p0) < PPB ? (nplanes - p0) : PPB);
  const C* src = in + p0 * N * N;
  for (int e = threadIdx.x; e < np * N * N; e += NT) {
    const int p = e / (N * N), rr = (e / N) % N, cc = e % N;
    s[(p * N + rr) * LD + cc] = src[e];
  }
  __syncthreads();
  const int p = threadIdx.x / N, q = threadIdx.x % N;
  T re[N], im[N];
  if (p < np) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const C v = s[(p * N + q) * LD + j];
      re[j] = v.x;
      im[j] = v.y;
    }
    fft_reg<T, N, SIGN>(re, im);
#pragma unroll
    for (int j = 0; j < N; ++j) s[(p * N + q) * LD + j] = C{re[j], im[j]};
  }
  __syncthreads();
  if (p < np) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const C v = s[(p * N + j) * LD + q];
      re[j] = v.x;
      im[j] = v.y;
    }
    fft_reg<T, N, SIGN>(re, im);
    C* dst = out + (p0 + p) * N * N;
#pragma unroll
    for (int j = 0; j < N; ++j) dst[j * N + q] = C{re[j], im[j]};
  }
}

// ------------------------------------------------------------------ column FFT (axis 0)
enum ColMode { COL_PLAIN = 0, COL_FWD_NYQ = 1, COL_PREMUL = 2 };

template <typename T, int N, int SIGN, int MODE>
__global__ __launch_bounds__(256) void k_col(const typename V2<T>::type* __restrict__ in,
                                             typename V2<T>::type* __restrict__ out, int64_t nvol,
                                             const T* __restrict__ wt) {
  using C = typename V2<T>::type;
  constexpr int K = N * N * N, NN = N * N;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nvol * NN) return;
  const int64_t vol = gid / NN;
  const int c = (int)(gid % NN);
  const C* src = in + vol * K + c;
  T re[N], im[N];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    C v = src[(size_t)l * NN];
    if (MODE == COL_PREMUL) {
      const T g = wt[(size_t)l * NN + c];
      v.x *= g;
      v.y *= g;
    }
    re[l] = v.x;
    im[l] = v.y;
  }
  fft_reg<T, N, SIGN>(re, im);
  C* dst = out + vol * K + c;
  if (MODE == COL_FWD_NYQ) {
    const T sc = T(1.0 / K);
    const bool zero_all = (c / N == N / 2) || (c % N == N / 2);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const bool z = zero_all || l == N / 2;
      dst[(size_t)l * NN] = z ? C{T(0), T(0)} : C{re[l] * sc, im[l] * sc};
    }
  } else {
#pragma unroll
    for (int l = 0; l < N; ++l) dst[(size_t)l * NN] = C{re[l], im[l]};
  }
}

// ------------------------------------------------------------------ z-stage
// Z[b][fld][t][i1][l2][l3] = sum_l1 F[b][fld][l1][l2][l3] exp(i xi_l1 s1_t) e^{2 pi i l1 i1 / N}
// A plane (b, fld, t, i1) is Hermitian in (l2, l3): the fields are real, their
// spectra zero at every Nyquist index, and xi_{-l} = -xi_l, so
// Z(l2, l3) = conj Z(-l2, -l3) and the row l2 = N/2 is zero.  With HALF the
// z-stage computes and stores rows l2 < N/2 only ([b][fld][t][i1][N/2][N]),
// and the pair kernel reads the other rows as mirrored conjugates.
template <int N, bool HALF>
constexpr int zplane() {
  return HALF ? N * N / 2 : N * N;
}

template <typename T, int N, bool HALF>
__global__ __launch_bounds__(256) void k_zstage(const typename V2<T>::type* __restrict__ F,
                                                typename V2<T>::type* __restrict__ Z, int64_t nvol, int n_theta,
                                                const typename V2<T>::type* __restrict__ ph1) {
  using C = typename V2<T>::type;
  constexpr int K = N * N * N, NN = N * N, PL = zplane<N, HALF>();
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nvol * PL) return;
  const int64_t vol = gid / PL;  // vol = b * nf + fld
  const int c = (int)(gid % PL);  // (l2, l3), l2 < N/2 with HALF
  T xr[N], xi[N];
  const C* src = F + vol * K + c;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    const C v = src[(size_t)l * NN];
    xr[l] = v.x;
    xi[l] = v.y;
  }
  for (int t = 0; t < n_theta; ++t) {
    T re[N], im[N];
    const C* ph = ph1 + (size_t)t * N;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const C p = ph[l];
      re[l] = xr[l] * p.x - xi[l] * p.y;
      im[l] = xr[l] * p.y + xi[l] * p.x;
    }
    fft_reg<T, N, +1>(re, im);
    C* dst = Z + (vol * n_theta + t) * (N * PL) + c;
#pragma unroll
    for (int l = 0; l < N; ++l) dst[(size_t)l * PL] = C{re[l], im[l]};
  }
}

// f's spectrum from the packed spectrum Z = fhat + i Mhat of the difference
// form (both Hermitian): fhat(l) = (Z(l) + conj Z(-l)) / 2, for the columns
// the z-stage reads (rows l2 < N/2 with HALF); volumes [b][K] in and out
template <typename T, int N, bool HALF>
__global__ __launch_bounds__(256) void k_unpack(const typename V2<T>::type* __restrict__ Zp,
                                                typename V2<T>::type* __restrict__ Fu, int64_t nb) {
  using C = typename V2<T>::type;
  constexpr int K = N * N * N, NN = N * N, PL = zplane<N, HALF>();
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nb * N * PL) return;
  const int64_t b = gid / (N * PL);
  const int rem = (int)(gid % (N * PL)), l1 = rem / PL, c = rem % PL, l2 = c / N, l3 = c % N;
  const int k = l1 * NN + c;
  const int km = ((N - l1) & (N - 1)) * NN + ((N - l2) & (N - 1)) * N + ((N - l3) & (N - 1));
  const C a = Zp[b * K + k], m = Zp[b * K + km];
  Fu[b * K + k] = C{T(0.5) * (a.x + m.x), T(0.5) * (a.y - m.y)};
}

// ------------------------------------------------------------------ direction pairs (hot loop)
constexpr int kPairWaves = 4;

template <typename T, int N>
constexpr size_t pairs_lds_bytes() {
  return (size_t)kPairWaves * (64 / N) * N * (N + 1) * sizeof(typename V2<T>::type) + (size_t)N * N * sizeof(T);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int N, int NF>
__global__ __launch_bounds__(64 * kPairWaves) void k_pairs(const typename V2<T>::type* __restrict__ Z,
                                                           typename V2<T>::type* __restrict__ Acc, int n_theta,
                                                           int n_phi, const typename V2<T>::type* __restrict__ ph23,
                                                           const T* __restrict__ pairw) {
  using C = typename V2<T>::type;
  constexpr int K = N * N * N, NN = N * N, SPW = 64 / N, LD = N + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  C* trans = reinterpret_cast<C*>(smem);
  T* red = reinterpret_cast<T*>(smem + (size_t)kPairWaves * SPW * N * LD * sizeof(C));
  const int b = blockIdx.x / N, i1 = blockIdx.x % N;
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const int s = ln / N, q = ln % N;
  C* tw = trans + (size_t)(wv * SPW + s) * N * LD;
  T acc[N];
#pragma unroll
  for (int j = 0; j < N; ++j) acc[j] = T(0);
  const int half = n_theta / 2;
  const int J = NF * n_phi;
  const int rounds = (J + SPW - 1) / SPW;
  const int v = s % NF;
  // with fewer polar pairs than waves, the rounds of a polar pair are split over
  // S waves; the per-wave accumulators are summed below
  const int S = half < kPairWaves ? kPairWaves / half : 1;
  for (int u = wv; u < half * S; u += kPairWaves) {
    const int tp = u / S, sub = u % S;
    const int tA = half + tp, tB = half - 1 - tp;
    // A(v + s) and B(v - s): plain form uses f for both; corrected variant 0 is
    // g(v + s), h(v - s), variant 1 is g(v - s), h(v + s).
    const int thA = (v == 0) ? tA : tB, thB = (v == 0) ? tB : tA;
    const int fA = 0, fB = NF - 1;
    const C* za = Z + (((size_t)b * NF + fA) * n_theta + thA) * K + (size_t)i1 * NN + q;
    const C* zb = Z + (((size_t)b * NF + fB) * n_theta + thB) * K + (size_t)i1 * NN + q;
    // a + i b with a = A P, b = B conj(P) (P carrying the sign sA) is
    // Re = Pr (Ar - Bi) + Pi (Br - Ai), Im = Pr (Ai + Br) + Pi (Ar + Bi)
    T u1[N], u2[N], u3[N], u4[N];
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const C x = za[(size_t)l * N], y = zb[(size_t)l * N];
      u1[l] = x.x - y.y;
      u2[l] = y.x - x.y;
      u3[l] = x.y + y.x;
      u4[l] = x.x + y.y;
    }
    const T sA = (v == 0) ? T(1) : T(-1);  // A uses P (v = 0) or conj(P) (v = 1)
    for (int rd = sub; rd < rounds; rd += S) {
      const int j = rd * SPW + s;
      const bool active = j < J;
      const int pq = tp * n_phi + (active ? j / NF : 0);
      T re[N], im[N];
      if (active) {
        const C* p2 = ph23 + (size_t)pq * 2 * N;
        const C p3 = p2[N + q];
        const T sp3x = sA * p3.x, sp3y = sA * p3.y;
#pragma unroll
        for (int l = 0; l < N; ++l) {
          const C a2 = p2[l];
          const T Pr = a2.x * p3.x - a2.y * p3.y;
          const T Pi = a2.x * sp3y + a2.y * sp3x;
          re[l] = Pr * u1[l] + Pi * u2[l];
          im[l] = Pr * u3[l] + Pi * u4[l];
        }
        fft_reg<T, N, +1>(re, im);  // along axis 1
#pragma unroll
        for (int l = 0; l < N; ++l) tw[l * LD + q] = C{re[l], im[l]};
      }
      wave_sync();
      if (active) {
#pragma unroll
        for (int l = 0; l < N; ++l) {
          const C x = tw[q * LD + l];
          re[l] = x.x;
          im[l] = x.y;
        }
        fft_reg<T, N, +1>(re, im);  // along axis 2
        const T wgt = pairw[pq] * T(NF == 1 ? 2 : 1);
#pragma unroll
        for (int l = 0; l < N; ++l) acc[l] += wgt * re[l] * im[l];
      }
      wave_sync();
    }
  }
  // sum slots of the wave: lanes q, q + N, ... hold partial rows of row q
#pragma unroll
  for (int off = N; off < 64; off <<= 1)
#pragma unroll
    for (int l = 0; l < N; ++l) acc[l] += __shfl_xor(acc[l], off, 64);
  for (int w2 = 0; w2 < kPairWaves; ++w2) {
    if (wv == w2 && ln < N) {
#pragma unroll
      for (int l = 0; l < N; ++l) red[q * N + l] = (w2 == 0 ? T(0) : red[q * N + l]) + acc[l];
    }
    __syncthreads();
  }
  // forward 2D transform of the accumulated real plane (axes 1 and 2)
  if (threadIdx.x < N) {
    const int row = threadIdx.x;
    T re[N], im[N];
#pragma unroll
    for (int l = 0; l < N; ++l) {
      re[l] = red[row * N + l];
      im[l] = T(0);
    }
    fft_reg<T, N, -1>(re, im);
#pragma unroll
    for (int l = 0; l < N; ++l) trans[row * LD + l] = C{re[l], im[l]};
  }
  __syncthreads();
  if (threadIdx.x < N) {
    const int col = threadIdx.x;
    T re[N], im[N];
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const C x = trans[l * LD + col];
      re[l] = x.x;
      im[l] = x.y;
    }
    fft_reg<T, N, -1>(re, im);
    C* dst = Acc + (size_t)b * K + (size_t)i1 * NN + col;
#pragma unroll
    for (int l = 0; l < N; ++l) dst[(size_t)l * N] = C{re[l], im[l]};
  }
}

// ------------------------------------------------------------------ direction pairs, N = 32
// Same computation as k_pairs.  A wave owns one (polar pair, variant) item -
// for the plain form the second index splits the azimuths by parity instead -
// keeps the item's four per-entry sums in registers and runs its azimuths.
// The 32x32 inverse transform of one azimuth is done in three register stages
// of 16 values per lane, joined by two exchanges through the wave's LDS tile:
//   stage 1, lane (q, h): column i3 = q, entries i2 = 2m + h.  Phase products,
//            then the 16-point transform over m: the even (h = 0) or odd
//            (h = 1) half of a radix-2 decimation in time along axis 2.
//   stage 2, lane (k, c): the radix-2 step of axis 2, E + W^k O and
//            E - W^k O for rows k and k + 16, at columns i3 = c + 4j; then
//            8-point transforms over j (axis 3 split as 4 x 8 in time).
//   stage 3, lane (rg, k'): rows i2 = rg + 8g; the twiddles W^(c k') and
//            4-point transforms over c give columns i3 = k' + 8t.
// No stage moves data between lanes by lane permutes, and no lane computes a
// twiddle it does not use.
// Waves per block of the N = 32 pair kernel: a block is one (cell, plane) and
// its waves share the plane's items; W = 8 holds one block per CU (the FP64
// kernel fills the register file at two waves per SIMD), W = 4 and W = 2 let
// two and four blocks share a CU, so that one block's loads and final
// reduction overlap another's transforms.  The choice is tuned per context.
constexpr int kPair32WaveChoices[3] = {8, 4, 2};

template <typename T>
constexpr size_t pairs32_lds_bytes(int W) {
  return (size_t)(W * 1056 + 64) * sizeof(typename V2<T>::type) + (size_t)W * 64 * 6 * sizeof(T);
}

// e^{2 pi i n / 32}, n = 0..31, for the per-lane twiddles of stages 2 and 3
constexpr Twiddle<32> kTw32{};

// The same twiddles as three-shear rotations: x e^{i a} is
//   x1 = x_r - t x_i,  im = x_i + s x1,  re = x1 - t im
// with t = tan(a / 2) = s / (1 + c) and s = sin a: three fused multiply-adds
// instead of four, as accurate as the product while |t| <= 1 (|a| <= pi / 2;
// near a = pi the intermediate x1 grows like t and the error with it).
// n = 16 (a = pi) has no finite t and is never used.
struct Shear32 {
  double t[32];
  constexpr Shear32() : t() {
    for (int n = 0; n < 32; ++n) t[n] = n == 16 ? 0.0 : kTw32.s[n] / (1.0 + kTw32.c[n]);
  }
};
constexpr Shear32 kSh32{};

template <typename T>
__device__ __forceinline__ void srot(T& xr, T& xi, T t, T s) {
  const T x1 = xr - t * xi;
  xi = xi + s * x1;
  xr = x1 - t * xi;
}

// Slots of the wave's tile, 33 slots per row.  Every slot is a lane base plus
// a compile-time offset, so a stage's 16 accesses share one address register.
// With the lane roles of the kernel, each access pattern (a stage's writes,
// the next stage's reads) touches distinct slots modulo 8 in every 8
// consecutive lanes and modulo 16 in every 16, so 16-byte accesses spread
// over all LDS banks (checked by enumeration over all patterns).
// stage-1 output: half h, frequency k, column q
__device__ __forceinline__ int s1_slot(int h, int k, int q) { return h * 528 + k * 33 + q; }
// stage-2 output: row r, column c + 4 kp
__device__ __forceinline__ int s2_slot(int r, int c, int kp) { return r * 33 + c + 4 * kp; }
constexpr int kPair32Tile = 1056;

template <typename T>
__device__ __forceinline__ void cmul(T& xr, T& xi, T wr, T wi) {
  const T r = xr * wr - xi * wi;
  xi = xr * wi + xi * wr;
  xr = r;
}

template <typename T, int NF, int kPair32Waves>
__global__ __launch_bounds__(64 * kPair32Waves, 2) void k_pairs32(const typename V2<T>::type* __restrict__ Z,
                                                               typename V2<T>::type* __restrict__ Acc, int n_theta,
                                                               int n_phi, const typename V2<T>::type* __restrict__ ph23,
                                                               const T* __restrict__ pairsw) {
  using C = typename V2<T>::type;
  constexpr int N = 32, K = N * N * N, NN = N * N, LD = N + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  C* tiles = reinterpret_cast<C*>(smem);
  C* twl = tiles + (size_t)kPair32Waves * kPair32Tile;  // e^{2 pi i n / 32}
  C* tsh = twl + 32;                                     // (t, s) of the same as shears
  // part of the per-item sums live in LDS instead of registers (FP64 has no
  // register left for them): [wave][u1 u2 (m = 15) | u3 u4 (m = 15) | u1 u2
  // (m = 14)][lane], 16-byte pairs
  C* ulast = tsh + 32;
  // the waves' partial planes reuse the wave tiles once every wave is done
  T* red = reinterpret_cast<T*>(tiles);
  const int b = blockIdx.x / N, i1 = blockIdx.x % N;
  // wave index made uniform, so that per-item and per-azimuth values load once
  // per wave through the scalar unit
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), ln = threadIdx.x & 63;
  const int q = ln & 31, h = ln >> 5;     // stage 1
  const int k2 = ln & 15, c2 = ln >> 4;   // stage 2
  const int kp = (ln & 1) | ((ln >> 2) & 6), rg = ((ln >> 1) & 3) | ((ln >> 3) & 4);  // stage 3
  C* tile = tiles + (size_t)wv * kPair32Tile;
  if (threadIdx.x < 32) {
    twl[threadIdx.x] = C{T(kTw32.c[threadIdx.x]), T(kTw32.s[threadIdx.x])};
    tsh[threadIdx.x] = C{T(kSh32.t[threadIdx.x]), T(kTw32.s[threadIdx.x])};
  }
  __syncthreads();
  T acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = T(0);
  const int half = n_theta / 2;
  const int items = half * 2;
  // with fewer items than waves (small sphere rules), the azimuth loop of an
  // item is split over S waves; the per-wave accumulators are summed below
  const int S = items < kPair32Waves ? kPair32Waves / items : 1;
  for (int u = wv; u < items * S; u += kPair32Waves) {
    const int it = u / S, sub = u % S;
    const int tp = it >> 1, v = (NF == 2) ? (it & 1) : 0;
    const int tA = half + tp, tB = half - 1 - tp;
    const int thA = (v == 0) ? tA : tB, thB = (v == 0) ? tB : tA;
    // half planes (rows l2 < 16): row 2m + h above 16 is the conjugate of row
    // 32 - 2m - h at column -q, row 16 is zero
    constexpr int PL = zplane<32, true>();
    const C* za = Z + (((size_t)b * NF + 0) * n_theta + thA) * (N * PL) + (size_t)i1 * PL;
    const C* zb = Z + (((size_t)b * NF + (NF - 1)) * n_theta + thB) * (N * PL) + (size_t)i1 * PL;
    // (m < 8: row 2m + h direct; m > 8: row 32 - h - 2m at column -q; m = 8:
    // row 15 mirrored for h = 1, row 0 read and zeroed for h = 0)
    // (the mirrored entry of row 32 - h - 2m is moff - 2mN entries from the
    // direct entry of row h, for both fields)
    // the lane roles re-derived here and after the item loop from the work-item
    // id (kept opaque, so that they are not hoisted): held live across the
    // loops they cost the FP64 kernel 56 bytes of spill per lane
    int tid_i = (int)__builtin_amdgcn_workitem_id_x();
    asm volatile("" : "+v"(tid_i));
    const int hi = (tid_i >> 5) & 1, qi = tid_i & 31;
    const C* za_d = za + (hi * N + qi);
    const C* zb_d = zb + (hi * N + qi);
    const int moff = (N - 2 * hi) * N + ((N - qi) & (N - 1)) - qi;
    auto zrow = [&](const C* zd, int m) -> C {
      if (m < 8) return zd[(size_t)(2 * m) * N];
      if (m > 8) {
        const C x = zd[moff - 2 * m * N];
        return C{x.x, -x.y};
      }
      const C x = zd[h ? moff - 16 * N : 0];
      return h ? C{x.x, -x.y} : C{T(0), T(0)};
    };
    // with the phase P = Pr + i Pi, the sign sA of the item, a = A P' and
    // b = B conj(P'), P' = Pr + i sA Pi, the combined field a + i b is
    //   Re = Pr (Ar - Bi) + Pi sA (Br - Ai),   Im = Pr (Ai + Br) + Pi sA (Ar + Bi),
    // so the four sums are formed once per item and each azimuth costs two
    // FMA pairs per entry
    const T sA = (v == 0) ? T(1) : T(-1);
    T u1[16], u2[16], u3[16], u4[16];  // entries 14 (u1, u2) and 15 unused
#pragma unroll
    for (int m = 0; m < 15; ++m) {
      const C x = zrow(za_d, m), y = zrow(zb_d, m);
      if (m < 14) {
        u1[m] = x.x - y.y;
        u2[m] = sA * (y.x - x.y);
      }
      u3[m] = x.y + y.x;
      u4[m] = sA * (x.x + y.y);
    }
    C* ul = ulast + (size_t)wv * 192 + ln;
    {
      const C x = zrow(za_d, 15), y = zrow(zb_d, 15);
      ul[0] = C{x.x - y.y, sA * (y.x - x.y)};
      ul[64] = C{x.y + y.x, sA * (x.x + y.y)};
      const C x14 = zrow(za_d, 14), y14 = zrow(zb_d, 14);
      ul[128] = C{x14.x - y14.y, sA * (y14.x - x14.y)};
    }
    const int phi_step = (NF == 2) ? 1 : 2;
    const int phi0 = ((NF == 2) ? 0 : (it & 1)) + sub * phi_step;
    const int jstep = phi_step * S;
    // the column phase of the next azimuth is loaded one azimuth ahead (the
    // index is clamped, so the last load repeats a valid entry)
    C p3n = ph23[((size_t)(tp * n_phi + (phi0 < n_phi ? phi0 : 0)) * 2 + 1) * N + q];
    for (int jj = phi0; jj < n_phi; jj += jstep) {
      const int pq = tp * n_phi + jj;
      const C* p2 = ph23 + (size_t)pq * 2 * N;
      // the pair weight w enters as sqrt(w) on the field, so that the
      // accumulation is one FMA per entry
      const T sw = pairsw[pq] * T(NF == 1 ? 1.4142135623730950488 : 1.0);
      const T p3x = p3n.x * sw, p3y = p3n.y * sw;
      {
        const int jn = (jj + jstep < n_phi) ? jj + jstep : jj;
        p3n = ph23[((size_t)(tp * n_phi + jn) * 2 + 1) * N + q];
      }
      T re[16], im[16];
      // stage 1
      if constexpr (sizeof(T) == 8) {
        // The row phase of row i2 is z^l, l its signed frequency and z = p2[1]
        // (the table entry of frequency 1), so the phases of rows 2m + h follow
        // from P(h) and P(16 + h) by two chains of products with z^2 (error
        // growth of a few ulp over seven steps).  This replaces sixteen table
        // loads per azimuth, which the register budget would serialise.  All
        // four table entries used are the same for the whole wave.
        const C z1 = p2[1], zz = p2[2], c16 = p2[16], c17 = p2[17];
        const T a0x = h ? z1.x : T(1), a0y = h ? z1.y : T(0);  // p2[0] = 1
        const T a8x = h ? c17.x : c16.x, a8y = h ? c17.y : c16.y;
        T ar = a0x * p3x - a0y * p3y, ai = a0x * p3y + a0y * p3x;
        T br = a8x * p3x - a8y * p3y, bi = a8x * p3y + a8y * p3x;
        const C v12 = ul[0], v34 = ul[64], w12 = ul[128];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          re[m] = ar * u1[m] + ai * u2[m];
          im[m] = ar * u3[m] + ai * u4[m];
          if (m < 6) {
            re[8 + m] = br * u1[8 + m] + bi * u2[8 + m];
            im[8 + m] = br * u3[8 + m] + bi * u4[8 + m];
          } else if (m == 6) {
            re[14] = br * w12.x + bi * w12.y;
            im[14] = br * u3[14] + bi * u4[14];
          } else {
            re[15] = br * v12.x + bi * v12.y;
            im[15] = br * v34.x + bi * v34.y;
          }
          if (m < 7) {
            cmul(ar, ai, zz.x, zz.y);
            cmul(br, bi, zz.x, zz.y);
          }
        }
      } else {
        const C v12 = ul[0], v34 = ul[64], w12 = ul[128];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          const C a2 = p2[2 * m + h];
          const T Pr = a2.x * p3x - a2.y * p3y;
          const T Pi = a2.x * p3y + a2.y * p3x;
          if (m < 14) {
            re[m] = Pr * u1[m] + Pi * u2[m];
            im[m] = Pr * u3[m] + Pi * u4[m];
          } else if (m == 14) {
            re[14] = Pr * w12.x + Pi * w12.y;
            im[14] = Pr * u3[14] + Pi * u4[14];
          } else {
            re[15] = Pr * v12.x + Pi * v12.y;
            im[15] = Pr * v34.x + Pi * v34.y;
          }
        }
      }
      fft_reg<T, 16, +1>(re, im);
#pragma unroll
      for (int k = 0; k < 16; ++k) tile[s1_slot(h, k, q)] = C{re[k], im[k]};
      wave_sync();
      // stage 2: re/im[j] row ra, re/im[8 + j] row rb, column c2 + 4j, with
      // (ra, rb) = (k2, k2 + 16).  FP64 takes the twiddle W^k2 as a shear
      // rotation; for k2 > 8 the rotation is by W^(k2 + 16) = -W^k2 instead
      // (its shear ratio stays within 1) and the two rows trade places.  FP32
      // keeps the products: there the exchanged rows cost paired LDS stores.
      // (The per-lane twiddles are read from LDS each time: kept in registers
      // across the loop they would cost spills in FP64.)
      constexpr bool kShear = sizeof(T) == 8;
      const bool swap = kShear && k2 > 8;
      const int ra = swap ? k2 + 16 : k2, rb = swap ? k2 : k2 + 16;
      const C wk = kShear ? tsh[ra] : twl[k2];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const C e = tile[s1_slot(0, k2, c2 + 4 * j)], o = tile[s1_slot(1, k2, c2 + 4 * j)];
        T tr = o.x, ti = o.y;
        if (kShear)
          srot(tr, ti, wk.x, wk.y);
        else
          cmul(tr, ti, wk.x, wk.y);
        re[j] = e.x + tr;
        im[j] = e.y + ti;
        re[8 + j] = e.x - tr;
        im[8 + j] = e.y - ti;
      }
      fft_reg<T, 8, +1>(re, im);
      fft_reg<T, 8, +1>(re + 8, im + 8);
      wave_sync();
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        tile[s2_slot(ra, c2, j)] = C{re[j], im[j]};
        tile[s2_slot(rb, c2, j)] = C{re[8 + j], im[8 + j]};
      }
      wave_sync();
      // stage 3: row rg + 8g, column kp + 8t in entry 4g + t.  The twiddles
      // W^n (n = kp, 2kp, 3kp) are shear rotations within pi / 2: for
      // 8 < n < 24 the rotation by W^(n + 16) = -W^n, with the sign (sg2,
      // sg3) moved into the 4-point sums (W^kp needs none, kp < 8)
      const int n2 = 2 * kp, n3 = 3 * kp;
      const bool f2 = n2 > 8, f3 = n3 > 8;
      const T sg2 = f2 ? T(-1) : T(1), sg3 = f3 ? T(-1) : T(1);
      const C w1 = tsh[kp], w2 = tsh[f2 ? n2 + 16 : n2], w3 = tsh[f3 ? (n3 + 16) & 31 : n3];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int r = rg + 8 * g;
        const C z0 = tile[s2_slot(r, 0, kp)], z1 = tile[s2_slot(r, 1, kp)];
        const C z2 = tile[s2_slot(r, 2, kp)], z3 = tile[s2_slot(r, 3, kp)];
        T x1r = z1.x, x1i = z1.y, x2r = z2.x, x2i = z2.y, x3r = z3.x, x3i = z3.y;
        srot(x1r, x1i, w1.x, w1.y);
        srot(x2r, x2i, w2.x, w2.y);
        srot(x3r, x3i, w3.x, w3.y);
        const T ar = z0.x + sg2 * x2r, ai = z0.y + sg2 * x2i, br = z0.x - sg2 * x2r, bi = z0.y - sg2 * x2i;
        const T cr = x1r + sg3 * x3r, ci = x1i + sg3 * x3i, dr = x1r - sg3 * x3r, di = x1i - sg3 * x3i;
        re[4 * g + 0] = ar + cr;
        im[4 * g + 0] = ai + ci;
        re[4 * g + 2] = ar - cr;
        im[4 * g + 2] = ai - ci;
        re[4 * g + 1] = br - di;  // b + i d
        im[4 * g + 1] = bi + dr;
        re[4 * g + 3] = br + di;  // b - i d
        im[4 * g + 3] = bi - dr;
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) acc[k] += re[k] * im[k];
      wave_sync();
    }
  }
  // The block's plane is the sum of its waves' partial planes, then a forward
  // 2D transform (axes 1 and 2).  Each wave stores its partial plane (rows
  // padded to LD entries) over the tiles, and one wave does each transform
  // pass with two lanes per row (then per column): lane half h forms
  // u(n) = x(n) + (-1)^h x(n + 16), times w^n for h = 1, whose 16-point
  // transform is entries 2j + h.  The transposed plane sits after the partials.
  __syncthreads();  // every wave is done with its tile before the partials overwrite them
  int tid_t = (int)__builtin_amdgcn_workitem_id_x();
  asm volatile("" : "+v"(tid_t));
  const int lnt = tid_t & 63;
  const int kpt = (lnt & 1) | ((lnt >> 2) & 6), rgt = ((lnt >> 1) & 3) | ((lnt >> 3) & 4);
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int t = 0; t < 4; ++t) red[wv * (N * LD) + (rgt + 8 * g) * LD + kpt + 8 * t] = acc[4 * g + t];
  __syncthreads();
  C* trans = tiles + kPair32Waves * (N * LD) / 2;
  const int hh = lnt >> 5, lq = lnt & 31;
  const T sg = hh ? T(-1) : T(1);
  if (wv == 0) {
    // rows: real input, summed over the waves in wave order
    T re[16], im[16];
#pragma unroll
    for (int n = 0; n < 16; ++n) {
      T x0 = T(0), x1 = T(0);
      for (int w = 0; w < kPair32Waves; ++w) {
        x0 += red[w * (N * LD) + lq * LD + n];
        x1 += red[w * (N * LD) + lq * LD + n + 16];
      }
      const T u = x0 + sg * x1;
      re[n] = hh ? u * T(kTw32.c[n]) : u;
      im[n] = hh ? -u * T(kTw32.s[n]) : T(0);
    }
    fft_reg<T, 16, -1>(re, im);
#pragma unroll
    for (int j = 0; j < 16; ++j) trans[lq * LD + 2 * j + hh] = C{re[j], im[j]};
  }
  __syncthreads();
  if (wv == 0) {
    // columns
    T re[16], im[16];
#pragma unroll
    for (int n = 0; n < 16; ++n) {
      const C x0 = trans[n * LD + lq], x1 = trans[(n + 16) * LD + lq];
      const T ur = x0.x + sg * x1.x, ui = x0.y + sg * x1.y;
      const T wr = hh ? T(kTw32.c[n]) : T(1), wi = hh ? -T(kTw32.s[n]) : T(0);
      re[n] = ur * wr - ui * wi;
      im[n] = ur * wi + ui * wr;
    }
    fft_reg<T, 16, -1>(re, im);
    C* dst = Acc + (size_t)b * K + (size_t)i1 * NN + (size_t)hh * N + lq;
#pragma unroll
    for (int j = 0; j < 16; ++j) dst[(size_t)(2 * j) * N] = C{re[j], im[j]};
  }
}

// ------------------------------------------------------------------ Carleman form (hard spheres)
// Direction p of the half sphere, with the tables A_p, B_p of the context:
//   NF = 1: c = (A_p + i B_p) fh, so IDFT(c) = a_p + i b_p (A_p, B_p real and
//           even, f real: a_p and b_p are real) and the gain adds a_p b_p;
//   NF = 2: z = gh + i hh (spectra of g = f - M and h = f + M), c_A = A_p z and
//           c_B = B_p z, so IDFT(c_A) = a[g] + i a[h] and IDFT(c_B) = b[g] + i b[h];
//           the symmetric bilinear gain (a[g] b[h] + a[h] b[g]) / 2 is
//           Im(IDFT(c_A) IDFT(c_B)) / 2.
// k_ccol premultiplies and makes the axis-0 inverse transform for nd
// consecutive directions (tables tab[d][2][K]), one thread per (cell,
// direction, field, column).  D is [cell][i1][nd][NF][N][N] for k_cplane,
// which needs all planes of one (cell, i1) adjacent, and [cell][nd][NF][i1][N][N]
// for N = 32 (k_cplane32), so that a thread's 32 stores are one plane (16 KB
// in FP64) apart instead of nd * NF planes.
template <typename T, int N, int NF>
__global__ __launch_bounds__(256) void k_ccol(const typename V2<T>::type* __restrict__ Fc,
                                              typename V2<T>::type* __restrict__ D, int64_t ncells,
                                              const T* __restrict__ tab, int nd) {
  using C = typename V2<T>::type;
  constexpr int K = N * N * N, NN = N * N;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= ncells * nd * NF * NN) return;
  const int col = (int)(gid % NN);
  const int which = (int)((gid / NN) % NF);
  const int d = (int)((gid / ((int64_t)NN * NF)) % nd);
  const int64_t b = gid / ((int64_t)NN * NF * nd);
  const C* fb = Fc + (size_t)b * NF * K + col;
  const T* ta = tab + (size_t)d * 2 * K + col;
  const T* tb = ta + K;
  T re[N], im[N];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    if (NF == 1) {
      const C x = fb[(size_t)l * NN];
      const T A = ta[(size_t)l * NN], B = tb[(size_t)l * NN];
      re[l] = A * x.x - B * x.y;
      im[l] = A * x.y + B * x.x;
    } else {
      const C g = fb[(size_t)l * NN], h = fb[(size_t)K + (size_t)l * NN];
      const T wgt = which ? tb[(size_t)l * NN] : ta[(size_t)l * NN];
      re[l] = wgt * (g.x - h.y);
      im[l] = wgt * (g.y + h.x);
    }
  }
  fft_reg<T, N, +1>(re, im);
  if (N == 32) {
    C* dst = D + (((size_t)b * nd + d) * NF + which) * K + col;
#pragma unroll
    for (int l = 0; l < N; ++l) dst[(size_t)l * NN] = C{re[l], im[l]};
  } else {
    C* dst = D + (((size_t)b * N * nd + d) * NF + which) * NN + col;
#pragma unroll
    for (int l = 0; l < N; ++l) dst[(size_t)l * nd * NF * NN] = C{re[l], im[l]};
  }
}

// Axes-1/2 inverse transform of the planes of D and accumulation of the
// direction's gain into gain [cell][K] (overwritten when first != 0).  A block
// holds PPB planes (PPB even, so the two fields of one (cell, i1) stay
// together when NF = 2).
template <typename T, int N, int NF>
__global__ __launch_bounds__((N * plane_ppb<T, N>())) void k_cplane(const typename V2<T>::type* __restrict__ D,
                                                                 T* __restrict__ gain, int64_t nplanes,
                                                                 int first) {
  using C = typename V2<T>::type;
  constexpr int PPB = plane_ppb<T, N>();
  static_assert(PPB % 2 == 0, "plane pairs must not straddle blocks");
  constexpr int NT = N * PPB;
  constexpr int LD = N + 1;
  __shared__ C s[PPB * N * LD];
  const int64_t p0 = (int64_t)blockIdx.x * PPB;
  const int np = (int)((nplanes - p0) < PPB ? (nplanes - p0) : PPB);
  const C* src = D + p0 * N * N;
  for (int e = threadIdx.x; e < np * N * N; e += NT) {
    const int p = e / (N * N), rr = (e / N) % N, cc = e % N;
    s[(p * N + rr) * LD + cc] = src[e];
  }
  __syncthreads();
  const int p = threadIdx.x / N, q = threadIdx.x % N;
  T re[N], im[N];
  if (p < np) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const C v = s[(p * N + q) * LD + j];
      re[j] = v.x;
      im[j] = v.y;
    }
    fft_reg<T, N, +1>(re, im);
#pragma unroll
    for (int j = 0; j < N; ++j) s[(p * N + q) * LD + j] = C{re[j], im[j]};
  }
  __syncthreads();
  if (p < np) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const C v = s[(p * N + j) * LD + q];
      re[j] = v.x;
      im[j] = v.y;
    }
    fft_reg<T, N, +1>(re, im);
  }
  const int64_t pos = (p0 + p) / NF;  // (cell, i1) of this plane
  if (NF == 1) {
    if (p < np) {
      T* dst = gain + pos * N * N;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const T v = re[j] * im[j];
        dst[j * N + q] = first ? v : dst[j * N + q] + v;
      }
    }
  } else {
    __syncthreads();
    if (p < np) {
#pragma unroll
      for (int j = 0; j < N; ++j) s[(p * N + j) * LD + q] = C{re[j], im[j]};
    }
    __syncthreads();
    if (p < np && (p & 1) == 0) {
      T* dst = gain + pos * N * N;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const C cb = s[((p + 1) * N + j) * LD + q];
        const T v = T(0.5) * (re[j] * cb.y + im[j] * cb.x);
        dst[j * N + q] = first ? v : dst[j * N + q] + v;
      }
    }
  }
}

// Inverse 32x32 transform of one plane held by a wave, with the three
// register stages and two LDS exchanges of k_pairs32.  On entry lane (q, h) =
// (ln & 31, ln >> 5) holds column q, rows 2m + h in entry m; on return lane
// (rg, kp) holds rows rg + 8g, columns kp + 8t in entry 4g + t, with
// kp = (ln & 1) | ((ln >> 2) & 6) and rg = ((ln >> 1) & 3) | ((ln >> 3) & 4).
// tile is the wave's kPair32Tile slots, twl the 32 roots e^{2 pi i n / 32}.
template <typename T>
__device__ __forceinline__ void plane32_inverse(T (&re)[16], T (&im)[16], typename V2<T>::type* tile,
                                                const typename V2<T>::type* twl, int ln) {
  using C = typename V2<T>::type;
  const int q = ln & 31, h = ln >> 5;
  const int k2 = ln & 15, c2 = ln >> 4;
  const int kp = (ln & 1) | ((ln >> 2) & 6), rg = ((ln >> 1) & 3) | ((ln >> 3) & 4);
  fft_reg<T, 16, +1>(re, im);
#pragma unroll
  for (int k = 0; k < 16; ++k) tile[s1_slot(h, k, q)] = C{re[k], im[k]};
  wave_sync();
  const C wk = twl[k2];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const C e = tile[s1_slot(0, k2, c2 + 4 * j)], o = tile[s1_slot(1, k2, c2 + 4 * j)];
    T tr = o.x, ti = o.y;
    cmul(tr, ti, wk.x, wk.y);
    re[j] = e.x + tr;
    im[j] = e.y + ti;
    re[8 + j] = e.x - tr;
    im[8 + j] = e.y - ti;
  }
  fft_reg<T, 8, +1>(re, im);
  fft_reg<T, 8, +1>(re + 8, im + 8);
  wave_sync();
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    tile[s2_slot(k2, c2, j)] = C{re[j], im[j]};
    tile[s2_slot(k2 + 16, c2, j)] = C{re[8 + j], im[8 + j]};
  }
  wave_sync();
  const C w1 = twl[kp], w2 = twl[2 * kp], w3 = twl[3 * kp];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int r = rg + 8 * g;
    const C z0 = tile[s2_slot(r, 0, kp)], z1 = tile[s2_slot(r, 1, kp)];
    const C z2 = tile[s2_slot(r, 2, kp)], z3 = tile[s2_slot(r, 3, kp)];
    T x1r = z1.x, x1i = z1.y, x2r = z2.x, x2i = z2.y, x3r = z3.x, x3i = z3.y;
    cmul(x1r, x1i, w1.x, w1.y);
    cmul(x2r, x2i, w2.x, w2.y);
    cmul(x3r, x3i, w3.x, w3.y);
    const T ar = z0.x + x2r, ai = z0.y + x2i, br = z0.x - x2r, bi = z0.y - x2i;
    const T cr = x1r + x3r, ci = x1i + x3i, dr = x1r - x3r, di = x1i - x3i;
    re[4 * g + 0] = ar + cr;
    im[4 * g + 0] = ai + ci;
    re[4 * g + 2] = ar - cr;
    im[4 * g + 2] = ai - ci;
    re[4 * g + 1] = br - di;
    im[4 * g + 1] = bi + dr;
    re[4 * g + 3] = br + di;
    im[4 * g + 3] = bi - dr;
  }
  wave_sync();  // the tile is free again
}

// N = 32 form of k_cplane: one wave per (cell, i1), the NF planes of that
// position transformed one after the other by plane32_inverse.  Waves never
// wait for each other, and a wave's tile is 16.9 KB (FP64) instead of the
// 67.6 KB block tile of k_cplane, so several waves per SIMD stay resident.
constexpr int kCplaneWaves = 2;

template <typename T, int NF>
__global__ __launch_bounds__(64 * kCplaneWaves) void k_cplane32(const typename V2<T>::type* __restrict__ D,
                                                                T* __restrict__ gain, int64_t npos, int nd,
                                                                int first) {
  using C = typename V2<T>::type;
  constexpr int N = 32, NN = N * N;
  __shared__ C s_tiles[kCplaneWaves * kPair32Tile];
  __shared__ C s_tw[32];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  if (threadIdx.x < 32) s_tw[threadIdx.x] = C{T(kTw32.c[threadIdx.x]), T(kTw32.s[threadIdx.x])};
  __syncthreads();
  const int64_t pos = (int64_t)blockIdx.x * kCplaneWaves + wv;
  if (pos >= npos) return;  // whole waves only; no block barrier follows
  C* tile = s_tiles + wv * kPair32Tile;
  const int q = ln & 31, h = ln >> 5;
  const int kp = (ln & 1) | ((ln >> 2) & 6), rg = ((ln >> 1) & 3) | ((ln >> 3) & 4);
  T acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = T(0);
  const int64_t cell = pos / N, i1 = pos % N;
  for (int d = 0; d < nd; ++d) {
    // D is [cell][nd][NF][i1][N][N]; the second field's plane is K entries on
    const C* src = D + (((size_t)cell * nd + d) * NF * N + i1) * NN + (size_t)h * N + q;
    T re[16], im[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const C v = src[(size_t)(2 * m) * N];
      re[m] = v.x;
      im[m] = v.y;
    }
    plane32_inverse<T>(re, im, tile, s_tw, ln);
    if (NF == 1) {
#pragma unroll
      for (int k = 0; k < 16; ++k) acc[k] += re[k] * im[k];
    } else {
      T ar[16], ai[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        ar[k] = re[k];
        ai[k] = im[k];
      }
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const C v = src[(size_t)N * NN + (size_t)(2 * m) * N];
        re[m] = v.x;
        im[m] = v.y;
      }
      plane32_inverse<T>(re, im, tile, s_tw, ln);
#pragma unroll
      for (int k = 0; k < 16; ++k) acc[k] += T(0.5) * (ar[k] * im[k] + ai[k] * re[k]);
    }
  }
  T* dst = gain + (size_t)pos * NN + (size_t)rg * N + kp;
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const size_t idx = (size_t)(8 * g) * N + 8 * t;
      dst[idx] = first ? acc[4 * g + t] : dst[idx] + acc[4 * g + t];
    }
}

// Q = gain - loss, with the gain already in physical space (real).
template <typename T, int N, int NF>
__global__ __launch_bounds__(256) void k_ccombine(const double* __restrict__ f, const double* __restrict__ GH,
                                                  const T* __restrict__ gain,
                                                  const typename V2<T>::type* __restrict__ Lc, double* __restrict__ Q,
                                                  int64_t n, const double* __restrict__ scale) {
  constexpr int K = N * N * N;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n) return;
  const int64_t b = gid / K;
  const int k = (int)(gid % K);
  double loss, is = 1.0;
  if (NF == 1) {
    loss = f[gid] * double(Lc[gid].x);
  } else {
    // bilinear form: the gain and L[g] carry the power-of-two scale of g
    is = 1.0 / scale[b];
    const double g = GH[b * 2 * K + k], h = GH[b * 2 * K + K + k];
    const double Lg = double(Lc[b * 2 * K + k].x) * is, Lh = double(Lc[b * 2 * K + K + k].x);
    loss = 0.5 * (g * Lh + h * Lg);
  }
  Q[gid] = double(gain[gid]) * is - loss;
}

// ------------------------------------------------------------------ axis-0 forward + radial weight
// Qh (+)= sum over the nslot held radial nodes s of W_s * DFT_axis0(Acc_s), in
// node order, so the sum is the same as one launch per node; the accumulator
// of a column is read and written once per launch instead of once per node.
// Two lanes share a column (lanes q and q + 32 of a wave, 32 columns per
// wave), splitting the length-N transform by decimation in frequency: lane
// half h forms u(n) = x(n) + (-1)^h x(n + N/2), times w^n for h = 1, whose
// N/2-point transform is X(2j + h).  Both halves load the same addresses in
// the same instruction, so the HBM traffic is that of one lane per column.
// At N = 32 in FP64 a lane holds its 16 accumulators and all 32 loads of a
// node in flight (one wave per SIMD); bounding it to two waves spills and
// measured no faster.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_colw(const typename V2<T>::type* __restrict__ Acc,
                                              typename V2<T>::type* __restrict__ Qh, int64_t nvol,
                                              const T* __restrict__ Wr, int nslot, int64_t slot_stride, int first) {
  using C = typename V2<T>::type;
  constexpr int K = N * N * N, NN = N * N, H = N / 2;
  constexpr Twiddle<N> tw{};
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int ln = (int)(gid & 63), h = ln >> 5;
  const int64_t col = (gid >> 6) * 32 + (ln & 31);
  if (col >= nvol * NN) return;
  const int64_t vol = col / NN;
  const int c = (int)(col % NN);
  const T sg = h ? T(-1) : T(1);
  C* dst = Qh + vol * K + (size_t)h * NN + c;  // outputs k = 2j + h
  T oR[H], oI[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const C o = first ? C{T(0), T(0)} : dst[(size_t)(2 * j) * NN];
    oR[j] = o.x;
    oI[j] = o.y;
  }
  for (int s = 0; s < nslot; ++s) {
    T re[H], im[H];
    const C* src = Acc + s * slot_stride + vol * K + c;
#pragma unroll
    for (int n = 0; n < H; ++n) {
      const C x0 = src[(size_t)n * NN], x1 = src[(size_t)(n + H) * NN];
      const T ur = x0.x + sg * x1.x, ui = x0.y + sg * x1.y;
      // w^n = e^{-2 pi i n / N} on the odd half, 1 (exactly) on the even half
      const T wr = h ? T(tw.c[n]) : T(1), wi = h ? -T(tw.s[n]) : T(0);
      re[n] = ur * wr - ui * wi;
      im[n] = ur * wi + ui * wr;
    }
    fft_reg<T, H, -1>(re, im);
    const T* w = Wr + (size_t)s * K + (size_t)h * NN + c;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const T g = w[(size_t)(2 * j) * NN];
      oR[j] += g * re[j];
      oI[j] += g * im[j];
    }
  }
#pragma unroll
  for (int j = 0; j < H; ++j) dst[(size_t)(2 * j) * NN] = C{oR[j], oI[j]};
}

// ------------------------------------------------------------------ gain of the Maxwellian, separable
// For M = e^alpha E_1(v_1) E_2(v_2) E_3(v_3) the pipeline's quantities factorise:
// its normalised spectrum is e^alpha / K prod_a Ehat_a(l_a) (Ehat_a the 1D DFT
// of E_a, zero at l_a = N/2), the shifted copies of a direction pair are
// a = e^alpha / K prod_a A_a(i_a), A_a = IDFT_1(Ehat_a phase_a), b likewise
// with the conjugate phases (the antipodal polar node on axis 1), and the
// forward transform of their product is e^{2 alpha} / K^2 prod_a D_a(k_a),
// D_a = DFT_1(A_a B_a).  With the pair q = (tp, j) of polar pair tp and
// azimuth j, weight 2 w_q, the gain spectrum of M is
//   Qh_M(k) = e^{2 alpha} / K^2 sum_r W_r(k) sum_tp D0_{r,tp}(k_1) G_{r,tp}(k_2, k_3),
//   G_{r,tp}(k_2, k_3) = sum_j 2 w_q D1_{r,q}(k_2) D2_{r,q}(k_3).
// k_max_sep1 (block per cell and radial node) forms D0 and G; k_max_sep2
// (block per cell, thread per (k_2, k_3)) sums over r and tp and subtracts
// Qh_M from the cell's gain spectrum.  The length-N transforms are register
// FFTs: a wave takes one polar pair and a lane one factor vector (axis 1 of
// the polar pair, or axis 2 or 3 of one azimuth), forming A and B by one
// transform, then the transform D of their product; the G sums then use every
// thread.  A few MFLOP per cell, against the GFLOPs of the direction-pair
// transforms they replace.
constexpr int kSepThreads = 256;
constexpr int kSepWaves = kSepThreads / 64;  // polar pairs per round
constexpr int kSepJB = 16;                   // azimuths per pass

template <int N>
__global__ __launch_bounds__(kSepThreads, 2) void k_max_sep1(const double* __restrict__ theta,
                                                          const double* __restrict__ nodes,
                                                          const double2* __restrict__ ph1,
                                                          const double2* __restrict__ ph23,
                                                          const double* __restrict__ pairw, int n_rho, int n_theta,
                                                          int n_phi, double2* __restrict__ D0s,
                                                          double2* __restrict__ Gs) {
  constexpr int NN = N * N, NV = 2 * kSepJB + 1;
  constexpr int GPT = NN / kSepThreads > 0 ? NN / kSepThreads : 1;
  const int b = blockIdx.x / n_rho, r = blockIdx.x % n_rho;
  const int half = n_theta / 2, npairs = half * n_phi;
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  __shared__ double2 s_E[3][N];               // Ehat_a
  __shared__ double2 s_D[kSepWaves][NV][N];   // the transforms D, per wave and vector
  __shared__ double s_w[kSepWaves][kSepJB];
  const double* th = theta + (size_t)b * 5;
  // Ehat_a = DFT(E_a), zero at the Nyquist index
  if (threadIdx.x < 3) {
    const int a = threadIdx.x;
    double re[N], im[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double x = nodes[i];
      re[i] = exp(th[1 + a] * x - th[4] * x * x);
      im[i] = 0.0;
    }
    fft_reg<double, N, -1>(re, im);
    re[N / 2] = 0.0;
    im[N / 2] = 0.0;
#pragma unroll
    for (int l = 0; l < N; ++l) s_E[a][l] = double2{re[l], im[l]};
  }
  __syncthreads();
  for (int tp0 = 0; tp0 < half; tp0 += kSepWaves) {
    const int ntp = (half - tp0) < kSepWaves ? (half - tp0) : kSepWaves;
    for (int j0 = 0; j0 < n_phi; j0 += kSepJB) {
      const int nj = (n_phi - j0) < kSepJB ? (n_phi - j0) : kSepJB;
      // vectors: 0 = axis 1 of the polar pair, 1 + 2 jl + {0, 1} = axes 2, 3 of azimuth jl
      const int nv = 1 + 2 * nj;
      const int tp = tp0 + wv;
      __syncthreads();
      if (wv < ntp && ln < nv) {
        const int v = ln;
        int a;
        const double2 *pa, *pb;
        bool conj_b;
        if (v == 0) {
          a = 0;
          pa = ph1 + ((size_t)r * n_theta + half + tp) * N;
          pb = ph1 + ((size_t)r * n_theta + half - 1 - tp) * N;
          conj_b = false;
        } else {
          const int jl = (v - 1) >> 1, ax = (v - 1) & 1;
          const int q = tp * n_phi + j0 + jl;
          a = 1 + ax;
          pa = pb = ph23 + (((size_t)r * npairs + q) * 2 + ax) * N;
          conj_b = true;
        }
        double2* row = &s_D[wv][v][0];
        // A and B are real up to rounding (Ehat_a phase is Hermitian: E_a is
        // real, a phase e^{i xi_l s} has xi_{-l} = -xi_l, and Ehat_a is zero at
        // N/2), so one transform of Ehat_a (phase_A + i phase_B) gives A + i B
        double re[N], im[N];
#pragma unroll
        for (int l = 0; l < N; ++l) {
          const double2 E = s_E[a][l], qa = pa[l], q0 = pb[l];
          const double qby = conj_b ? -q0.y : q0.y;
          const double ar = E.x * qa.x - E.y * qa.y, ai = E.x * qa.y + E.y * qa.x;
          const double br = E.x * q0.x - E.y * qby, bi = E.x * qby + E.y * q0.x;
          re[l] = ar - bi;
          im[l] = ai + br;
        }
        fft_reg<double, N, +1>(re, im);
        // D = DFT(A B)
#pragma unroll
        for (int i = 0; i < N; ++i) {
          re[i] = re[i] * im[i];
          im[i] = 0.0;
        }
        fft_reg<double, N, -1>(re, im);
#pragma unroll
        for (int k = 0; k < N; ++k) row[k] = double2{re[k], im[k]};
      }
      if (wv < ntp && ln < nj) s_w[wv][ln] = 2.0 * pairw[tp * n_phi + j0 + ln];
      __syncthreads();
      if (j0 == 0 && threadIdx.x < ntp * N) {
        const int w = threadIdx.x / N, k = threadIdx.x % N;
        D0s[(((size_t)b * n_rho + r) * half + tp0 + w) * N + k] = s_D[w][0][k];
      }
      // G of each polar pair of the round, entries kk = t + u * kSepThreads:
      // one k_3 = t mod N per thread, so its factor loads once per azimuth;
      // the sums of later azimuth passes add to what the first one stored
      const int k3 = threadIdx.x % N;
      for (int w = 0; w < ntp; ++w) {
        double2* Gout = Gs + (((size_t)b * n_rho + r) * half + tp0 + w) * NN;
        double2 g[GPT];
#pragma unroll
        for (int u = 0; u < GPT; ++u) {
          const int kk = threadIdx.x + u * kSepThreads;
          g[u] = (j0 == 0 || kk >= NN) ? double2{0.0, 0.0} : Gout[kk];
        }
        for (int jl = 0; jl < nj; ++jl) {
          const double2 d2 = s_D[w][2 + 2 * jl][k3];
          const double wq = s_w[w][jl];
          const double e2r = wq * d2.x, e2i = wq * d2.y;
#pragma unroll
          for (int u = 0; u < GPT; ++u) {
            const int kk = threadIdx.x + u * kSepThreads;
            const double2 d1 = s_D[w][1 + 2 * jl][(kk < NN ? kk : 0) / N];
            g[u].x += d1.x * e2r - d1.y * e2i;
            g[u].y += d1.x * e2i + d1.y * e2r;
          }
        }
#pragma unroll
        for (int u = 0; u < GPT; ++u) {
          const int kk = threadIdx.x + u * kSepThreads;
          if (kk < NN) Gout[kk] = g[u];
        }
      }
    }
  }
}

// k_max_sep2: two threads own one (k_2, k_3) column of a cell, each with half
// of its N k_1 sums (the halves are the block's two half-blocks, so that a
// wave's columns stay contiguous); each G entry is read by both from the same
// cache line; 128 columns per block.  With all N sums in one thread the FP64
// kernel held 266 registers, one wave per SIMD.  The sums are FP64; the gain
// spectrum Qh is that of the spectral stage (T).
constexpr int kSep2Threads = 256;
constexpr int kSep2Cols = kSep2Threads / 2;

template <int N, typename T>
__global__ __launch_bounds__(kSep2Threads) void k_max_sep2(const double* __restrict__ theta,
                                                           const double2* __restrict__ D0s,
                                                           const double2* __restrict__ Gs,
                                                           const double* __restrict__ W,
                                                           typename V2<T>::type* __restrict__ Qh, int n_rho,
                                                           int n_theta) {
  using C = typename V2<T>::type;
  constexpr int K = N * N * N, NN = N * N;
  constexpr int TPC = 4;  // polar pairs per register batch
  constexpr int KH = N / 2;
  const int hk = threadIdx.x / kSep2Cols;  // which half of the k_1 sums
  const int b = blockIdx.x, t = blockIdx.y * kSep2Cols + threadIdx.x % kSep2Cols;
  const int half = n_theta / 2;
  __shared__ double2 s_D0[TPC][N];
  double2 acc[KH];
#pragma unroll
  for (int k = 0; k < KH; ++k) acc[k] = double2{0.0, 0.0};
  for (int r = 0; r < n_rho; ++r) {
    for (int tp0 = 0; tp0 < half; tp0 += TPC) {
      const int nt = (half - tp0) < TPC ? (half - tp0) : TPC;
      __syncthreads();
      for (int e = threadIdx.x; e < nt * N; e += kSep2Threads)
        s_D0[e / N][e % N] = D0s[(((size_t)b * n_rho + r) * half + tp0 + e / N) * N + e % N];
      __syncthreads();
      double2 g[TPC];
#pragma unroll
      for (int u = 0; u < TPC; ++u)
        g[u] = (t < NN && u < nt) ? Gs[(((size_t)b * n_rho + r) * half + tp0 + u) * NN + t] : double2{0.0, 0.0};
      if (t < NN) {
        const double* Wr = W + (size_t)r * K + t;
#pragma unroll
        for (int k = 0; k < KH; ++k) {
          const int k1 = hk * KH + k;
          double sr = 0.0, si = 0.0;
#pragma unroll
          for (int u = 0; u < TPC; ++u) {
            const double2 d = s_D0[u < nt ? u : 0][k1];
            const double on = u < nt ? 1.0 : 0.0;
            sr += on * (d.x * g[u].x - d.y * g[u].y);
            si += on * (d.x * g[u].y + d.y * g[u].x);
          }
          const double w = Wr[(size_t)k1 * NN];
          acc[k].x += w * sr;
          acc[k].y += w * si;
        }
      }
    }
  }
  if (t < NN) {
    const double ea = exp(theta[(size_t)b * 5]);
    const double sc = ea * ea / ((double)K * (double)K);
    C* q = Qh + (size_t)b * K + t;
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const int k1 = hk * KH + k;
      const C v = q[(size_t)k1 * NN];
      q[(size_t)k1 * NN] = C{T(double(v.x) - sc * acc[k].x), T(double(v.y) - sc * acc[k].y)};
    }
  }
}

// ------------------------------------------------------------------ combine
template <typename T, int N, int NF>
__global__ __launch_bounds__(256) void k_combine(const double* __restrict__ f, const double* __restrict__ GH,
                                                 const typename V2<T>::type* __restrict__ Qp,
                                                 const typename V2<T>::type* __restrict__ Lc, double* __restrict__ Q,
                                                 int64_t n, const double* __restrict__ scale) {
  constexpr int K = N * N * N;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n) return;
  const int64_t b = gid / K;
  const int k = (int)(gid % K);
  double gain = double(Qp[gid].x);
  double loss;
  if (NF == 1) {
    loss = f[gid] * double(Lc[gid].x);
  } else if (NF == 3) {
    // difference form: f L[f] - M L[M], the packed loss transform L[f] + i L[M]
    loss = f[gid] * double(Lc[gid].x) - GH[gid] * double(Lc[gid].y);
  } else {
    // bilinear form: the gain and L[g] carry the power-of-two scale of g
    const double is = 1.0 / scale[b];
    const double g = GH[b * 2 * K + k], h = GH[b * 2 * K + K + k];
    const double Lg = double(Lc[b * 2 * K + k].x) * is, Lh = double(Lc[b * 2 * K + K + k].x);
    loss = 0.5 * (g * Lh + h * Lg);
    gain *= is;
  }
  Q[gid] = gain - loss;
}

// ------------------------------------------------------------------ host driver
// Workspace of one cell: spectra and loss transforms of nvol volumes (f, or the
// two fields of the corrected form), the fields for the final combine, the
// z-stage planes of the nz fields that go through the direction pairs, the
// accumulated planes of nacc radial nodes (folded into the gain spectrum by
// one column pass), the gain spectrum, and for the FP64 difference form the
// separable Maxwellian factors D0, G and the Maxwellian parameters.
struct QLayout {
  bool diff;   // FP64 corrected form as Q[f,f] - Q[M,M] (separable Maxwellian gain)
  int nvol;    // spectrum / loss volumes per cell
  int nz;      // fields through the z-stage and the direction pairs
  int nacc;    // radial nodes whose accumulated planes are held at once
  size_t per;  // bytes per cell
};

// radial nodes held per column pass: the plan's value (0: all of them, the
// accumulator then being written once), at most n_rho; 1 for the Carleman
// form, which has no radial loop
static int acc_nodes(const bz_ctx* ctx) {
  if (ctx->p.method == BZ_METHOD_CARLEMAN) return 1;
  const int a = ctx->acc_nodes > 0 ? ctx->acc_nodes : ctx->n_rho;
  return a < ctx->n_rho ? a : ctx->n_rho;
}

// diff32: the FP32 stage in the difference form (BZ_FP32_DIFF)
template <typename T>
static QLayout q_layout(int N, int n_theta, int n_rho, int nacc, bool corrected, bool carleman, bool diff32) {
  const size_t K = (size_t)N * N * N, cs = 2 * sizeof(T);
  QLayout q;
  q.diff = (sizeof(T) == 8 || diff32) && corrected && !carleman;
  q.nvol = corrected ? 2 : 1;
  q.nz = q.diff ? 1 : q.nvol;
  q.nacc = nacc;
  // Z: half planes for the N = 32 pair kernel; the Carleman form keeps the
  // full region for its direction fields
  const size_t zk = (N == 32 && !carleman) ? K / 2 : K;
  // the difference form transforms f + i M as one volume: Fc holds it and the
  // unpacked spectrum of f, Lc one packed loss volume
  q.per = K * (q.nvol * cs /*Fc*/ + (q.diff ? 1 : q.nvol) * cs /*Lc*/ + (q.diff ? 8 : q.nvol * 8) /*GH*/ +
               (size_t)nacc * cs /*Acc*/ + cs /*Qh*/) +
          zk * (size_t)q.nz * n_theta * cs /*Z*/;
  if (q.diff) q.per += (size_t)n_rho * (n_theta / 2) * ((size_t)N + (size_t)N * N) * 16 /*D0, G*/ + 5 * 8 /*theta*/;
  else if (corrected) q.per += 8 /*scale of g*/;
  return q;
}

template <typename T>
static QLayout q_layout(const bz_ctx* ctx, bool corrected) {
  return q_layout<T>(ctx->N, ctx->n_theta, ctx->n_rho, acc_nodes(ctx), corrected,
                     ctx->p.method == BZ_METHOD_CARLEMAN, ctx->p.precision == BZ_FP32_DIFF);
}

// cells per chunk of the collision workspace: the plan's chunk size if it
// sets one, else as many as an 8 GiB budget holds (about 3% of the device's
// HBM; 594 cells of the FP64 corrected form at 32^3, M = 128, n_rho = 16 with
// every radial node held); never more than the bytes of a caller-provided
// workspace hold
constexpr size_t kWsBudget = (size_t)8 << 30;

template <typename T, int N>
static int64_t chunk_cells(const bz_ctx* ctx, int64_t batch, bool corrected, size_t ws_ext_bytes = 0) {
  const size_t per = q_layout<T>(ctx, corrected).per;
  int64_t chunk = ctx->chunk_cap > 0 ? ctx->chunk_cap : (int64_t)(kWsBudget / per);
  if (ws_ext_bytes > 0 && chunk > (int64_t)(ws_ext_bytes / per)) chunk = (int64_t)(ws_ext_bytes / per);
  if (chunk < 1) chunk = 1;
  if (chunk > batch) chunk = batch;
  return chunk;
}

template <typename T, int NF>
static const void* pair_kernel(int N, int W) {
  if (N == 32) {
    if (W == 2) return (const void*)k_pairs32<T, NF, 2>;
    if (W == 4) return (const void*)k_pairs32<T, NF, 4>;
    return (const void*)k_pairs32<T, NF, 8>;
  }
  if (N == 16) return (const void*)k_pairs<T, 16, NF>;
  return (const void*)k_pairs<T, 8, NF>;
}

// waves per block of the N = 32 pair kernel for this context (tuned, else 8)
static int pair_waves(const bz_ctx* ctx) { return ctx->pair_waves > 0 ? ctx->pair_waves : 8; }

template <typename T, int N>
static bz_status prepare_chunked(bz_ctx* ctx, int64_t batch, bool corrected) {
  if (batch == 0) return BZ_OK;
  const QLayout ql = q_layout<T>(ctx, corrected);
  bz_status s = ensure_ws(ctx, ql.per * chunk_cells<T, N>(ctx, batch, corrected));
  if (s != BZ_OK) return s;
  const int W = pair_waves(ctx);
  const size_t lds = (N == 32) ? pairs32_lds_bytes<T>(W) : pairs_lds_bytes<T, N>();
  const void* kp = ql.nz == 2 ? pair_kernel<T, 2>(N, W) : pair_kernel<T, 1>(N, W);
  BZ_HIP(hipFuncSetAttribute(kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return BZ_OK;
}

template <typename T, int N>
static bz_status run_chunked(bz_ctx* ctx, const double* f, double* Q, int64_t batch, bool corrected, double* theta_out,
                             hipStream_t st, void* ws_ext, size_t ws_ext_bytes) {
  using C = typename V2<T>::type;
  constexpr int K = N * N * N, NN = N * N;
  const QLayout ql = q_layout<T>(ctx, corrected);
  const int nf = ql.nvol, nz = ql.nz;
  const int nt = ctx->n_theta;
  const size_t per = ql.per;
  bz_status s = BZ_OK;
  int64_t chunk;
  unsigned char* base;
  if (ws_ext) {
    // the caller's workspace: no allocation, chunks sized to it
    if (per > ws_ext_bytes) return set_err(ctx, BZ_EINVAL, "one cell's collision workspace exceeds the given workspace");
    chunk = chunk_cells<T, N>(ctx, batch, corrected, ws_ext_bytes);
    base = (unsigned char*)ws_ext;
  } else {
    chunk = chunk_cells<T, N>(ctx, batch, corrected);
    s = ensure_ws(ctx, per * chunk);
    if (s != BZ_OK) return s;
    base = (unsigned char*)ctx->ws;
  }
  C* Fc = (C*)base;
  C* Lc = Fc + (size_t)chunk * nf * K;
  double* GH = (double*)(Lc + (size_t)chunk * (ql.diff ? 1 : nf) * K);
  // the difference form's unpacked spectrum of f: the second Fc slot
  C* Fu = Fc + (size_t)chunk * K;
  C* Z = (C*)(GH + (size_t)chunk * (ql.diff ? 1 : nf) * K);
  const bool zfull = N != 32 || ctx->p.method == BZ_METHOD_CARLEMAN;
  C* Acc = Z + (size_t)chunk * nz * nt * (zfull ? K : K / 2);
  const int nacc = ql.nacc;
  const int64_t slot = (int64_t)chunk * K;  // one radial node's accumulated planes
  C* Qh = Acc + (size_t)nacc * slot;
  const int half = nt / 2;
  double2* D0s = (double2*)(Qh + (size_t)chunk * K);
  double2* Gs = D0s + (ql.diff ? (size_t)chunk * ctx->n_rho * half * N : 0);
  double* th_ws = (double*)(Gs + (ql.diff ? (size_t)chunk * ctx->n_rho * half * NN : 0));
  const bool f64 = sizeof(T) == 8;
  const C* ph1 = (const C*)(f64 ? (const void*)ctx->d_ph1 : (const void*)ctx->d_ph1_f);
  const C* ph23 = (const C*)(f64 ? (const void*)ctx->d_ph23 : (const void*)ctx->d_ph23_f);
  const T* pairw = (const T*)(f64 ? (const void*)ctx->d_pairw : (const void*)ctx->d_pairw_f);
  const T* pairsw = (const T*)(f64 ? (const void*)ctx->d_pairsw : (const void*)ctx->d_pairsw_f);
  // the N = 32 kernel takes sqrt of the pair weights, the general one the weights
  const T* pw = (N == 32) ? pairsw : pairw;
  const T* W = (const T*)(f64 ? (const void*)ctx->d_W : (const void*)ctx->d_W_f);
  const bool carleman = ctx->p.method == BZ_METHOD_CARLEMAN;
  // the loss weight: the radial sigma-form weight, or sum_p A_p B_p of the Carleman form
  const T* Gm = carleman ? (const T*)(f64 ? (const void*)ctx->d_cbeta : (const void*)ctx->d_cbeta_f)
                         : (const T*)(f64 ? (const void*)ctx->d_Gm : (const void*)ctx->d_Gm_f);
  const T* cw = (const T*)(f64 ? (const void*)ctx->d_cw : (const void*)ctx->d_cw_f);
  constexpr int PPB = plane_ppb<T, N>();
  const int PW = pair_waves(ctx);
  const size_t lds = (N == 32) ? pairs32_lds_bytes<T>(PW) : pairs_lds_bytes<T, N>();
  const void* kp = nz == 2 ? pair_kernel<T, 2>(N, PW) : pair_kernel<T, 1>(N, PW);
  BZ_HIP(hipFuncSetAttribute(kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const int pair_threads = (N == 32) ? 64 * PW : 64 * kPairWaves;
  for (int64_t c0 = 0; c0 < batch; c0 += chunk) {
    const int64_t B = (batch - c0) < chunk ? (batch - c0) : chunk;
    const double* fb = f + c0 * K;
    // transformed volumes: f + i M packed in one in the difference form
    const int64_t nvol = ql.diff ? B : B * nf;
    // the difference form needs the Maxwellian parameters for its separable part
    double* th_b = theta_out ? theta_out + c0 * 5 : (ql.diff ? th_ws : nullptr);
    // the bilinear form's per-cell scale of g (the region the difference form
    // keeps its parameters in)
    double* sc_b = (corrected && !ql.diff) ? th_ws : nullptr;
    hipLaunchKernelGGL((k_prep<T, N>), dim3((unsigned)B), dim3(kPrepThreads), 0, st, fb, GH, Fc, th_b, ctx->d_nodes,
                       ctx->w, ql.diff ? 2 : (corrected ? 1 : 0), sc_b);
    const unsigned gcol = (unsigned)((nvol * NN + 255) / 256);
    const unsigned gpl = (unsigned)((nvol * N + PPB - 1) / PPB);
    hipLaunchKernelGGL((k_plane<T, N, -1>), dim3(gpl), dim3(N * PPB), 0, st, Fc, Fc, nvol * N);
    hipLaunchKernelGGL((k_col<T, N, -1, COL_FWD_NYQ>), dim3(gcol), dim3(256), 0, st, Fc, Fc, nvol, (const T*)nullptr);
    // loss: L[u] = IDFT(Gm * uhat)
    hipLaunchKernelGGL((k_col<T, N, +1, COL_PREMUL>), dim3(gcol), dim3(256), 0, st, Fc, Lc, nvol, Gm);
    hipLaunchKernelGGL((k_plane<T, N, +1>), dim3(gpl), dim3(N * PPB), 0, st, Lc, Lc, nvol * N);
    constexpr bool zhalf = N == 32;
    if (ql.diff) {
      const unsigned gu = (unsigned)((B * N * zplane<N, zhalf>() + 255) / 256);
      hipLaunchKernelGGL((k_unpack<T, N, zhalf>), dim3(gu), dim3(256), 0, st, Fc, Fu, B);
    }
    // the fields through the z-stage: the unpacked spectrum of f, or the spectra
    const C* Fz = ql.diff ? Fu : Fc;
    if (carleman) {
      // gain accumulated in physical space in the Qh region (B*K reals); the
      // direction fields use the Z region ([B][N][nf][N][N] complex)
      T* gain = (T*)Qh;
      C* D = Z;
      const unsigned gcp = (unsigned)((B * N * nf + PPB - 1) / PPB);
      const unsigned gc32 = (unsigned)((B * N + kCplaneWaves - 1) / kCplaneWaves);
      // algorithmic FLOPs of one direction per cell: nf complex 3D transforms,
      // the table products (6 per entry) and the accumulation (3 per entry)
      const double dir_flops = nf * (15.0 * NN * N * __builtin_ctz(N) + 6.0 * NN * N) + 3.0 * NN * N;
      // N = 32 takes up to 4 directions per launch pair (the gain is read and
      // written once per group); the workspace holds min(4, n_theta) of them
      const int group = (N == 32) ? (nt < 4 ? nt : 4) : 1;
      for (int p = 0; p < ctx->n_dir; p += group) {
        const int nd = (ctx->n_dir - p) < group ? (ctx->n_dir - p) : group;
        const T* tab = cw + (size_t)p * 2 * K;
        if ((s = prof_mark(ctx, st, false, 0.0)) != BZ_OK) return s;
        const int first = p == 0 ? 1 : 0;
        const unsigned gcc = (unsigned)((B * nd * nf * NN + 255) / 256);
        if (nf == 1) {
          hipLaunchKernelGGL((k_ccol<T, N, 1>), dim3(gcc), dim3(256), 0, st, Fc, D, B, tab, nd);
          if (N == 32)
            hipLaunchKernelGGL((k_cplane32<T, 1>), dim3(gc32), dim3(64 * kCplaneWaves), 0, st, D, gain, B * N, nd,
                               first);
          else
            hipLaunchKernelGGL((k_cplane<T, N, 1>), dim3(gcp), dim3(N * PPB), 0, st, D, gain, B * N, first);
        } else {
          hipLaunchKernelGGL((k_ccol<T, N, 2>), dim3(gcc), dim3(256), 0, st, Fc, D, B, tab, nd);
          if (N == 32)
            hipLaunchKernelGGL((k_cplane32<T, 2>), dim3(gc32), dim3(64 * kCplaneWaves), 0, st, D, gain, B * N, nd,
                               first);
          else
            hipLaunchKernelGGL((k_cplane<T, N, 2>), dim3(gcp), dim3(N * PPB), 0, st, D, gain, B * N * 2, first);
        }
        if ((s = prof_mark(ctx, st, true, (double)B * nd * dir_flops)) != BZ_OK) return s;
      }
      const unsigned ge = (unsigned)((B * K + 255) / 256);
      if (corrected)
        hipLaunchKernelGGL((k_ccombine<T, N, 2>), dim3(ge), dim3(256), 0, st, fb, GH, gain, Lc, Q + c0 * K, B * K,
                           sc_b);
      else
        hipLaunchKernelGGL((k_ccombine<T, N, 1>), dim3(ge), dim3(256), 0, st, fb, GH, gain, Lc, Q + c0 * K, B * K,
                           sc_b);
      BZ_HIP(hipGetLastError());
      continue;
    }
    const int64_t nzvol = B * nz;
    const unsigned gz = (unsigned)((nzvol * zplane<N, zhalf>() + 255) / 256);
    for (int r = 0; r < ctx->n_rho; ++r) {
      hipLaunchKernelGGL((k_zstage<T, N, zhalf>), dim3(gz), dim3(256), 0, st, Fz, Z, nzvol, nt,
                         ph1 + (size_t)r * nt * N);
      const C* ph23r = ph23 + (size_t)r * ctx->n_pairs * 2 * N;
      const double job_flops = 10.0 * NN * __builtin_ctz(N) + 17.0 * NN;
      if ((s = prof_mark(ctx, st, false, 0.0)) != BZ_OK) return s;
      {
        C* acc_r = Acc + (size_t)(r % nacc) * slot;
        void* args[] = {(void*)&Z, (void*)&acc_r, (void*)&nt, (void*)&ctx->n_phi, (void*)&ph23r, (void*)&pw};
        BZ_HIP(hipLaunchKernel(kp, dim3((unsigned)(B * N)), dim3(pair_threads), args, lds, st));
      }
      if ((s = prof_mark(ctx, st, true, (double)B * N * ctx->n_pairs * nz * job_flops)) != BZ_OK) return s;
      // fold the held nodes into the gain spectrum once the slots are full
      if (r % nacc == nacc - 1 || r == ctx->n_rho - 1) {
        const int r0 = r - r % nacc, ns = r - r0 + 1;
        const unsigned gq = (unsigned)((2 * B * NN + 255) / 256);  // two lanes per column
        hipLaunchKernelGGL((k_colw<T, N>), dim3(gq), dim3(256), 0, st, Acc, Qh, B, W + (size_t)r0 * K, ns, slot,
                           r0 == 0 ? 1 : 0);
      }
    }
    if (ql.diff) {
      // subtract the gain of the Maxwellian, by separable transforms
      hipLaunchKernelGGL((k_max_sep1<N>), dim3((unsigned)(B * ctx->n_rho)), dim3(kSepThreads), 0, st, th_b,
                         ctx->d_nodes, (const double2*)ctx->d_ph1, (const double2*)ctx->d_ph23, ctx->d_pairw,
                         ctx->n_rho, nt, ctx->n_phi, D0s, Gs);
      hipLaunchKernelGGL((k_max_sep2<N, T>), dim3((unsigned)B, (unsigned)((NN + kSep2Cols - 1) / kSep2Cols)),
                         dim3(kSep2Threads), 0, st, (const double*)th_b, (const double2*)D0s, (const double2*)Gs,
                         ctx->d_W, Qh, ctx->n_rho, nt);
    }
    const unsigned gq = (unsigned)((B * NN + 255) / 256);
    hipLaunchKernelGGL((k_col<T, N, +1, COL_PLAIN>), dim3(gq), dim3(256), 0, st, Qh, Qh, B, (const T*)nullptr);
    hipLaunchKernelGGL((k_plane<T, N, +1>), dim3((unsigned)((B * N + PPB - 1) / PPB)), dim3(N * PPB), 0, st, Qh, Qh,
                       B * N);
    const unsigned ge = (unsigned)((B * K + 255) / 256);
    if (ql.diff)
      hipLaunchKernelGGL((k_combine<T, N, 3>), dim3(ge), dim3(256), 0, st, fb, GH, Qh, Lc, Q + c0 * K, B * K,
                         sc_b);
    else if (corrected)
      hipLaunchKernelGGL((k_combine<T, N, 2>), dim3(ge), dim3(256), 0, st, fb, GH, Qh, Lc, Q + c0 * K, B * K,
                         sc_b);
    else
      hipLaunchKernelGGL((k_combine<T, N, 1>), dim3(ge), dim3(256), 0, st, fb, GH, Qh, Lc, Q + c0 * K, B * K,
                         sc_b);
    BZ_HIP(hipGetLastError());
  }
  return BZ_OK;
}

size_t eval_q_ws_per_cell(const bz_ctx* ctx, bool corrected) {
  return ctx->p.precision != BZ_FP64 ? q_layout<float>(ctx, corrected).per : q_layout<double>(ctx, corrected).per;
}

bz_status eval_q_prepare(bz_ctx* ctx, int64_t batch, bool corrected) {
  const bool fp32 = ctx->p.precision != BZ_FP64;
  switch (ctx->N) {
    case 8:
      return fp32 ? prepare_chunked<float, 8>(ctx, batch, corrected) : prepare_chunked<double, 8>(ctx, batch, corrected);
    case 16:
      return fp32 ? prepare_chunked<float, 16>(ctx, batch, corrected)
                  : prepare_chunked<double, 16>(ctx, batch, corrected);
    case 32:
      return fp32 ? prepare_chunked<float, 32>(ctx, batch, corrected)
                  : prepare_chunked<double, 32>(ctx, batch, corrected);
  }
  return set_err(ctx, BZ_EUNSUPPORTED, "N must be 8, 16 or 32");
}

bz_status eval_q(bz_ctx* ctx, const double* f, double* Q, int64_t batch, bool corrected, double* theta_out,
                 hipStream_t st, void* ws_ext, size_t ws_ext_bytes) {
  if (batch == 0) return BZ_OK;
  const bool fp32 = ctx->p.precision != BZ_FP64;
  switch (ctx->N) {
    case 8:
      return fp32 ? run_chunked<float, 8>(ctx, f, Q, batch, corrected, theta_out, st, ws_ext, ws_ext_bytes)
                  : run_chunked<double, 8>(ctx, f, Q, batch, corrected, theta_out, st, ws_ext, ws_ext_bytes);
    case 16:
      return fp32 ? run_chunked<float, 16>(ctx, f, Q, batch, corrected, theta_out, st, ws_ext, ws_ext_bytes)
                  : run_chunked<double, 16>(ctx, f, Q, batch, corrected, theta_out, st, ws_ext, ws_ext_bytes);
    case 32:
      return fp32 ? run_chunked<float, 32>(ctx, f, Q, batch, corrected, theta_out, st, ws_ext, ws_ext_bytes)
                  : run_chunked<double, 32>(ctx, f, Q, batch, corrected, theta_out, st, ws_ext, ws_ext_bytes);
    default:
      return set_err(ctx, BZ_EUNSUPPORTED, "N must be 8, 16 or 32");
  }
}

}  // namespace bz
