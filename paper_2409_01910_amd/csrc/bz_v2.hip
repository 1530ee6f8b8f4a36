// Two-dimensional velocity space (d = 2): the Fourier spectral collision
// operator in its sigma form on the circle, the discrete Maxwellian, and the
// steady-state corrected form, for independent cells on an N x N grid.
//
// Section 4.2 runs its binary-collision examples with two-dimensional
// velocities and Maxwell molecules.  With f periodic on [-L, L)^2,
// f(v_j) = sum_l fh_l exp(i xi_l.(v_j - v_0)), the sigma form (Section 2.2,
// eq. collision, relative speed truncated at R_g = 2R) is
//   gain  Qh+_k = sum_r W_r(|xi_k|) DFT_k[ sum_p 2 w_p f(v + s) f(v - s) ],
//         s = rho_r sigma_p / 2 over the M/2 antipodal pairs of the circle rule,
//   loss  Q- = f IDFT[ Gm(|xi|) fh ],
// with W_r and Gm as built by the host tables (S_2(z) = 2 pi J0(z)).  The
// shift f(v + s) is the phase exp(i xi.s) on fh.
//
// The steady-state corrected form of eq. discrete_Q is evaluated as the
// symmetric bilinear form Q_s(g, h) with g = f - M, h = f + M, which equals
// Q[f,f] - Q[M,M] without the cancellation of the difference: for each pair,
// one complex transform of gh phi + i hh conj(phi) gives g(v + s) and h(v - s)
// at once (both real), and a second one h(v + s) and g(v - s).
//
// With BZ_METHOD_CARLEMAN (Maxwell molecules) the same machinery evaluates the
// Carleman form (k_c2): no radial quadrature, one or two transforms per
// half-circle direction.
//
// Layout and work split: one workgroup of 512 threads per cell.  K = N^2 is at
// most 2304, so the two spectra (gh, hh) and the two ping-pong buffers of a
// transform (rows padded to N + 1) fit in LDS together (151 KB at N = 48), and
// every pass of every transform stays on chip: the cell's field is read from
// HBM once and Q written once.  Transforms are Stockham autosort passes of
// radix 4, 3 and 2 along the fast axis, then along the slow axis; thread t owns
// the points k = t + 512 i for the pointwise work (accumulators in registers).
#include <cmath>
#include <type_traits>

#include "bz_common.hpp"
#include "bz_internal.hpp"

namespace bz {
namespace {

// Threads per workgroup: 512, and 768 for the 48 x 48 grid, where each radix-4
// pass has 576 butterflies and each radix-3 pass 768, so that every pass takes
// one round of the workgroup instead of two.  FP32 workgroups of 512 threads
// are held to 128 registers so that two share a CU.
constexpr int kV2MaxThreads = 768;
template <typename T, int N>
constexpr int v2_threads() {
  return N == 48 ? 768 : 512;
}
// FP32 48 x 48 workgroups (76 KB of LDS) are held to 80 registers, so that two
// share a CU.
template <typename T, int N>
constexpr int v2_waves_per_eu() {
  return sizeof(T) == 4 ? (v2_threads<T, N>() == 512 ? 4 : 6) : 1;
}
template <typename T, int N>
constexpr int c2_waves_per_eu() {
  return v2_waves_per_eu<T, N>();
}

// complex values of the transform stage: double2 (FP64) or float2 (FP32)
template <typename T>
struct Cx;
template <>
struct Cx<double> {
  using C = double2;
  __device__ static C make(double a, double b) { return make_double2(a, b); }
};
template <>
struct Cx<float> {
  using C = float2;
  __device__ static C make(float a, float b) { return make_float2(a, b); }
};
template <typename T>
using cx_t = typename Cx<T>::C;

template <typename T>
__device__ __forceinline__ cx_t<T> cmul(cx_t<T> a, cx_t<T> b) {
  return Cx<T>::make(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cx_t<T> cconj(cx_t<T> a) {
  return Cx<T>::make(a.x, -a.y);
}

// The q-th radix of a length-n transform: 4 while it divides, then 3, then 2
// (1 past the last pass).
constexpr int radix_at(int n, int q) {
  for (int i = 0;; ++i) {
    const int r = n % 4 == 0 ? 4 : n % 3 == 0 ? 3 : n % 2 == 0 ? 2 : 1;
    if (r == 1 || i == q) return r;
    n /= r;
  }
}

// y_k = sum_m v_m exp(SIGN 2 pi i m k / R), in place, R in {2, 3, 4}
template <typename T, int R, int SIGN>
__device__ __forceinline__ void small_dft(cx_t<T> (&v)[R]) {
  using X = Cx<T>;
  if constexpr (R == 2) {
    const cx_t<T> a = v[0], b = v[1];
    v[0] = X::make(a.x + b.x, a.y + b.y);
    v[1] = X::make(a.x - b.x, a.y - b.y);
  } else if constexpr (R == 3) {
    const T h = T(0.86602540378443864676 * SIGN);  // SIGN * sqrt(3) / 2
    const cx_t<T> t1 = X::make(v[1].x + v[2].x, v[1].y + v[2].y);
    const cx_t<T> t2 = X::make(v[0].x - T(0.5) * t1.x, v[0].y - T(0.5) * t1.y);
    const cx_t<T> t3 = X::make(h * (v[1].x - v[2].x), h * (v[1].y - v[2].y));
    v[0] = X::make(v[0].x + t1.x, v[0].y + t1.y);
    // i * t3 = (-t3.y, t3.x)
    v[1] = X::make(t2.x - t3.y, t2.y + t3.x);
    v[2] = X::make(t2.x + t3.y, t2.y - t3.x);
  } else {
    const cx_t<T> a = X::make(v[0].x + v[2].x, v[0].y + v[2].y);
    const cx_t<T> b = X::make(v[0].x - v[2].x, v[0].y - v[2].y);
    const cx_t<T> c = X::make(v[1].x + v[3].x, v[1].y + v[3].y);
    // SIGN * i * (v1 - v3)
    const cx_t<T> e = X::make(T(-SIGN) * (v[1].y - v[3].y), T(SIGN) * (v[1].x - v[3].x));
    v[0] = X::make(a.x + c.x, a.y + c.y);
    v[2] = X::make(a.x - c.x, a.y - c.y);
    v[1] = X::make(b.x + e.x, b.y + e.y);
    v[3] = X::make(b.x - e.x, b.y - e.y);
  }
}

// One Stockham pass of radix R over all N lines of an N x N tile along one
// axis (AXIS 1: rows; AXIS 0: columns).  The tile's rows are P = N + 1 complex
// values apart, and consecutive threads take consecutive lines, so that the
// lanes of a wave hit distinct LDS banks along either axis.  NS is the product
// of the radices of the earlier passes on this axis; tw[q] = exp(2 pi i q / N).
template <typename T, int N, int R, int NS, int AXIS, int SIGN>
__device__ __forceinline__ void stockham_pass(const cx_t<T>* __restrict__ src, cx_t<T>* __restrict__ dst,
                                              const cx_t<T>* tw) {
  constexpr int NR = N / R, items = N * NR, step = N / (NS * R), P = N + 1;
  constexpr int es = AXIS == 1 ? 1 : P, ls = AXIS == 1 ? P : 1;
  for (int t = threadIdx.x; t < items; t += blockDim.x) {
    const int j = t / N, line = t - j * N;
    const int k = j % NS;
    const int base = line * ls;
    cx_t<T> v[R];
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = src[base + (j + m * NR) * es];
    if constexpr (NS > 1) {  // the first pass of an axis has unit twiddles
#pragma unroll
      for (int m = 1; m < R; ++m) {
        cx_t<T> w = tw[k * m * step];
        if (SIGN < 0) w = cconj<T>(w);
        v[m] = cmul<T>(v[m], w);
      }
    }
    small_dft<T, R, SIGN>(v);
    const int d0 = (j / NS) * NS * R + k;
#pragma unroll
    for (int m = 0; m < R; ++m) dst[base + (d0 + m * NS) * es] = v[m];
  }
}

template <typename T, int N, int SIGN, int AXIS, int Q, int NS>
__device__ __forceinline__ void axis_passes(cx_t<T>*& src, cx_t<T>*& dst, const cx_t<T>* tw) {
  constexpr int R = radix_at(N, Q);
  if constexpr (R > 1) {
    stockham_pass<T, N, R, NS, AXIS, SIGN>(src, dst, tw);
    __syncthreads();
    cx_t<T>* t = src;
    src = dst;
    dst = t;
    axis_passes<T, N, SIGN, AXIS, Q + 1, NS * R>(src, dst, tw);
  }
}

// 2D transform X_k = sum_j x_j exp(SIGN 2 pi i k.j / N) of tile a (b is the
// ping-pong partner); returns the tile that holds the result.  Synchronises
// before returning.
template <typename T, int N, int SIGN>
__device__ __forceinline__ cx_t<T>* dft2(cx_t<T>* a, cx_t<T>* b, const cx_t<T>* tw) {
  cx_t<T>* src = a;
  cx_t<T>* dst = b;
  axis_passes<T, N, SIGN, 1, 0, 1>(src, dst, tw);
  axis_passes<T, N, SIGN, 0, 0, 1>(src, dst, tw);
  return src;
}

// Fused transforms for the inner loops.  A radix pass in general form: item t
// (line fastest, as in stockham_pass) gathers its R inputs through ld(line, e)
// or ld(o, line, e) and hands its R outputs to st(o, line, e, v), where e is
// the position along the pass axis and o = round * R + m numbers the inputs and
// outputs a thread handles.
// Twiddle powers w^m are formed from one table value.
template <typename T, int N, int R, int NS, int SIGN, int NT, class Ld, class St>
__device__ __forceinline__ void radix_pass(const Ld& ld, const St& st, const cx_t<T>* tw) {
  constexpr int NR = N / R, items = N * NR, step = N / (NS * R);
  constexpr int rounds = (items + NT - 1) / NT;
#pragma unroll
  for (int q = 0; q < rounds; ++q) {
    const int t = threadIdx.x + q * NT;
    if (items % NT == 0 || t < items) {
      const int j = t / N, line = t - j * N;
      const int k = j % NS;
      cx_t<T> v[R];
#pragma unroll
      for (int m = 0; m < R; ++m) {
        if constexpr (std::is_invocable_v<Ld, int, int, int>)
          v[m] = ld(q * R + m, line, j + m * NR);
        else
          v[m] = ld(line, j + m * NR);
      }
      if constexpr (NS > 1) {
        cx_t<T> w = tw[k * step];
        if (SIGN < 0) w = cconj<T>(w);
        cx_t<T> wm = w;
#pragma unroll
        for (int m = 1; m < R; ++m) {
          v[m] = cmul<T>(v[m], wm);
          if (m + 1 < R) wm = cmul<T>(wm, w);
        }
      }
      small_dft<T, R, SIGN>(v);
      const int d0 = (j / NS) * NS * R + k;
#pragma unroll
      for (int m = 0; m < R; ++m) st(q * R + m, line, d0 + m * NS, v[m]);
    }
  }
}

constexpr int n_radix(int n) {
  int q = 0;
  while (radix_at(n, q) > 1) ++q;
  return q;
}

// All passes of a 2D transform, axis A (0: columns, 1: rows) first.  The first
// pass reads its input through ld0 (line and e along axis A) and
// writes tile oth; the last pass (along the other axis) hands its outputs to
// sink(o, line, e, v) instead of a tile.  Tiles cur and oth alternate between
// the passes in between; the pass count is even, so the last pass reads oth.
// Synchronises after every pass but the last: a caller that starts another
// transform right away gives it the tiles swapped (its first pass then writes
// the tile no thread still reads), and synchronises before it writes a tile
// itself.
template <typename T, int N, int SIGN, int NT, int A, int AXIS, int Q, int NS, class Ld, class Sk>
__device__ __forceinline__ void fused_passes(const Ld& ld0, const Sk& sink, cx_t<T>* cur, cx_t<T>* oth,
                                             const cx_t<T>* tw) {
  constexpr int R = radix_at(N, Q), RN = radix_at(N, Q + 1), P = N + 1;
  constexpr int es = AXIS == 1 ? 1 : P, ls = AXIS == 1 ? P : 1;
  constexpr bool first = AXIS == A && Q == 0, last = AXIS != A && RN == 1;
  static_assert(!(first && last), "a transform has at least two passes");
  const auto ld_lds = [cur](int line, int e) { return cur[line * ls + e * es]; };
  const auto st_lds = [oth](int, int line, int e, cx_t<T> v) { oth[line * ls + e * es] = v; };
  if constexpr (first)
    radix_pass<T, N, R, NS, SIGN, NT>(ld0, st_lds, tw);
  else if constexpr (last)
    radix_pass<T, N, R, NS, SIGN, NT>(ld_lds, sink, tw);
  else
    radix_pass<T, N, R, NS, SIGN, NT>(ld_lds, st_lds, tw);
  if constexpr (!last) __syncthreads();
  if constexpr (RN > 1)
    fused_passes<T, N, SIGN, NT, A, AXIS, Q + 1, NS * R>(ld0, sink, oth, cur, tw);
  else if constexpr (AXIS == A)
    fused_passes<T, N, SIGN, NT, A, 1 - A, 0, 1>(ld0, sink, oth, cur, tw);
}

template <typename T, int N, int SIGN, int NT, int A, class Ld, class Sk>
__device__ __forceinline__ void dft2_fused(const Ld& ld0, const Sk& sink, cx_t<T>* cur, cx_t<T>* oth,
                                           const cx_t<T>* tw) {
  fused_passes<T, N, SIGN, NT, A, A, 0, 1>(ld0, sink, cur, oth, tw);
}

// Outputs per thread of the last pass of dft2_fused, and the grid point
// k = i_1 N + i_2 of output o (-1 if the thread has no such output); the last
// pass runs along axis 1 - A.
template <int N, int NT>
constexpr int fused_own() {
  constexpr int R = radix_at(N, n_radix(N) - 1);
  return (N * (N / R) + NT - 1) / NT * R;
}
template <int N, int NT, int A>
__device__ __forceinline__ int fused_point(int o) {
  constexpr int R = radix_at(N, n_radix(N) - 1), NS = N / R, items = N * (N / R);
  const int q = o / R, m = o - q * R, t = threadIdx.x + q * NT;
  if (t >= items) return -1;
  const int j = t / N, line = t - j * N, k = j % NS;
  const int e = (j / NS) * NS * R + k + m * NS;
  return A == 0 ? line * N + e : e * N + line;
}

// The first pass of every direction transform reads the same spectra entries
// (columns first: thread (j, line) reads (i_1, i_2) = (j + m N / R, line)).
// In the Carleman kernel in FP64 on 48 x 48 (one workgroup per CU by its LDS,
// registers to spare) each thread keeps its entries of both spectra in
// registers: 3.17 -> 3.02 ms per 4096 cells.  (The sigma kernel ran slower so.)
template <typename T, int N>
constexpr bool spec_in_regs() {
  return sizeof(T) == 8 && N == 48;
}
template <typename T, int N, int NT>
constexpr int spec_own() {
  constexpr int R = radix_at(N, 0);
  return spec_in_regs<T, N>() ? (N * (N / R) + NT - 1) / NT * R : 1;
}
template <typename T, int N, int NT, int S>
__device__ __forceinline__ void load_spec(const cx_t<T>* SG, const cx_t<T>* SH, cx_t<T> (&sg)[S], cx_t<T> (&sh)[S]) {
  constexpr int R = radix_at(N, 0), items = N * (N / R);
#pragma unroll
  for (int o = 0; o < S; ++o) {
    sg[o] = sh[o] = Cx<T>::make(T(0), T(0));
    if constexpr (spec_in_regs<T, N>()) {
      const int q = o / R, m = o - q * R, t = threadIdx.x + q * NT;
      if (t < items) {
        const int j = t / N, line = t - j * N, k = (j + m * (N / R)) * N + line;
        sg[o] = SG[k];
        sh[o] = SH[k];
      }
    }
  }
}

// position of grid point k = i_1 N + i_2 in a transform tile (row pitch N + 1)
__device__ __forceinline__ int tix(int k, int N) { return k + k / N; }

// The corrected form carries g = f - M and h = f + M as the two parts of one
// complex transform, whose rounding is relative to the larger part.  g enters
// the transforms scaled by the power of two that brings max|g| to max|h|
// (exact in any precision), so that its rounding error scales with g itself;
// the gain and L_g carry that scale and are divided by it.  Returns the
// exponent, uniform over the block (a scalar register); every thread of the
// block must take part.
template <int NOWN>
__device__ __forceinline__ int g_scale(const double (&g)[NOWN], const double (&h)[NOWN], double* red) {
  double gm = 0.0, hm = 0.0;
#pragma unroll
  for (int i = 0; i < NOWN; ++i) {
    gm = fmax(gm, fabs(g[i]));
    hm = fmax(hm, fabs(h[i]));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    gm = fmax(gm, __shfl_xor(gm, off, 64));
    hm = fmax(hm, __shfl_xor(hm, off, 64));
  }
  const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[wid] = gm;
    red[nw + wid] = hm;
  }
  __syncthreads();
  gm = 0.0;
  hm = 0.0;
  for (int w = 0; w < nw; ++w) {
    gm = fmax(gm, red[w]);
    hm = fmax(hm, red[nw + w]);
  }
  __syncthreads();
  int e = (gm > 0.0 && hm > gm) ? ilogb(hm) - ilogb(gm) : 0;
  e = e < 60 ? e : 60;
  return __builtin_amdgcn_readfirstlane(e);
}

__device__ __forceinline__ double gauss2(const double* th, double x, double y) {
  return exp(th[0] + th[1] * x + th[2] * y - th[3] * (x * x + y * y));
}

// Collision term of one cell per workgroup.  theta (corrected only) holds the
// cell's discrete Maxwellian.  mass: Q <- Q - M sum(Q) / sum(M).  T is the
// arithmetic of the transform stage (transforms, direction products and their
// accumulation); the fields g, h, M, the loss combination, Q and the mass
// projection are FP64.
template <typename T, int N>
__global__ void __launch_bounds__((v2_threads<T, N>())) __attribute__((amdgpu_waves_per_eu(v2_waves_per_eu<T, N>())))
k_q2(const double* __restrict__ f, const double* __restrict__ theta,
                                                   double* __restrict__ Q,
                                                   const double* __restrict__ nodes,
                                                   const double* __restrict__ tw_g, const double* __restrict__ ph,
                                                   int n_rho, int n_pairs,
                                                   double w_pair, const double* __restrict__ W,
                                                   const double* __restrict__ Gm, int corrected, int mass) {
  using C = cx_t<T>;
  using X = Cx<T>;
  extern __shared__ double2 smem_[];
  C* smem = reinterpret_cast<C*>(smem_);
  constexpr int K = N * N, KP = N * (N + 1);  // KP: a transform tile with padded rows
  constexpr int kThreads = v2_threads<T, N>(), kV2Own = (K + kThreads - 1) / kThreads;
  const int cell = blockIdx.x, tid = threadIdx.x;
  C* SG = smem;
  C* SH = SG + K;
  C* B0 = SH + K;
  C* B1 = B0 + KP;
  C* TW = B1 + KP;
  C* E = TW + N;  // axis phases of two consecutive pairs: [2][2][N]
  double* red = reinterpret_cast<double*>(E + 4 * N);
  for (int j = tid; j < N; j += blockDim.x) TW[j] = X::make(T(tw_g[2 * j]), T(tw_g[2 * j + 1]));
  for (int j = tid; j < 2 * N; j += blockDim.x) E[j] = X::make(T(ph[2 * j]), T(ph[2 * j + 1]));

  const double* fc = f + (size_t)cell * K;
  double th[4] = {0.0, 0.0, 0.0, 0.0};
  if (corrected)
    for (int q = 0; q < 4; ++q) th[q] = theta[(size_t)cell * 4 + q];
  double g[kV2Own], h[kV2Own], Mk[kV2Own];
#pragma unroll
  for (int i = 0; i < kV2Own; ++i) {
    const int k = tid + i * kThreads;
    g[i] = h[i] = Mk[i] = 0.0;
    if (k < K) {
      const double fv = fc[k];
      if (corrected) {
        Mk[i] = gauss2(th, nodes[k / N], nodes[k % N]);
        g[i] = fv - Mk[i];
        h[i] = fv + Mk[i];
      } else {
        g[i] = h[i] = fv;
      }
    }
  }
  const int ge = corrected ? g_scale<kV2Own>(g, h, red) : 0;
#pragma unroll
  for (int i = 0; i < kV2Own; ++i) {
    const int k = tid + i * kThreads;
    if (k < K) B0[tix(k, N)] = X::make(T(ldexp(g[i], ge)), T(h[i]));
  }
  __syncthreads();
  // spectra: Z = DFT(g + i h); gh_l = (Z_l + conj Z_-l) / 2K, hh_l = (Z_l - conj Z_-l) / 2iK,
  // Nyquist modes zeroed
  {
    const C* Z = dft2<T, N, -1>(B0, B1, TW);
    const T s = T(0.5 / K);
    for (int k = tid; k < K; k += blockDim.x) {
      const int l1 = k / N, l2 = k - l1 * N;
      const int m = ((N - l1) % N) * N + (N - l2) % N;
      const C a = Z[tix(k, N)], b = Z[tix(m, N)];
      const bool nyq = l1 == N / 2 || l2 == N / 2;
      SG[k] = nyq ? X::make(T(0), T(0)) : X::make(s * (a.x + b.x), s * (a.y - b.y));
      SH[k] = nyq ? X::make(T(0), T(0)) : X::make(s * (a.y + b.y), -s * (a.x - b.x));
    }
    __syncthreads();
  }

  // The direction-pair transforms run columns first (their inputs are read
  // along i_2 from the unpadded spectra) and leave their outputs in registers
  // (acc, ag, bh: the points of fused_point<N, kThreads, 0>); the transform of
  // acc per radial node runs rows first, so that its outputs (qr, qi: the
  // points of fused_point<N, kThreads, 1>) meet W_r along i_2.
  constexpr int OWN = fused_own<N, kThreads>();
  T qr[OWN], qi[OWN];
#pragma unroll
  for (int o = 0; o < OWN; ++o) qr[o] = qi[o] = T(0);
  // The axis phases exp(i xi_l s_a), s = rho_r sigma_p / 2, come from the table
  // ph, one pair ahead: threads below 2N load the next pair's phases while the
  // current pair is transformed and store them in the other half of E after
  // its first transform (barriers of the second transform, or the one below
  // in the plain form, order the store before the next pair's reads).
  const int n_rp = n_rho * n_pairs;
  C* ta = B1;  // (cur, oth) of the next direction-pair transform
  C* tb = B0;
  for (int r = 0; r < n_rho; ++r) {
    T acc[OWN];
#pragma unroll
    for (int o = 0; o < OWN; ++o) acc[o] = T(0);
    for (int p = 0; p < n_pairs; ++p) {
      const int rp = r * n_pairs + p;
      double nph[2] = {0.0, 0.0};
      if (tid < 2 * N && rp + 1 < n_rp) {
        const double* q = ph + ((size_t)(rp + 1) * 2 * N + tid) * 2;
        nph[0] = q[0];
        nph[1] = q[1];
      }
      const C* E0 = E + (rp & 1) * 2 * N;
      const C* E1 = E0 + N;
      T ag[OWN], bh[OWN];
      const T wp = T(w_pair), hwp = T(0.5 * w_pair);
      for (int pass = 0; pass < (corrected ? 2 : 1); ++pass) {
        const C* Xs = pass == 0 ? SG : SH;
        const C* Ys = pass == 0 ? SH : SG;
        // input u + i w at (i_1, i_2) = (e, line): u = Xs ph, w = Ys conj(ph)
        const auto ld0 = [&](int line, int e) {
          const int k = e * N + line;
          const C ph = cmul<T>(E0[e], E1[line]);
          const C u = cmul<T>(Xs[k], ph), w = cmul<T>(Ys[k], cconj<T>(ph));
          return X::make(u.x - w.y, u.y + w.x);
        };
        const auto sink = [&](int o, int, int, C t) {
          if (pass == 0) {
            ag[o] = t.x;
            bh[o] = t.y;
            if (!corrected) acc[o] += wp * t.x * t.y;
          } else {
            acc[o] += hwp * (ag[o] * bh[o] + t.x * t.y);
          }
        };
        dft2_fused<T, N, +1, kThreads, 0>(ld0, sink, ta, tb, TW);
        C* const tt = ta;
        ta = tb;
        tb = tt;
        if (pass == 0) {
          if (tid < 2 * N && rp + 1 < n_rp) E[((rp + 1) & 1) * 2 * N + tid] = X::make(T(nph[0]), T(nph[1]));
          if (!corrected) __syncthreads();
        }
      }
    }
    // Qh += W_r DFT(acc_r)
    __syncthreads();
#pragma unroll
    for (int o = 0; o < OWN; ++o) {
      const int k = fused_point<N, kThreads, 0>(o);
      if (k >= 0) B0[tix(k, N)] = X::make(acc[o], T(0));
    }
    __syncthreads();
    const double* Wr = W + (size_t)r * K;
    const auto ld0 = [&](int line, int e) { return B0[line * (N + 1) + e]; };
    const auto sink = [&](int o, int line, int e, C a) {
      const T wr = T(Wr[e * N + line]);
      qr[o] += wr * a.x;
      qi[o] += wr * a.y;
    };
    dft2_fused<T, N, -1, kThreads, 1>(ld0, sink, B0, B1, TW);
    ta = B1;  // its last pass reads B1: the next first pass writes B0
    tb = B0;
  }
  // gain = IDFT(Qh)
  double gain[kV2Own];
#pragma unroll
  for (int o = 0; o < OWN; ++o) {
    const int k = fused_point<N, kThreads, 1>(o);
    if (k >= 0) B0[tix(k, N)] = X::make(qr[o], qi[o]);
  }
  __syncthreads();
  {
    const C* G = dft2<T, N, +1>(B0, B1, TW);
#pragma unroll
    for (int i = 0; i < kV2Own; ++i) {
      const int k = tid + i * kThreads;
      gain[i] = k < K ? double(G[tix(k, N)].x) : 0.0;
    }
    __syncthreads();
  }
  // loss: IDFT(Gm hh + i Gm gh) = L_h + i L_g;  Q- = (g L_h + h L_g) / 2
  for (int k = tid; k < K; k += blockDim.x) {
    const T gm = T(Gm[k]);
    const C a = SH[k], b = SG[k];
    B0[tix(k, N)] = X::make(gm * (a.x - b.y), gm * (a.y + b.x));
  }
  __syncthreads();
  const C* Lx = dft2<T, N, +1>(B0, B1, TW);
  double q[kV2Own], sq = 0.0, sm = 0.0;
#pragma unroll
  for (int i = 0; i < kV2Own; ++i) {
    const int k = tid + i * kThreads;
    q[i] = 0.0;
    if (k < K) {
      const C l = Lx[tix(k, N)];
      q[i] = ldexp(gain[i], -ge) - 0.5 * (g[i] * double(l.x) + h[i] * ldexp(double(l.y), -ge));
      sq += q[i];
      sm += Mk[i];
    }
  }
  double c = 0.0;
  if (mass) {
    double v[2] = {sq, sm};
    block_sum<2>(v, red);
    c = v[0] / v[1];
  }
  double* Qc = Q + (size_t)cell * K;
#pragma unroll
  for (int i = 0; i < kV2Own; ++i) {
    const int k = tid + i * kThreads;
    if (k < K) Qc[k] = q[i] - c * Mk[i];
  }
}

// Carleman form for 2D Maxwell molecules, one cell per workgroup: the gain is
// sum_p IDFT(A_p fh) IDFT(B_p fh) over the M/2 half-circle directions (tables
// cw [nd][2][K]: A_p = 2 w_p psi2(xi.e_p), B_p = psi2(xi.e_p_perp)), accumulated
// in physical space; the loss is f IDFT(beta fh), beta = sum_p A_p B_p.  In the
// corrected form, Q_s(g, h): per direction one complex transform of
// A_p gh + i B_p hh gives g_a and h_b, a second one h_a and g_b, and the gain
// gains (g_a h_b + h_a g_b) / 2.  Spectra, tiles and the FP64 / FP32 split are
// those of k_q2.
template <typename T, int N>
__global__ void __launch_bounds__((v2_threads<T, N>())) __attribute__((amdgpu_waves_per_eu(c2_waves_per_eu<T, N>())))
k_c2(const double* __restrict__ f, const double* __restrict__ theta, double* __restrict__ Q,
     const double* __restrict__ nodes, const double* __restrict__ tw_g, const double* __restrict__ cw, int nd,
     const double* __restrict__ beta, int corrected, int mass) {
  using C = cx_t<T>;
  using X = Cx<T>;
  extern __shared__ double2 smem_[];
  C* smem = reinterpret_cast<C*>(smem_);
  constexpr int K = N * N, KP = N * (N + 1);
  constexpr int kThreads = v2_threads<T, N>(), kOwn = (K + kThreads - 1) / kThreads;
  const int cell = blockIdx.x, tid = threadIdx.x;
  C* SG = smem;
  C* SH = SG + K;
  C* B0 = SH + K;
  C* B1 = B0 + KP;
  C* TW = B1 + KP;
  double* red = reinterpret_cast<double*>(TW + 3 * N);
  for (int j = tid; j < N; j += blockDim.x) TW[j] = X::make(T(tw_g[2 * j]), T(tw_g[2 * j + 1]));
  const double* fc = f + (size_t)cell * K;
  double th[4] = {0.0, 0.0, 0.0, 0.0};
  if (corrected)
    for (int q = 0; q < 4; ++q) th[q] = theta[(size_t)cell * 4 + q];
  double g[kOwn], h[kOwn], Mk[kOwn];
#pragma unroll
  for (int i = 0; i < kOwn; ++i) {
    const int k = tid + i * kThreads;
    g[i] = h[i] = Mk[i] = 0.0;
    if (k < K) {
      const double fv = fc[k];
      if (corrected) {
        Mk[i] = gauss2(th, nodes[k / N], nodes[k % N]);
        g[i] = fv - Mk[i];
        h[i] = fv + Mk[i];
      } else {
        g[i] = h[i] = fv;
      }
    }
  }
  const int ge = corrected ? g_scale<kOwn>(g, h, red) : 0;
#pragma unroll
  for (int i = 0; i < kOwn; ++i) {
    const int k = tid + i * kThreads;
    if (k < K) B0[tix(k, N)] = X::make(T(ldexp(g[i], ge)), T(h[i]));
  }
  __syncthreads();
  {
    const C* Z = dft2<T, N, -1>(B0, B1, TW);
    const T s = T(0.5 / K);
    for (int k = tid; k < K; k += blockDim.x) {
      const int l1 = k / N, l2 = k - l1 * N;
      const int m = ((N - l1) % N) * N + (N - l2) % N;
      const C a = Z[tix(k, N)], b = Z[tix(m, N)];
      const bool nyq = l1 == N / 2 || l2 == N / 2;
      SG[k] = nyq ? X::make(T(0), T(0)) : X::make(s * (a.x + b.x), s * (a.y - b.y));
      SH[k] = nyq ? X::make(T(0), T(0)) : X::make(s * (a.y + b.y), -s * (a.x - b.x));
    }
    __syncthreads();
  }
  // Per direction, columns first (inputs read along i_2, tables coalesced),
  // outputs kept in registers at the points of fused_point<N, kThreads, 0>.
  constexpr int OWN = fused_own<N, kThreads>();
  C sg[spec_own<T, N, kThreads>()], sh[spec_own<T, N, kThreads>()];
  load_spec<T, N, kThreads>(SG, SH, sg, sh);
  C* ta = B1;  // (cur, oth) of the next direction transform
  C* tb = B0;
  T gacc[OWN];
#pragma unroll
  for (int o = 0; o < OWN; ++o) gacc[o] = T(0);
  for (int p = 0; p < nd; ++p) {
    const double* Ap = cw + (size_t)p * 2 * K;
    const double* Bp = Ap + K;
    T ga[OWN], hb[OWN];
    for (int pass = 0; pass < (corrected ? 2 : 1); ++pass) {
      const C* Xs = pass == 0 ? SG : SH;
      const C* Ys = pass == 0 ? SH : SG;
      const auto ld0 = [&](int o, int line, int e) {  // A u + i B w at (i_1, i_2) = (e, line)
        const int k = e * N + line;
        const T a = T(Ap[k]), b = T(Bp[k]);
        C u, w;
        if constexpr (spec_in_regs<T, N>()) {
          u = pass == 0 ? sg[o] : sh[o];
          w = pass == 0 ? sh[o] : sg[o];
        } else {
          u = Xs[k];
          w = Ys[k];
        }
        return X::make(a * u.x - b * w.y, a * u.y + b * w.x);
      };
      const auto sink = [&](int o, int, int, C t) {
        if (pass == 0) {
          ga[o] = t.x;
          hb[o] = t.y;
          if (!corrected) gacc[o] += t.x * t.y;
        } else {
          gacc[o] += T(0.5) * (ga[o] * hb[o] + t.x * t.y);
        }
      };
      dft2_fused<T, N, +1, kThreads, 0>(ld0, sink, ta, tb, TW);
      C* const tt = ta;
      ta = tb;
      tb = tt;
    }
  }
  // the gain back to the points k = tid + i * kThreads
  __syncthreads();
#pragma unroll
  for (int o = 0; o < OWN; ++o) {
    const int k = fused_point<N, kThreads, 0>(o);
    if (k >= 0) B1[tix(k, N)] = X::make(gacc[o], T(0));
  }
  __syncthreads();
  T gain[kOwn];
#pragma unroll
  for (int i = 0; i < kOwn; ++i) {
    const int k = tid + i * kThreads;
    gain[i] = k < K ? B1[tix(k, N)].x : T(0);
  }
  __syncthreads();
  // loss: IDFT(beta hh + i beta gh) = L_h + i L_g;  Q- = (g L_h + h L_g) / 2
  for (int k = tid; k < K; k += blockDim.x) {
    const T bt = T(beta[k]);
    const C a = SH[k], b = SG[k];
    B0[tix(k, N)] = X::make(bt * (a.x - b.y), bt * (a.y + b.x));
  }
  __syncthreads();
  const C* Lx = dft2<T, N, +1>(B0, B1, TW);
  double q[kOwn], sq = 0.0, sm = 0.0;
#pragma unroll
  for (int i = 0; i < kOwn; ++i) {
    const int k = tid + i * kThreads;
    q[i] = 0.0;
    if (k < K) {
      const C l = Lx[tix(k, N)];
      q[i] = ldexp(double(gain[i]), -ge) - 0.5 * (g[i] * double(l.x) + h[i] * ldexp(double(l.y), -ge));
      sq += q[i];
      sm += Mk[i];
    }
  }
  double c = 0.0;
  if (mass) {
    double v[2] = {sq, sm};
    block_sum<2>(v, red);
    c = v[0] / v[1];
  }
  double* Qc = Q + (size_t)cell * K;
#pragma unroll
  for (int i = 0; i < kOwn; ++i) {
    const int k = tid + i * kThreads;
    if (k < K) Qc[k] = q[i] - c * Mk[i];
  }
}

// 4 x 4 symmetric positive definite solve (LDL^T without pivoting)
__device__ __forceinline__ void solve_spd4(double G[4][4], const double b[4], double y[4]) {
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
}

constexpr int kMaxThreads = 256;

// sums over the cell of w phi_i exp(theta.phi~) (4 moments) and of
// w phi_i phi_j exp(theta.phi~) (10 Gram entries), phi = (1, v_1, v_2, |v|^2);
// identical in every thread
__device__ __forceinline__ void gauss_sums2(const double* th, const double* nodes, int N, double w, double* red,
                                            double (&s)[14]) {
  for (int q = 0; q < 14; ++q) s[q] = 0.0;
  for (int k = threadIdx.x; k < N * N; k += blockDim.x) {
    const double x = nodes[k / N], y = nodes[k % N], e = w * gauss2(th, x, y);
    const double ph[4] = {1.0, x, y, x * x + y * y};
    for (int i = 0; i < 4; ++i) s[i] += ph[i] * e;
    int o = 4;
    for (int i = 0; i < 4; ++i)
      for (int j = i; j < 4; ++j) s[o++] += ph[i] * ph[j] * e;
  }
  block_sum<14>(s, red);
}

// Discrete Maxwellian (eqs. discrete_conservation, discrete_Gaussian) of one
// cell per workgroup: Newton on theta = (alpha, beta_1, beta_2, gamma) from the
// continuous-moment guess, with the Gram system as Jacobian and step halving
// while the max-norm residual does not decrease; converged when it is below
// 1e-13 (|m_0| + |m_3|).
__global__ void __launch_bounds__(kMaxThreads) k_max2(const double* __restrict__ f, double* __restrict__ theta,
                                                      double* __restrict__ Mout, int32_t* __restrict__ iters,
                                                      const double* __restrict__ nodes, int N, double w) {
  __shared__ double red[14 * (kMaxThreads / 64)];
  const int K = N * N, cell = blockIdx.x;
  const double* fc = f + (size_t)cell * K;
  double t[14];
  for (int q = 0; q < 14; ++q) t[q] = 0.0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double x = nodes[k / N], y = nodes[k % N], e = w * fc[k];
    t[0] += e;
    t[1] += x * e;
    t[2] += y * e;
    t[3] += (x * x + y * y) * e;
  }
  block_sum<14>(t, red);
  const double rho = t[0], U0 = t[1] / rho, U1 = t[2] / rho;
  double T = (t[3] / rho - U0 * U0 - U1 * U1) / 2.0;
  if (!(T > 1e-3)) T = 1e-3;
  double th[4] = {log(rho / (2.0 * kPi * T)) - (U0 * U0 + U1 * U1) / (2.0 * T), U0 / T, U1 / T, 1.0 / (2.0 * T)};
  const double scale = fabs(t[0]) + fabs(t[3]) + 1e-300, tol = 1e-13;
  double s[14], r[4];
  gauss_sums2(th, nodes, N, w, red, s);
  double nrm = 0.0;
  for (int i = 0; i < 4; ++i) {
    r[i] = s[i] - t[i];
    nrm = fmax(nrm, fabs(r[i]));
  }
  if (!isfinite(nrm)) nrm = INFINITY;
  int it = 0, status = -1;
  for (; it < 60; ++it) {
    if (nrm <= tol * scale) {
      status = it;
      break;
    }
    double G[4][4], rhs[4], step[4];
    int o = 4;
    for (int i = 0; i < 4; ++i)
      for (int j = i; j < 4; ++j) G[i][j] = G[j][i] = s[o++];
    for (int i = 0; i < 4; ++i) rhs[i] = -r[i];
    solve_spd4(G, rhs, step);
    step[3] = -step[3];  // theta.phi~ carries -gamma |v|^2
    double a = 1.0, thn[4], sn[14], n_new = INFINITY;
    while (true) {
      for (int i = 0; i < 4; ++i) thn[i] = th[i] + a * step[i];
      gauss_sums2(thn, nodes, N, w, red, sn);
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
    if (dmax <= 1e-15 * (1.0 + tmax)) {
      status = nrm <= 1e-10 * scale ? it + 1 : -(it + 2);
      break;
    }
  }
  if (status == -1) status = nrm <= tol * scale ? it : -(it + 1);
  if (threadIdx.x == 0) {
    for (int i = 0; i < 4; ++i) theta[(size_t)cell * 4 + i] = th[i];
    if (iters) iters[cell] = status;
  }
  if (Mout)
    for (int k = threadIdx.x; k < K; k += blockDim.x) Mout[(size_t)cell * K + k] = gauss2(th, nodes[k / N], nodes[k % N]);
}

size_t q2_lds_bytes(int N, size_t csize) {
  return (size_t)(2 * N * N + 2 * N * (N + 1) + 5 * N) * csize + 2 * (kV2MaxThreads / 64) * 8;
}

}  // namespace

bz_status v2_maxwellian(bz_ctx* ctx, const double* f, double* theta, double* M, int32_t* iters, int64_t batch,
                        hipStream_t st) {
  if (batch == 0) return BZ_OK;
  if (batch > INT32_MAX) return set_err(ctx, BZ_EINVAL, "batch too large");
  hipLaunchKernelGGL(k_max2, dim3((unsigned)batch), dim3(kMaxThreads), 0, st, f, theta, M, iters, ctx->d_nodes,
                     ctx->N, ctx->w);
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

bz_status v2_eval_q(bz_ctx* ctx, const double* f, double* Q, int64_t batch, bool corrected, bool mass,
                    double* theta_out, hipStream_t st, void* ws_ext, size_t ws_ext_bytes) {
  if (batch == 0) return BZ_OK;
  if (batch > INT32_MAX) return set_err(ctx, BZ_EINVAL, "batch too large");
  const int N = ctx->N;
  double* th = nullptr;
  if (corrected) {
    th = theta_out;
    if (!th && ws_ext) {
      if ((size_t)batch * 4 * sizeof(double) > ws_ext_bytes)
        return set_err(ctx, BZ_EINVAL, "the Maxwellian parameters of the batch exceed the given workspace");
      th = (double*)ws_ext;
    } else if (!th) {
      bz_status s = ensure_ws(ctx, (size_t)batch * 4 * sizeof(double));
      if (s != BZ_OK) return s;
      th = (double*)ctx->ws;
    }
    bz_status s = v2_maxwellian(ctx, f, th, nullptr, nullptr, batch, st);
    if (s != BZ_OK) return s;
  }
  const bool fp32 = ctx->p.precision == BZ_FP32;
  const size_t lds = q2_lds_bytes(N, fp32 ? sizeof(float2) : sizeof(double2));
  const double w_pair = 2.0 * (2.0 * kPi / ctx->n_phi);
  const int corr = corrected ? 1 : 0, ms = mass ? 1 : 0;
  const bool carl = ctx->p.method == BZ_METHOD_CARLEMAN;
#define BZ_Q2_LAUNCH_T(TT, NN)                                                                                      \
  if (carl) {                                                                                                      \
    BZ_HIP(hipFuncSetAttribute((const void*)k_c2<TT, NN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));   \
    hipLaunchKernelGGL((k_c2<TT, NN>), dim3((unsigned)batch), dim3(v2_threads<TT, NN>()), lds, st, f, th, Q, ctx->d_nodes,      \
                       ctx->d_v2tw, ctx->d_cw, ctx->n_dir, ctx->d_cbeta, corr, ms);                                \
  } else {                                                                                                         \
    BZ_HIP(hipFuncSetAttribute((const void*)k_q2<TT, NN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));   \
    hipLaunchKernelGGL((k_q2<TT, NN>), dim3((unsigned)batch), dim3(v2_threads<TT, NN>()), lds, st, f, th, Q, ctx->d_nodes,      \
                       ctx->d_v2tw, ctx->d_v2ph, ctx->n_rho, ctx->n_phi / 2, w_pair,                                \
                       ctx->d_W, ctx->d_Gm, corr, ms);                                                             \
  }
#define BZ_Q2_LAUNCH(NN)         \
  case NN:                       \
    if (fp32) {                  \
      BZ_Q2_LAUNCH_T(float, NN)  \
    } else {                     \
      BZ_Q2_LAUNCH_T(double, NN) \
    }                            \
    break;
  switch (N) {
    BZ_Q2_LAUNCH(8)
    BZ_Q2_LAUNCH(12)
    BZ_Q2_LAUNCH(16)
    BZ_Q2_LAUNCH(24)
    BZ_Q2_LAUNCH(32)
    BZ_Q2_LAUNCH(48)
    default: return set_err(ctx, BZ_EINVAL, "d = 2 needs N in {8, 12, 16, 24, 32, 48}");
  }
#undef BZ_Q2_LAUNCH
#undef BZ_Q2_LAUNCH_T
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

}  // namespace bz
