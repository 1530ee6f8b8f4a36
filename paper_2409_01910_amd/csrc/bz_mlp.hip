// Learned warm start for the cell solve: a three-layer MLP
//   y = W3^T tanh(W2^T tanh(W1^T x + b1) + b2) + b3
// evaluated with BF16 matrix-core products (FP32 accumulation) for inference
// and FP32 matrix-core products for training (forward, backward, Adam).
//
// Features of one cell (input width K + 6): the transport inflow of eq. r
// times dx (K values), the five macroscopic moments (rho, U_1, U_2, U_3, T) of
// the previous iterate, and log10(eps).  Output: K values, the correction
// g^0 - M[f_old] divided by the model's output scale.
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "bz_common.hpp"
#include "bz_internal.hpp"

namespace bz {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}

// ------------------------------------------------------------------ GEMM
// C[i][j] (+)= sum_k A(i, k) B(k, j), A(i, k) = A[i * sai + k * sak],
// B(k, j) = B[k * sbk + j * sbj]; TI = unsigned short (BF16 bits) or float.
// 64 x 64 tile per work-group of 4 waves, each wave a 32 x 32 block of 2 x 2
// 16 x 16 matrix-core tiles; K in steps of 16 staged through LDS.  Split K:
// work-group z of the grid's third dimension sums k in [z kslice, (z+1) kslice)
// into the partial tile C + z cstride (reduced afterwards in a fixed order).
template <typename TI>
__global__ __launch_bounds__(256) void k_gemm(const TI* __restrict__ A, int64_t sai, int64_t sak,
                                              const TI* __restrict__ B, int64_t sbk, int64_t sbj,
                                              float* __restrict__ C, int64_t ldc, int M, int N, int Kall, int accumulate,
                                              int kslice, int64_t cstride) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ TI As[BM][BK + 2];
  __shared__ TI Bs[BK][BN + 2];
  const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
  const int kbeg = blockIdx.z * kslice;
  const int K = (kbeg + kslice) < Kall ? (kbeg + kslice) : Kall;
  C += (int64_t)blockIdx.z * cstride;
  const int t = threadIdx.x, wv = t >> 6, ln = t & 63;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < K; k0 += BK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + 256 * u;
      const int ii = e / BK, kk = e % BK;
      const int gi = i0 + ii, gk = k0 + kk;
      As[ii][kk] = (gi < M && gk < K) ? A[(int64_t)gi * sai + (int64_t)gk * sak] : TI(0);
      const int kb = e / BN, jj = e % BN;
      const int gkb = k0 + kb, gj = j0 + jj;
      Bs[kb][jj] = (gkb < K && gj < N) ? B[(int64_t)gkb * sbk + (int64_t)gj * sbj] : TI(0);
    }
    __syncthreads();
    const int r16 = ln & 15, g4 = ln >> 4;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int row = wr + 16 * a + r16, col = wc + 16 * b + r16;
        if constexpr (sizeof(TI) == 2) {
          s16x4 av, bv;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            av[j] = (short)As[row][4 * g4 + j];
            bv[j] = (short)Bs[4 * g4 + j][col];
          }
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[a][b], 0, 0, 0);
        } else {
#pragma unroll
          for (int kq = 0; kq < 4; ++kq)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(As[row][4 * kq + g4], Bs[4 * kq + g4][col], acc[a][b],
                                                             0, 0, 0);
        }
      }
    __syncthreads();
  }
  const int r16 = ln & 15, g4 = ln >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wr + 16 * a + 4 * g4 + r, gj = j0 + wc + 16 * b + r16;
        if (gi < M && gj < N) {
          float* c = C + (int64_t)gi * ldc + gj;
          *c = accumulate ? *c + acc[a][b][r] : acc[a][b][r];
        }
      }
}

// C[i][j] (+)= sum_z P[z][i][j] over the splits, in order (deterministic)
__global__ void k_split_reduce(const float* __restrict__ P, float* __restrict__ C, int64_t ldc, int M, int N, int S,
                               int accumulate) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)M * N) return;
  const int i = (int)(g / N), j = (int)(g % N);
  float acc = 0.f;
  for (int z = 0; z < S; ++z) acc += P[(int64_t)z * M * N + g];
  float* c = C + (int64_t)i * ldc + j;
  *c = accumulate ? *c + acc : acc;
}

// ------------------------------------------------------------------ elementwise
__global__ void k_bias_act(float* Z, const float* __restrict__ bias, int64_t rows, int cols, int act,
                           unsigned short* __restrict__ zb) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= rows * cols) return;
  float v = Z[g] + bias[g % cols];
  if (act) v = tanhf(v);
  Z[g] = v;
  if (zb) zb[g] = f2bf(v);
}

// dA = dH * (1 - H^2)
__global__ void k_tanh_back(float* dA, const float* __restrict__ dH, const float* __restrict__ H, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) dA[g] = dH[g] * (1.f - H[g] * H[g]);
}

// out[j] = sum_i D[i][j]
__global__ void k_colsum(const float* __restrict__ D, float* __restrict__ out, int64_t rows, int cols) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  double s = 0.0;
  for (int64_t i = 0; i < rows; ++i) s += D[i * cols + j];
  out[j] = (float)s;
}

// dY = 2 (Y - T) / n ; per-block partial sums of (Y - T)^2
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, float* __restrict__ dY, int64_t n,
                      double* __restrict__ part) {
  __shared__ double s_red[4];
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[1] = {0.0};
  if (g < n) {
    const float d = Y[g] - T[g];
    dY[g] = 2.f * d / (float)n;
    acc[0] = (double)d * d;
  }
  block_sum<1>(acc, s_red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_to_bf16(const float* __restrict__ x, unsigned short* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// features of one cell (block per cell); writes float and/or BF16 rows of width K + 6
// (dxs, when non-null, gives each cell its own width in place of dx)
template <int N>
__global__ __launch_bounds__(256) void k_features(const double* __restrict__ inflow, const double* __restrict__ theta,
                                                  const double* __restrict__ eps, double dx_all,
                                                  float* __restrict__ Xf, unsigned short* __restrict__ Xb,
                                                  const double* __restrict__ nodes, double w,
                                                  const double* __restrict__ dxs = nullptr) {
  constexpr int K = N * N * N, W = K + 6;
  const int b = blockIdx.x;
  const double dx = dxs ? dxs[b] : dx_all;
  const double* th = theta + (size_t)b * 5;
  const double* in = inflow + (size_t)b * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const float x = (float)(in[k] * dx);
    if (Xf) Xf[(size_t)b * W + k] = x;
    if (Xb) Xb[(size_t)b * W + k] = f2bf(x);
  }
  if (threadIdx.x == 0) {
    double s[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < N; ++i) {
        const double x = nodes[i];
        s[a] += exp(th[1 + a] * x - th[4] * x * x);
      }
    const double rho = w * exp(th[0]) * s[0] * s[1] * s[2];
    const double T = 0.5 / th[4];
    const double f[6] = {rho, th[1] * T, th[2] * T, th[3] * T, T, log10(eps[b])};
    for (int i = 0; i < 6; ++i) {
      if (Xf) Xf[(size_t)b * W + K + i] = (float)f[i];
      if (Xb) Xb[(size_t)b * W + K + i] = f2bf((float)f[i]);
    }
  }
}

// g0 = M_theta + y_scale * Y
template <int N>
__global__ __launch_bounds__(256) void k_warm_guess(const float* __restrict__ Y, const double* __restrict__ theta,
                                                    double y_scale, double* __restrict__ g0,
                                                    const double* __restrict__ nodes) {
  constexpr int K = N * N * N;
  const int b = blockIdx.x;
  const double* th = theta + (size_t)b * 5;
  __shared__ double s_E[3][N];
  if (threadIdx.x < 3 * N) {
    const int a = threadIdx.x / N, i = threadIdx.x % N;
    const double x = nodes[i];
    s_E[a][i] = exp(th[1 + a] * x - th[4] * x * x);
  }
  __syncthreads();
  const double ea = exp(th[0]);
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double M = ea * s_E[0][k / (N * N)] * s_E[1][(k / N) % N] * s_E[2][k % N];
    g0[(size_t)b * K + k] = M + y_scale * (double)Y[(size_t)b * K + k];
  }
}

// two-dimensional velocities (N x N grid, block per cell): rows of width K + 5,
// the transport part times dx, then rho, U_1, U_2, T of the cell's discrete
// Maxwellian exp(th0 + th1 x + th2 y - th3 (x^2 + y^2)), then log10(eps)
__global__ __launch_bounds__(256) void k_features2(const double* __restrict__ inflow, const double* __restrict__ theta,
                                                   const double* __restrict__ eps_c, double eps_all, double dx,
                                                   float* __restrict__ Xf, unsigned short* __restrict__ Xb,
                                                   const double* __restrict__ nodes, int N, double w) {
  const int K = N * N, W = K + 5;
  const int b = blockIdx.x;
  const double* th = theta + (size_t)b * 4;
  const double* in = inflow + (size_t)b * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const float x = (float)(in[k] * dx);
    if (Xf) Xf[(size_t)b * W + k] = x;
    if (Xb) Xb[(size_t)b * W + k] = f2bf(x);
  }
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < N; ++i) {
      const double x = nodes[i];
      s0 += exp(th[1] * x - th[3] * x * x);
      s1 += exp(th[2] * x - th[3] * x * x);
    }
    const double rho = w * exp(th[0]) * s0 * s1;
    const double T = 0.5 / th[3];
    const double e = eps_c ? eps_c[b] : eps_all;
    const double f[5] = {rho, th[1] * T, th[2] * T, T, log10(e)};
    for (int i = 0; i < 5; ++i) {
      if (Xf) Xf[(size_t)b * W + K + i] = (float)f[i];
      if (Xb) Xb[(size_t)b * W + K + i] = f2bf((float)f[i]);
    }
  }
}

// g0 = M_theta + y_scale * Y on the N x N grid
__global__ __launch_bounds__(256) void k_warm_guess2(const float* __restrict__ Y, const double* __restrict__ theta,
                                                     double y_scale, double* __restrict__ g0,
                                                     const double* __restrict__ nodes, int N) {
  const int K = N * N;
  const int b = blockIdx.x;
  const double* th = theta + (size_t)b * 4;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double x = nodes[k / N], y = nodes[k % N];
    const double M = exp(th[0] + th[1] * x + th[2] * y - th[3] * (x * x + y * y));
    g0[(size_t)b * K + k] = M + y_scale * (double)Y[(size_t)b * K + k];
  }
}

}  // namespace bz

struct bz_mlp {
  bz_ctx* ctx = nullptr;
  int n_in = 0, H = 0, n_out = 0;
  int64_t n_par = 0;
  float* p = nullptr;  // FP32 master parameters (flat)
  float* g = nullptr;  // gradient (flat)
  float* m = nullptr;  // Adam moments
  float* v = nullptr;
  unsigned short* wb = nullptr;  // BF16 copies of W1, W2, W3
  bool wb_valid = false;
  int64_t step = 0;
  double y_scale = 1.0;
  // scratch, grown with the batch
  int64_t cap = 0;
  float *h1 = nullptr, *h2 = nullptr, *y = nullptr, *d1 = nullptr, *d2 = nullptr, *dy = nullptr;
  unsigned short *xb = nullptr, *h1b = nullptr, *h2b = nullptr;
  double* part = nullptr;
  float* ksplit = nullptr;  // partial tiles of split-K products [kMaxSplit][B][max(H, ...)]
  int64_t ksplit_cap = 0;   // floats
};

namespace bz {

struct Off {
  int64_t W1, b1, W2, b2, W3, b3;
};
static Off offsets(const bz_mlp* m) {
  Off o;
  o.W1 = 0;
  o.b1 = o.W1 + (int64_t)m->n_in * m->H;
  o.W2 = o.b1 + m->H;
  o.b2 = o.W2 + (int64_t)m->H * m->H;
  o.W3 = o.b2 + m->H;
  o.b3 = o.W3 + (int64_t)m->H * m->n_out;
  return o;
}

static unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

constexpr int kMaxSplit = 64;

// Products with few output tiles and a long K (the first layer on a batch of a
// few dozen cells: 32 x 256 outputs over K = 32774) split K over up to
// kMaxSplit work-groups per tile so that the chip fills, and reduce the
// partial tiles in order afterwards; the others run as one launch.
template <typename TI>
static void gemm(const TI* A, int64_t sai, int64_t sak, const TI* B, int64_t sbk, int64_t sbj, float* C, int64_t ldc,
                 int M, int N, int K, bool acc, hipStream_t st, float* partial = nullptr, int64_t partial_cap = 0) {
  const int tiles = ((N + 63) / 64) * ((M + 63) / 64);
  int S = 1;
  if (partial && tiles < 256 && K >= 2048) {
    S = (512 + tiles - 1) / tiles;
    if (S > kMaxSplit) S = kMaxSplit;
    if (S > K / 1024) S = K / 1024;
    while (S > 1 && (int64_t)S * M * N > partial_cap) --S;
  }
  if (S <= 1) {
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
    hipLaunchKernelGGL((k_gemm<TI>), grid, dim3(256), 0, st, A, sai, sak, B, sbk, sbj, C, ldc, M, N, K, acc ? 1 : 0,
                       K, (int64_t)0);
    return;
  }
  const int kslice = ((K + S - 1) / S + 15) / 16 * 16;
  S = (K + kslice - 1) / kslice;
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)S);
  hipLaunchKernelGGL((k_gemm<TI>), grid, dim3(256), 0, st, A, sai, sak, B, sbk, sbj, partial, (int64_t)N, M, N, K, 0,
                     kslice, (int64_t)M * N);
  const int64_t n = (int64_t)M * N;
  hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, partial, C, ldc, M, N, S,
                     acc ? 1 : 0);
}

static bz_status ensure_cap(bz_mlp* mp, int64_t B) {
  bz_ctx* ctx = mp->ctx;
  if (B <= mp->cap) return BZ_OK;
  void* ptrs[] = {mp->h1, mp->h2, mp->y, mp->d1, mp->d2, mp->dy, mp->xb, mp->h1b, mp->h2b, mp->part, mp->ksplit};
  BZ_HIP(hipDeviceSynchronize());
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  const int64_t H = mp->H, O = mp->n_out, I = mp->n_in;
  BZ_HIP(hipMalloc((void**)&mp->h1, sizeof(float) * B * H));
  BZ_HIP(hipMalloc((void**)&mp->h2, sizeof(float) * B * H));
  BZ_HIP(hipMalloc((void**)&mp->y, sizeof(float) * B * O));
  BZ_HIP(hipMalloc((void**)&mp->d1, sizeof(float) * B * H));
  BZ_HIP(hipMalloc((void**)&mp->d2, sizeof(float) * B * H));
  BZ_HIP(hipMalloc((void**)&mp->dy, sizeof(float) * B * O));
  BZ_HIP(hipMalloc((void**)&mp->xb, sizeof(unsigned short) * B * I));
  BZ_HIP(hipMalloc((void**)&mp->h1b, sizeof(unsigned short) * B * H));
  BZ_HIP(hipMalloc((void**)&mp->h2b, sizeof(unsigned short) * B * H));
  BZ_HIP(hipMalloc((void**)&mp->part, sizeof(double) * ((B * O + 255) / 256)));
  // split-K partials: the products that split have M = B and N = H
  mp->ksplit_cap = (int64_t)kMaxSplit * B * H;
  BZ_HIP(hipMalloc((void**)&mp->ksplit, sizeof(float) * mp->ksplit_cap));
  mp->cap = B;
  return BZ_OK;
}

static bz_status refresh_bf16(bz_mlp* mp, hipStream_t st) {
  bz_ctx* ctx = mp->ctx;
  if (mp->wb_valid) return BZ_OK;
  const Off o = offsets(mp);
  const int64_t n1 = (int64_t)mp->n_in * mp->H, n2 = (int64_t)mp->H * mp->H, n3 = (int64_t)mp->H * mp->n_out;
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n1)), dim3(256), 0, st, mp->p + o.W1, mp->wb, n1);
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n2)), dim3(256), 0, st, mp->p + o.W2, mp->wb + n1, n2);
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n3)), dim3(256), 0, st, mp->p + o.W3, mp->wb + n1 + n2, n3);
  BZ_HIP(hipGetLastError());
  mp->wb_valid = true;
  return BZ_OK;
}

// forward; X is float [B][n_in] (FP32 path) or BF16 bits (BF16 path); output in mp->y
static bz_status forward(bz_mlp* mp, const void* X, int64_t B, bool bf16, hipStream_t st) {
  bz_ctx* ctx = mp->ctx;
  bz_status s = ensure_cap(mp, B);
  if (s != BZ_OK) return s;
  const Off o = offsets(mp);
  const int I = mp->n_in, H = mp->H, O = mp->n_out;
  if (bf16) {
    if ((s = refresh_bf16(mp, st)) != BZ_OK) return s;
    const unsigned short* W1 = mp->wb;
    const unsigned short* W2 = W1 + (int64_t)I * H;
    const unsigned short* W3 = W2 + (int64_t)H * H;
    gemm<unsigned short>((const unsigned short*)X, I, 1, W1, H, 1, mp->h1, H, (int)B, H, I, false, st, mp->ksplit, mp->ksplit_cap);
    hipLaunchKernelGGL(k_bias_act, dim3(nblk(B * H)), dim3(256), 0, st, mp->h1, mp->p + o.b1, B, H, 1, mp->h1b);
    gemm<unsigned short>(mp->h1b, H, 1, W2, H, 1, mp->h2, H, (int)B, H, H, false, st, mp->ksplit, mp->ksplit_cap);
    hipLaunchKernelGGL(k_bias_act, dim3(nblk(B * H)), dim3(256), 0, st, mp->h2, mp->p + o.b2, B, H, 1, mp->h2b);
    gemm<unsigned short>(mp->h2b, H, 1, W3, O, 1, mp->y, O, (int)B, O, H, false, st, mp->ksplit, mp->ksplit_cap);
  } else {
    gemm<float>((const float*)X, I, 1, mp->p + o.W1, H, 1, mp->h1, H, (int)B, H, I, false, st, mp->ksplit, mp->ksplit_cap);
    hipLaunchKernelGGL(k_bias_act, dim3(nblk(B * H)), dim3(256), 0, st, mp->h1, mp->p + o.b1, B, H, 1,
                       (unsigned short*)nullptr);
    gemm<float>(mp->h1, H, 1, mp->p + o.W2, H, 1, mp->h2, H, (int)B, H, H, false, st, mp->ksplit, mp->ksplit_cap);
    hipLaunchKernelGGL(k_bias_act, dim3(nblk(B * H)), dim3(256), 0, st, mp->h2, mp->p + o.b2, B, H, 1,
                       (unsigned short*)nullptr);
    gemm<float>(mp->h2, H, 1, mp->p + o.W3, O, 1, mp->y, O, (int)B, O, H, false, st, mp->ksplit, mp->ksplit_cap);
  }
  hipLaunchKernelGGL(k_bias_act, dim3(nblk(B * O)), dim3(256), 0, st, mp->y, mp->p + o.b3, B, O, 0,
                     (unsigned short*)nullptr);
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

// loss and gradient into mp->g (FP32 products); returns the loss if loss != nullptr (synchronises)
static bz_status grad(bz_mlp* mp, const float* X, const float* T, int64_t B, double* loss, hipStream_t st) {
  bz_ctx* ctx = mp->ctx;
  bz_status s = forward(mp, X, B, false, st);
  if (s != BZ_OK) return s;
  const Off o = offsets(mp);
  const int I = mp->n_in, H = mp->H, O = mp->n_out;
  const int64_t n = B * O;
  hipLaunchKernelGGL(k_mse, dim3(nblk(n)), dim3(256), 0, st, mp->y, T, mp->dy, n, mp->part);
  // dW3 = h2^T dy ; db3 = colsum(dy) ; dh2 = dy W3^T
  gemm<float>(mp->h2, 1, H, mp->dy, O, 1, mp->g + o.W3, O, H, O, (int)B, false, st, mp->ksplit, mp->ksplit_cap);
  hipLaunchKernelGGL(k_colsum, dim3(nblk(O)), dim3(256), 0, st, mp->dy, mp->g + o.b3, B, O);
  gemm<float>(mp->dy, O, 1, mp->p + o.W3, 1, O, mp->d2, H, (int)B, H, O, false, st, mp->ksplit, mp->ksplit_cap);
  hipLaunchKernelGGL(k_tanh_back, dim3(nblk(B * H)), dim3(256), 0, st, mp->d2, mp->d2, mp->h2, B * H);
  gemm<float>(mp->h1, 1, H, mp->d2, H, 1, mp->g + o.W2, H, H, H, (int)B, false, st, mp->ksplit, mp->ksplit_cap);
  hipLaunchKernelGGL(k_colsum, dim3(nblk(H)), dim3(256), 0, st, mp->d2, mp->g + o.b2, B, H);
  gemm<float>(mp->d2, H, 1, mp->p + o.W2, 1, H, mp->d1, H, (int)B, H, H, false, st, mp->ksplit, mp->ksplit_cap);
  hipLaunchKernelGGL(k_tanh_back, dim3(nblk(B * H)), dim3(256), 0, st, mp->d1, mp->d1, mp->h1, B * H);
  gemm<float>(X, 1, I, mp->d1, H, 1, mp->g + o.W1, H, I, H, (int)B, false, st, mp->ksplit, mp->ksplit_cap);
  hipLaunchKernelGGL(k_colsum, dim3(nblk(H)), dim3(256), 0, st, mp->d1, mp->g + o.b1, B, H);
  BZ_HIP(hipGetLastError());
  if (loss) {
    const int64_t nb = nblk(n);
    std::vector<double> h(nb);
    BZ_HIP(hipMemcpyAsync(h.data(), mp->part, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    BZ_HIP(hipStreamSynchronize(st));
    double sum = 0.0;
    for (double x : h) sum += x;
    *loss = sum / (double)n;
  }
  return BZ_OK;
}

}  // namespace bz

using bz::set_err;

extern "C" {

bz_status bz_mlp_create(bz_ctx* ctx, int n_in, int hidden, int n_out, uint64_t seed, bz_mlp** out) {
  if (!ctx || !out) return BZ_EINVAL;
  *out = nullptr;
  if (n_in < 1 || hidden < 1 || n_out < 1 || hidden > 4096) return set_err(ctx, BZ_EINVAL, "bad MLP sizes");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  bz_mlp* mp = new bz_mlp();
  mp->ctx = ctx;
  mp->n_in = n_in;
  mp->H = hidden;
  mp->n_out = n_out;
  const bz::Off o = bz::offsets(mp);
  mp->n_par = o.b3 + n_out;
  const size_t bytes = sizeof(float) * mp->n_par;
  if (hipMalloc((void**)&mp->p, bytes) != hipSuccess || hipMalloc((void**)&mp->g, bytes) != hipSuccess ||
      hipMalloc((void**)&mp->m, bytes) != hipSuccess || hipMalloc((void**)&mp->v, bytes) != hipSuccess ||
      hipMalloc((void**)&mp->wb, sizeof(unsigned short) *
                                     ((int64_t)n_in * hidden + (int64_t)hidden * hidden + (int64_t)hidden * n_out)) !=
          hipSuccess) {
    bz_mlp_destroy(mp);
    return set_err(ctx, BZ_ENOMEM, "MLP allocation");
  }
  // Glorot-uniform weights, zero biases (host-seeded, deterministic)
  std::vector<float> h(mp->n_par, 0.0f);
  std::mt19937_64 rng(seed);
  auto fill = [&](int64_t off, int fan_in, int fan_out) {
    const double a = std::sqrt(6.0 / (fan_in + fan_out));
    std::uniform_real_distribution<double> U(-a, a);
    for (int64_t i = 0; i < (int64_t)fan_in * fan_out; ++i) h[off + i] = (float)U(rng);
  };
  fill(o.W1, n_in, hidden);
  fill(o.W2, hidden, hidden);
  fill(o.W3, hidden, n_out);
  if (hipMemcpy(mp->p, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(mp->m, 0, bytes) != hipSuccess || hipMemset(mp->v, 0, bytes) != hipSuccess) {
    bz_mlp_destroy(mp);
    return set_err(ctx, BZ_EHIP, "MLP init");
  }
  *out = mp;
  return BZ_OK;
}

void bz_mlp_destroy(bz_mlp* mp) {
  if (!mp) return;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {mp->p, mp->g, mp->m, mp->v, mp->wb, mp->h1, mp->h2, mp->y, mp->d1, mp->d2, mp->dy,
                  mp->xb, mp->h1b, mp->h2b, mp->part, mp->ksplit};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete mp;
}

int64_t bz_mlp_num_params(bz_mlp* mp) { return mp ? mp->n_par : 0; }

bz_status bz_mlp_get_params(bz_mlp* mp, float* host, int64_t n) {
  if (!mp || !host || n != mp->n_par) return BZ_EINVAL;
  bz_ctx* ctx = mp->ctx;
  BZ_HIP(hipDeviceSynchronize());
  BZ_HIP(hipMemcpy(host, mp->p, sizeof(float) * n, hipMemcpyDeviceToHost));
  return BZ_OK;
}

bz_status bz_mlp_set_params(bz_mlp* mp, const float* host, int64_t n) {
  if (!mp || !host || n != mp->n_par) return BZ_EINVAL;
  bz_ctx* ctx = mp->ctx;
  BZ_HIP(hipDeviceSynchronize());
  BZ_HIP(hipMemcpy(mp->p, host, sizeof(float) * n, hipMemcpyHostToDevice));
  mp->wb_valid = false;
  return BZ_OK;
}

bz_status bz_mlp_set_output_scale(bz_mlp* mp, double y_scale) {
  if (!mp || !(y_scale > 0) || !std::isfinite(y_scale)) return BZ_EINVAL;
  mp->y_scale = y_scale;
  return BZ_OK;
}

bz_status bz_mlp_forward(bz_mlp* mp, const float* X, float* Y, int64_t batch, int bf16, void* stream) {
  if (!mp) return BZ_EINVAL;
  bz_ctx* ctx = mp->ctx;
  if (batch < 0 || (batch > 0 && (!X || !Y))) return set_err(ctx, BZ_EINVAL, "bad forward arguments");
  if (batch == 0) return BZ_OK;
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  bz_status s = bz::ensure_cap(mp, batch);
  if (s != BZ_OK) return s;
  const void* Xin = X;
  if (bf16) {
    const int64_t n = batch * mp->n_in;
    hipLaunchKernelGGL(bz::k_to_bf16, dim3(bz::nblk(n)), dim3(256), 0, st, X, mp->xb, n);
    Xin = mp->xb;
  }
  if ((s = bz::forward(mp, Xin, batch, bf16 != 0, st)) != BZ_OK) return s;
  BZ_HIP(hipMemcpyAsync(Y, mp->y, sizeof(float) * batch * mp->n_out, hipMemcpyDeviceToDevice, st));
  return BZ_OK;
}

bz_status bz_mlp_grad(bz_mlp* mp, const float* X, const float* T, int64_t batch, float* grad_out, double* loss,
                      void* stream) {
  if (!mp) return BZ_EINVAL;
  bz_ctx* ctx = mp->ctx;
  if (batch < 1 || !X || !T) return set_err(ctx, BZ_EINVAL, "bad gradient arguments");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  bz_status s = bz::grad(mp, X, T, batch, loss, st);
  if (s != BZ_OK) return s;
  if (grad_out) BZ_HIP(hipMemcpyAsync(grad_out, mp->g, sizeof(float) * mp->n_par, hipMemcpyDeviceToDevice, st));
  return BZ_OK;
}

bz_status bz_mlp_train_step(bz_mlp* mp, const float* X, const float* T, int64_t batch, double lr, double* loss,
                            void* stream) {
  if (!mp) return BZ_EINVAL;
  bz_ctx* ctx = mp->ctx;
  if (batch < 1 || !X || !T || !(lr > 0)) return set_err(ctx, BZ_EINVAL, "bad training arguments");
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  bz_status s = bz::grad(mp, X, T, batch, loss, st);
  if (s != BZ_OK) return s;
  mp->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)mp->step), c2 = 1.f - std::pow(b2, (float)mp->step);
  hipLaunchKernelGGL(bz::k_adam, dim3(bz::nblk(mp->n_par)), dim3(256), 0, st, mp->p, mp->g, mp->m, mp->v, mp->n_par,
                     (float)lr, b1, b2, 1e-8f, c1, c2);
  BZ_HIP(hipGetLastError());
  mp->wb_valid = false;
  return BZ_OK;
}

bz_status bz_mlp_features(bz_ctx* ctx, const double* inflow_r, const double* theta, const double* eps, double dx,
                          float* X, int64_t batch, void* stream) {
  if (!ctx) return BZ_EINVAL;
  if (batch < 0 || (batch > 0 && (!inflow_r || !theta || !eps || !X)) || !(dx > 0))
    return set_err(ctx, BZ_EINVAL, "bad feature arguments");
  if (ctx->d == 1) return set_err(ctx, BZ_EUNSUPPORTED, "a context with d = 1 serves the BGK slab only");
  if (batch == 0) return BZ_OK;
  if (hipSetDevice(ctx->p.device) != hipSuccess) return set_err(ctx, BZ_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (ctx->d == 2) {
    hipLaunchKernelGGL(bz::k_features2, dim3((unsigned)batch), dim3(256), 0, st, inflow_r, theta, eps, 0.0, dx, X,
                       (unsigned short*)nullptr, ctx->d_nodes, ctx->N, ctx->w);
    BZ_HIP(hipGetLastError());
    return BZ_OK;
  }
  switch (ctx->N) {
    case 8: hipLaunchKernelGGL((bz::k_features<8>), dim3((unsigned)batch), dim3(256), 0, st, inflow_r, theta, eps, dx, X, (unsigned short*)nullptr, ctx->d_nodes, ctx->w); break;
    case 16: hipLaunchKernelGGL((bz::k_features<16>), dim3((unsigned)batch), dim3(256), 0, st, inflow_r, theta, eps, dx, X, (unsigned short*)nullptr, ctx->d_nodes, ctx->w); break;
    case 32: hipLaunchKernelGGL((bz::k_features<32>), dim3((unsigned)batch), dim3(256), 0, st, inflow_r, theta, eps, dx, X, (unsigned short*)nullptr, ctx->d_nodes, ctx->w); break;
    default: return set_err(ctx, BZ_EUNSUPPORTED, "N");
  }
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

}  // extern "C"

namespace bz {

// learned initial guesses of a batch: features (BF16) -> MLP (BF16 products) -> g0
bz_status learned_guess(bz_ctx* ctx, bz_mlp* mp, const double* inflow_r, const double* theta, const double* eps,
                        double dx, double* g0, int64_t batch, hipStream_t st) {
  if (mp->n_in != ctx->K + 6 || mp->n_out != ctx->K) return set_err(ctx, BZ_EINVAL, "MLP sizes do not match K");
  bz_status s = ensure_cap(mp, batch);
  if (s != BZ_OK) return s;
  switch (ctx->N) {
    case 8: hipLaunchKernelGGL((k_features<8>), dim3((unsigned)batch), dim3(256), 0, st, inflow_r, theta, eps, dx, (float*)nullptr, mp->xb, ctx->d_nodes, ctx->w); break;
    case 16: hipLaunchKernelGGL((k_features<16>), dim3((unsigned)batch), dim3(256), 0, st, inflow_r, theta, eps, dx, (float*)nullptr, mp->xb, ctx->d_nodes, ctx->w); break;
    case 32: hipLaunchKernelGGL((k_features<32>), dim3((unsigned)batch), dim3(256), 0, st, inflow_r, theta, eps, dx, (float*)nullptr, mp->xb, ctx->d_nodes, ctx->w); break;
    default: return set_err(ctx, BZ_EUNSUPPORTED, "N");
  }
  if ((s = forward(mp, mp->xb, batch, true, st)) != BZ_OK) return s;
  switch (ctx->N) {
    case 8: hipLaunchKernelGGL((k_warm_guess<8>), dim3((unsigned)batch), dim3(256), 0, st, mp->y, theta, mp->y_scale, g0, ctx->d_nodes); break;
    case 16: hipLaunchKernelGGL((k_warm_guess<16>), dim3((unsigned)batch), dim3(256), 0, st, mp->y, theta, mp->y_scale, g0, ctx->d_nodes); break;
    case 32: hipLaunchKernelGGL((k_warm_guess<32>), dim3((unsigned)batch), dim3(256), 0, st, mp->y, theta, mp->y_scale, g0, ctx->d_nodes); break;
  }
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

// the learned candidates of a batch of cells with per-cell eps and dx (the
// slab scans): features (BF16) -> MLP (BF16 products) -> G = M_theta + scale y
bz_status ws_candidates(bz_ctx* ctx, bz_mlp* mp, const double* inflow, const double* theta, const double* eps,
                        const double* dxs, double* G, int64_t batch, hipStream_t st) {
  if (mp->n_in != ctx->K + 6 || mp->n_out != ctx->K) return set_err(ctx, BZ_EINVAL, "MLP sizes do not match K");
  bz_status s = ensure_cap(mp, batch);
  if (s != BZ_OK) return s;
  switch (ctx->N) {
    case 8: hipLaunchKernelGGL((k_features<8>), dim3((unsigned)batch), dim3(256), 0, st, inflow, theta, eps, 0.0, (float*)nullptr, mp->xb, ctx->d_nodes, ctx->w, dxs); break;
    case 16: hipLaunchKernelGGL((k_features<16>), dim3((unsigned)batch), dim3(256), 0, st, inflow, theta, eps, 0.0, (float*)nullptr, mp->xb, ctx->d_nodes, ctx->w, dxs); break;
    case 32: hipLaunchKernelGGL((k_features<32>), dim3((unsigned)batch), dim3(256), 0, st, inflow, theta, eps, 0.0, (float*)nullptr, mp->xb, ctx->d_nodes, ctx->w, dxs); break;
    default: return set_err(ctx, BZ_EUNSUPPORTED, "N");
  }
  if ((s = forward(mp, mp->xb, batch, true, st)) != BZ_OK) return s;
  switch (ctx->N) {
    case 8: hipLaunchKernelGGL((k_warm_guess<8>), dim3((unsigned)batch), dim3(256), 0, st, mp->y, theta, mp->y_scale, G, ctx->d_nodes); break;
    case 16: hipLaunchKernelGGL((k_warm_guess<16>), dim3((unsigned)batch), dim3(256), 0, st, mp->y, theta, mp->y_scale, G, ctx->d_nodes); break;
    case 32: hipLaunchKernelGGL((k_warm_guess<32>), dim3((unsigned)batch), dim3(256), 0, st, mp->y, theta, mp->y_scale, G, ctx->d_nodes); break;
  }
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

// the learned candidates of a batch of cells with two-dimensional velocities,
// one eps and one dx: features (BF16) -> MLP (BF16 products) -> G = M_theta + scale y
bz_status ws_candidates2(bz_ctx* ctx, bz_mlp* mp, const double* inflow, const double* theta, double eps, double dx,
                         double* G, int64_t batch, hipStream_t st) {
  if (mp->n_in != ctx->K + 5 || mp->n_out != ctx->K) return set_err(ctx, BZ_EINVAL, "MLP sizes do not match K");
  bz_status s = ensure_cap(mp, batch);
  if (s != BZ_OK) return s;
  hipLaunchKernelGGL(k_features2, dim3((unsigned)batch), dim3(256), 0, st, inflow, theta, (const double*)nullptr, eps,
                     dx, (float*)nullptr, mp->xb, ctx->d_nodes, ctx->N, ctx->w);
  if ((s = forward(mp, mp->xb, batch, true, st)) != BZ_OK) return s;
  hipLaunchKernelGGL(k_warm_guess2, dim3((unsigned)batch), dim3(256), 0, st, mp->y, theta, mp->y_scale, G,
                     ctx->d_nodes, ctx->N);
  BZ_HIP(hipGetLastError());
  return BZ_OK;
}

// sizes the network's scratch for `batch` rows and its BF16 weight copies, so
// that later candidates make no allocation (graph capture of sweeps)
bz_status ws_prepare(bz_mlp* mp, int64_t batch, hipStream_t st) {
  bz_status s = ensure_cap(mp, batch);
  if (s != BZ_OK) return s;
  return refresh_bf16(mp, st);
}

bz_ctx* ws_ctx(bz_mlp* mp) { return mp->ctx; }
int ws_n_in(bz_mlp* mp) { return mp->n_in; }
int ws_n_out(bz_mlp* mp) { return mp->n_out; }

}  // namespace bz
