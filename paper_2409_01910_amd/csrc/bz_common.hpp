// Shared device helpers of the bz HIP library (gfx950, wave64).
//
// * compile-time twiddle tables (cos/sin of 2 pi j / n evaluated by constexpr
//   Taylor series after exact octant reduction),
// * an in-register radix-2 FFT of N points per lane (N = 8, 16, 32),
// * wave and block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bz {

constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int k = 1; k < 12; ++k) {
    t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 12; ++k) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}
constexpr double sin_turn(double x);
// cos(2 pi x) for x in [0, 1), reduced exactly to |2 pi x| <= pi/4
constexpr double cos_turn(double x) {
  return x > 0.5 ? cos_turn(1.0 - x)
         : x > 0.25 ? -cos_turn(0.5 - x)
         : x > 0.125 ? sin_turn(0.25 - x)
                     : taylor_cos(2.0 * kPi * x);
}
constexpr double sin_turn(double x) {
  return x > 0.5 ? -sin_turn(1.0 - x)
         : x > 0.25 ? sin_turn(0.5 - x)
         : x > 0.125 ? cos_turn(0.25 - x)
                     : taylor_sin(2.0 * kPi * x);
}

template <int N>
struct Twiddle {
  double c[N];
  double s[N];
  constexpr Twiddle() : c(), s() {
    for (int k = 0; k < N; ++k) {
      c[k] = cos_turn(double(k) / N);
      s[k] = sin_turn(double(k) / N);
    }
  }
};

template <int N>
constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < N; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// In-register DFT of N points held by one lane:
//   X_l = sum_j x_j exp(SIGN * 2 pi i l j / N)   (SIGN = -1 forward, +1 inverse,
// no normalisation).  Radix-2 decimation in time; all indices are compile-time
// constants after unrolling, so re[] / im[] stay in VGPRs and twiddles fold
// into immediates.  A general twiddle w = c + i s enters its butterfly as a
// scaled rotation: for x = a + i b, x w = c ((a - t b) + i (b + t a)) with
// t = s / c when |s| <= |c|, else x w = s ((u a - b) + i (a + u b)) with
// u = c / s, so that the scale c or s folds into the butterfly's fused
// multiply-adds (6 instructions per butterfly instead of 8; the ratio is at
// most 1 in magnitude).
template <typename T, int N, int SIGN>
__device__ __forceinline__ void fft_reg(T* re, T* im) {
  constexpr Twiddle<N> tw{};
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int j = bitrev<N>(i);
    if (j > i) {
      T t = re[i];
      re[i] = re[j];
      re[j] = t;
      t = im[i];
      im[i] = im[j];
      im[j] = t;
    }
  }
#pragma unroll
  for (int half = 1; half < N; half <<= 1) {
#pragma unroll
    for (int k = 0; k < half; ++k) {
      const int idx = k * (N / (2 * half));
      const T c = T(tw.c[idx]);
      const T s = T(SIGN * tw.s[idx]);
#pragma unroll
      for (int i = k; i < N; i += 2 * half) {
        const int j = i + half;
        if (k != 0 && 4 * k != 2 * half) {
          const double cd = tw.c[idx], sd = SIGN * tw.s[idx];
          T yr, yi, m;
          if (cd * cd >= sd * sd) {
            const T t = T(sd / cd);
            yr = re[j] - t * im[j];
            yi = im[j] + t * re[j];
            m = c;
          } else {
            const T u = T(cd / sd);
            yr = re[j] * u - im[j];
            yi = re[j] + im[j] * u;
            m = s;
          }
          re[j] = re[i] - m * yr;
          im[j] = im[i] - m * yi;
          re[i] = re[i] + m * yr;
          im[i] = im[i] + m * yi;
          continue;
        }
        T xr, xi;
        if (k == 0) {
          xr = re[j];
          xi = im[j];
        } else {  // w = SIGN * i
          xr = -T(SIGN) * im[j];
          xi = T(SIGN) * re[j];
        }
        re[j] = re[i] - xr;
        im[j] = im[i] - xi;
        re[i] += xr;
        im[i] += xi;
      }
    }
  }
}

// BGK-penalty frequency of eq. Pf: nu = 4 pi rho <|g|^gamma>, the binary loss
// frequency averaged over pairs from the cell's Maxwellian, whose temperature
// parameter is T = 1 / (2 theta_4); gfac = 4^{gamma/2} Gamma((3 + gamma)/2) / Gamma(3/2).
// For Maxwell molecules (gamma = 0) it is 4 pi rho exactly.
__device__ __forceinline__ double penalty_nu(double rho, double theta4, double gam, double gfac) {
  return gam == 0.0 ? 4.0 * kPi * rho : 4.0 * kPi * rho * gfac * pow(0.5 / theta4, 0.5 * gam);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// DPP lane move of a double (both 32-bit halves); lanes the row mask leaves
// out, and lanes whose source is out of range, receive 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_move(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, ROW_MASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, ROW_MASK, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sums of NV values over each 32-lane half of the wave, with DPP row moves
// instead of LDS permutes: quad exchanges, two row rotations (16-lane row
// sums), then row 0 into row 1 and row 2 into row 3.  lo[q] = sum over lanes
// 0..31, hi[q] = sum over lanes 32..63, both in every lane.
template <int NV>
__device__ __forceinline__ void half_wave_sums(double (&v)[NV], double (&lo)[NV], double (&hi)[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] += dpp_move<0xB1>(v[q]);  // quad_perm [1,0,3,2]
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] += dpp_move<0x4E>(v[q]);  // quad_perm [2,3,0,1]
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] += dpp_move<0x124>(v[q]);  // row_ror:4
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] += dpp_move<0x128>(v[q]);  // row_ror:8
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] += dpp_move<0x142, 0xA>(v[q]);  // row_bcast:15 into rows 1, 3
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    lo[q] = read_lane(v[q], 31);
    hi[q] = read_lane(v[q], 63);
  }
}

// Sums of NV values over the whole wave with DPP row moves: quad exchanges and
// two row rotations give 16-lane row sums, row 0 is added into row 1 and row 2
// into row 3, then lane 31 into rows 2 and 3; lane 63 holds the total.  Full
// wave only.
template <int NV>
__device__ __forceinline__ void wave_sums_dpp(double (&v)[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] += dpp_move<0xB1>(v[q]);
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] += dpp_move<0x4E>(v[q]);
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] += dpp_move<0x124>(v[q]);
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] += dpp_move<0x128>(v[q]);
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] += dpp_move<0x142, 0xA>(v[q]);  // row_bcast:15 into rows 1, 3
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] += dpp_move<0x143, 0xC>(v[q]);  // row_bcast:31 into rows 2, 3
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = read_lane(v[q], 63);
}

// Deterministic block sum of NV values per thread; result valid in all threads.
// scratch must hold NV * (blockDim.x / 64) doubles.  Every thread of the block
// must take part.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  wave_sums_dpp<NV>(v);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) scratch[q * nw + wid] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += scratch[q * nw + w];
    v[q] = s;
  }
  __syncthreads();
}

}  // namespace bz
