// Device helpers shared by the film and bulk kernels: row transforms (real
// <-> half-spectrum along x), strided column transforms, block reductions.
#pragma once
#include "fft.h"

// Minimum resident waves per SIMD promised to the compiler (it then keeps the
// register count within 512 / n).
#ifndef MAG_WAVES_PER_EU
#define MAG_WAVES_PER_EU(...) __attribute__((amdgpu_waves_per_eu(__VA_ARGS__)))
#endif

namespace mag {

constexpr int kLdsBudget = 64 * 1024;   // bytes of LDS per work-group for FFT scratch

// ---------------------------------------------------------------- launch shapes
constexpr int pow2floor(int v) { return v < 2 ? 1 : 2 * pow2floor(v / 2); }

// Row transforms: a real row of length 2M is a complex pencil of length M,
// LDS pitch M + M/16 (padding breaks the stride-R bank pattern of the
// Stockham writes).
template <int M, typename T>
struct RowShape {
  static constexpr int TT = Plan<M>::TT;
  static constexpr int PITCH = M + M / 16;
  static constexpr int PT = (256 / TT) > 0 ? (256 / TT) : 1;
  static constexpr int PL = pow2floor(kLdsBudget / (2 * (int)sizeof(T) * PITCH));
  static constexpr int P = PT < PL ? PT : PL;          // rows per block
  static constexpr int THREADS = P * TT;
};

// Column transforms: P pencils per block, consecutive pencils on consecutive lanes.
template <int N, typename T>
struct ColShape {
  static constexpr int TT = Plan<N>::TT;
  static constexpr int PW = sizeof(T) == 8 ? 8 : 16;         // 128-byte rows of complex
  static constexpr int PL = kLdsBudget / (N * 2 * (int)sizeof(T));
  static constexpr int PT = 1024 / TT;
  static constexpr int P0 = PW < PL ? PW : PL;
  static constexpr int P = (P0 < PT ? P0 : PT) > 0 ? (P0 < PT ? P0 : PT) : 1;
  static constexpr int THREADS = P * TT;
};

// ---------------------------------------------------------------- reductions
// Fixed-order block sum of one double per thread; result valid in thread 0.
template <int THREADS>
__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

// Sum of part[0..n) in a fixed order that does not depend on the block size
// (THREADS >= 256): 256 strided partial sums, then a pairwise tree.  Every
// block of every kernel that calls it on the same data gets the same bits,
// and so does a one-block finalize kernel that sums the same way.
template <int THREADS>
__device__ __forceinline__ double fixed_sum256(const double *__restrict__ part, int n, double *sh) {
  static_assert(THREADS >= 256, "fixed_sum256 needs at least 256 threads");
  const int t = threadIdx.x;
  if (t < 256) {
    double s = 0.0;
    for (int i = t; i < n; i += 256) s += part[i];
    sh[t] = s;
  }
  __syncthreads();
#pragma unroll
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Sum over the 64 lanes of a wavefront by an xor butterfly: every lane ends
// with the same bits (each step adds two equal-order partial sums).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Sum of part[0..n) computed by one wavefront in a fixed order (lane l adds
// part[l], part[l+64], ... in index order, then the butterfly): every wavefront of every block
// that calls it on the same data gets the same bits, with no barrier.
__device__ __forceinline__ double parts_sum(const double *__restrict__ part, int n) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  int i = lane;
  // eight loads in flight per lane, added in index order
  for (; i + 7 * 64 < n; i += 8 * 64) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[i + u * 64];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; i < n; i += 64) s += part[i];
  return wave_sum(s);
}

// Block total of one double per thread (fixed order: butterfly per wavefront,
// then the wavefront sums in order); valid in thread 0.  sh: THREADS / 64
// doubles.  Contains one barrier.
template <int THREADS>
__device__ __forceinline__ double block_total(double v, double *sh) {
  constexpr int NW = (THREADS + 63) / 64;
  const double w = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NW; ++i) s += sh[i];
  }
  return s;
}

// ---------------------------------------------------------------- row helpers
// After a length-M forward FFT of z[m] = x[2m] + i x[2m+1] (thread j holds
// Z[j + rho TT] in v), form the half spectrum X[k], k = 0..M, of the real row:
// X[k] = (Z[k] + conj Z[M-k])/2 - (i/2) W^k (Z[k] - conj Z[M-k]), W = exp(-2 pi i / 2M).
// Writes X to dst[0..M].  lre/lim: the row's LDS scratch (M entries).
template <int M, typename T>
__device__ __forceinline__ void r2c_finish(const cx<T> *v, int j, T *lre, T *lim,
                                           const cx<T> *__restrict__ twN, cx<T> *dst,
                                           bool active) {
  constexpr int RMAX = Plan<M>::RMAX, TT = Plan<M>::TT;
  __syncthreads();
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int k = j + rho * TT;
    lre[k] = v[rho].x;
    lim[k] = v[rho].y;
  }
  __syncthreads();
  if (!active) return;
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int k = j + rho * TT;
    const int km = (M - k) & (M - 1);
    const cx<T> zk = v[rho];
    const cx<T> zm = {lre[km], -lim[km]};            // conj Z[M-k]
    const cx<T> s = zk + zm, d = zk - zm;
    const cx<T> w = twN[k];                          // W^k
    const cx<T> wd = cmul(w, d);                     // W^k (Z - conj Z')
    // X = s/2 - (i/2) wd = (s.x + wd.y)/2 + i (s.y - wd.x)/2
    dst[k] = {(T)0.5 * (s.x + wd.y), (T)0.5 * (s.y - wd.x)};
  }
  if (j == 0) {
    const cx<T> z0 = v[0];
    dst[M] = {z0.x - z0.y, (T)0};
  }
}

// Before a length-M inverse FFT: from the half spectrum X[0..M] build
// Z[k] = (X[k] + conj X[M-k]) + i W^{-k} (X[k] - conj X[M-k]) for k = j + rho TT.
// The inverse transform of Z yields x[2m] + i x[2m+1] scaled by 2M.
template <int M, typename T>
__device__ __forceinline__ void c2r_start(cx<T> *v, int j, const cx<T> *src,
                                          const cx<T> *__restrict__ twN, bool active) {
  constexpr int RMAX = Plan<M>::RMAX, TT = Plan<M>::TT;
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int k = j + rho * TT;
    if (!active) {
      v[rho] = {(T)0, (T)0};
      continue;
    }
    const cx<T> xk = src[k];
    const cx<T> xm = src[M - k];
    const cx<T> s = {xk.x + xm.x, xk.y - xm.y};       // X[k] + conj X[M-k]
    const cx<T> d = {xk.x - xm.x, xk.y + xm.y};       // X[k] - conj X[M-k]
    const cx<T> wd = cmulc(d, twN[k]);                // W^{-k} d
    v[rho] = {s.x - wd.y, s.y + wd.x};                // s + i wd
  }
}

}  // namespace mag
