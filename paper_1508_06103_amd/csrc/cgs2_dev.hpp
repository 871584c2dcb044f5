// Device bodies of the fused classical Gram-Schmidt passes, shared by the
// single-solve kernels and the batched ones: each workgroup of 256 threads
// (four wavefronts) takes one element range [lo, hi) and leaves per-range
// partial sums that a second stage adds in a fixed order.
#pragma once

#include "common.hpp"

namespace stkkt {

constexpr int kCgsThreads = 256;
constexpr int kCgsMaxK = 64;   // basis vectors a fused pass accepts
constexpr int kCgsHalf = 32;

__device__ inline double cgs_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Tiles of one wavefront: lanes are elements, a wavefront takes 64-element
// tiles; the KR >= k basis entries of a tile are loaded once into registers
// and serve both the update and the dots, so V is read once.  The
// wavefront's dot sums go to red[wave][g].
template <int KR>
__device__ inline void update_dot_tiles(double *__restrict__ w, const double *__restrict__ V, long long ldv, int k,
                                        cptr<double> hc, long long lo, long long hi,
                                        double (*red)[kCgsMaxK]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long ntiles = (hi - lo + 63) / 64;
  double acc[KR];
#pragma unroll
  for (int j = 0; j < KR; ++j) acc[j] = 0.0;
  for (long long t = wave; t < ntiles; t += kCgsThreads / 64) {
    const long long e = lo + 64 * t + lane;
    const bool valid = e < hi;
    double v[KR];
#pragma unroll
    for (int j = 0; j < KR; ++j) v[j] = (j < k && valid) ? V[(long long)j * ldv + e] : 0.0;
    const double wold = valid ? w[e] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < KR; ++j)
      if (j < k) s += hc[j] * v[j];
    const double wn = valid ? wold - s : 0.0;
    if (valid) w[e] = wn;
#pragma unroll
    for (int j = 0; j < KR; ++j) acc[j] += v[j] * wn;
  }
#pragma unroll
  for (int j = 0; j < KR; ++j)
    if (j < k) {
      const double r = cgs_wave_sum(acc[j]);
      if (lane == 0) red[wave][j] = r;
    }
}

// out[g * ostride] = sum over [lo, hi) of V_g[e] w[e], g < k <= KR: the same
// tiles as the update+dot, without the update (the first CGS pass).
template <int KR>
__device__ inline void dot_range(const double *__restrict__ w, const double *__restrict__ V, long long ldv, int k,
                                 long long lo, long long hi, double *__restrict__ out, long long ostride) {
  __shared__ double red[kCgsThreads / 64][kCgsMaxK];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long ntiles = (hi - lo + 63) / 64;
  double acc[KR];
#pragma unroll
  for (int j = 0; j < KR; ++j) acc[j] = 0.0;
  for (long long t = wave; t < ntiles; t += kCgsThreads / 64) {
    const long long e = lo + 64 * t + lane;
    const bool valid = e < hi;
    const double we = valid ? w[e] : 0.0;
#pragma unroll
    for (int j = 0; j < KR; ++j) acc[j] += ((j < k && valid) ? V[(long long)j * ldv + e] : 0.0) * we;
  }
#pragma unroll
  for (int j = 0; j < KR; ++j)
    if (j < k) {
      const double r = cgs_wave_sum(acc[j]);
      if (lane == 0) red[wave][j] = r;
    }
  __syncthreads();
  if ((int)threadIdx.x < k) {
    double s = 0.0;
#pragma unroll
    for (int wv = 0; wv < kCgsThreads / 64; ++wv) s += red[wv][threadIdx.x];
    out[(long long)threadIdx.x * ostride] = s;
  }
}

// w[e] <- w[e] - sum_{g<k} h[g] V_g[e] for e in [lo, hi), then
// out[g * ostride] = sum over the range of V_g[e] w_new[e], g < k <= KR.
// Every wavefront works on its own tiles with no synchronisation.  Kernels
// are instantiated with KR = 32, 48, 56 and 64 (the smallest KR >= k: more
// registers per wavefront, fewer wavefronts per SIMD, more loads in flight
// per wavefront).
template <int KR>
__device__ inline void update_dot_range(double *__restrict__ w, const double *__restrict__ V, long long ldv, int k,
                                        const double *__restrict__ h, long long lo, long long hi,
                                        double *__restrict__ out, long long ostride) {
  __shared__ double red[kCgsThreads / 64][kCgsMaxK];
  update_dot_tiles<KR>(w, V, ldv, k, as_const(h), lo, hi, red);
  __syncthreads();
  if ((int)threadIdx.x < k) {
    double s = 0.0;
#pragma unroll
    for (int wv = 0; wv < kCgsThreads / 64; ++wv) s += red[wv][threadIdx.x];
    out[(long long)threadIdx.x * ostride] = s;
  }
}

// w[e] <- w[e] - sum_{g<k} h[g] V_g[e] for e in [lo, hi); returns (in thread
// 0) the range's sum of w_new[e]^2.
// The basis entries of an element are loaded together (up to KR, KR >= k;
// instantiated like the update+dot) before the sum, in the same order.
template <int KR>
__device__ inline double update_norm_range(double *__restrict__ w, const double *__restrict__ V, long long ldv, int k,
                                           const double *__restrict__ h, long long lo, long long hi) {
  __shared__ double red[kCgsThreads / 64];
  const cptr<double> hc = as_const(h);
  double acc = 0.0;
  for (long long e = lo + threadIdx.x; e < hi; e += kCgsThreads) {
    double v[KR];
#pragma unroll
    for (int g = 0; g < KR; ++g) v[g] = g < k ? V[(long long)g * ldv + e] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int g = 0; g < KR; ++g)
      if (g < k) s += hc[g] * v[g];
    const double wn = w[e] - s;
    w[e] = wn;
    acc += wn * wn;
  }
  acc = cgs_wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int wv = 0; wv < kCgsThreads / 64; ++wv) s += red[wv];
  return s;
}

}  // namespace stkkt
