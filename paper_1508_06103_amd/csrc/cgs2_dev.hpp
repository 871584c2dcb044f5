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

// w[e] <- w[e] - sum_{g<k} h[g] V_g[e] for e in [lo, hi), then
// out[g * ostride] = sum over the range of V_g[e] w_new[e], g < k (k <= 64).
//
// Lanes are elements and a wavefront takes 64-element tiles; the basis
// entries of a tile are loaded once into registers and serve both the update
// and the dots, so V is read once.  Up to 32 basis vectors every wavefront
// works on its own tiles with no synchronisation.  Above 32 the two
// wavefronts of a pair share a tile, each holding half of the basis entries,
// and add their halves of the update sum through LDS (one barrier per tile).
__device__ inline void update_dot_range(double *__restrict__ w, const double *__restrict__ V, long long ldv, int k,
                                        const double *__restrict__ h, long long lo, long long hi,
                                        double *__restrict__ out, long long ostride) {
  __shared__ double sp[2][kCgsThreads / 64][64];
  __shared__ double red[kCgsThreads / 64][kCgsMaxK];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const cptr<double> hc = as_const(h);
  const long long ntiles = (hi - lo + 63) / 64;
  double acc[kCgsHalf];
#pragma unroll
  for (int j = 0; j < kCgsHalf; ++j) acc[j] = 0.0;
  if (k <= kCgsHalf) {
    for (long long t = wave; t < ntiles; t += kCgsThreads / 64) {
      const long long e = lo + 64 * t + lane;
      const bool valid = e < hi;
      double v[kCgsHalf];
#pragma unroll
      for (int j = 0; j < kCgsHalf; ++j) v[j] = (j < k && valid) ? V[(long long)j * ldv + e] : 0.0;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < kCgsHalf; ++j)
        if (j < k) s += hc[j] * v[j];
      const double wn = valid ? w[e] - s : 0.0;
      if (valid) w[e] = wn;
#pragma unroll
      for (int j = 0; j < kCgsHalf; ++j) acc[j] += v[j] * wn;
    }
#pragma unroll
    for (int j = 0; j < kCgsHalf; ++j)
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
    return;
  }
  const int pair = wave >> 1, half = wave & 1;
  const int g0 = kCgsHalf * half;
  const int kh = k - g0 < kCgsHalf ? k - g0 : kCgsHalf;   // basis vectors of this half
  const long long niter = (ntiles + 1) / 2;                // the same count for every wavefront
  for (long long it = 0; it < niter; ++it) {
    const long long t = pair + 2 * it;
    const long long e = lo + 64 * t + lane;
    const bool valid = t < ntiles && e < hi;
    double v[kCgsHalf];
#pragma unroll
    for (int j = 0; j < kCgsHalf; ++j) v[j] = (j < kh && valid) ? V[(long long)(g0 + j) * ldv + e] : 0.0;
    // w is read before the barrier: only this pass writes it, after the barrier
    const double wold = valid ? w[e] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kCgsHalf; ++j)
      if (j < kh) s += hc[g0 + j] * v[j];
    const int b = (int)(it & 1);
    sp[b][wave][lane] = s;
    __syncthreads();
    const double stot = sp[b][2 * pair][lane] + sp[b][2 * pair + 1][lane];
    const double wn = valid ? wold - stot : 0.0;
    if (valid && half == 0) w[e] = wn;
#pragma unroll
    for (int j = 0; j < kCgsHalf; ++j) acc[j] += v[j] * wn;
  }
#pragma unroll
  for (int j = 0; j < kCgsHalf; ++j)
    if (j < kh) {
      const double r = cgs_wave_sum(acc[j]);
      if (lane == 0) red[wave][g0 + j] = r;
    }
  __syncthreads();
  if ((int)threadIdx.x < k) {
    const int hf = (int)threadIdx.x >= kCgsHalf ? 1 : 0;
    out[(long long)threadIdx.x * ostride] = red[hf][threadIdx.x] + red[2 + hf][threadIdx.x];
  }
}

// w[e] <- w[e] - sum_{g<k} h[g] V_g[e] for e in [lo, hi); returns (in thread
// 0) the range's sum of w_new[e]^2.
__device__ inline double update_norm_range(double *__restrict__ w, const double *__restrict__ V, long long ldv, int k,
                                           const double *__restrict__ h, long long lo, long long hi) {
  __shared__ double red[kCgsThreads / 64];
  const cptr<double> hc = as_const(h);
  double acc = 0.0;
  for (long long e = lo + threadIdx.x; e < hi; e += kCgsThreads) {
    double s = 0.0;
    for (int g = 0; g < k; ++g) s += hc[g] * V[(long long)g * ldv + e];
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
