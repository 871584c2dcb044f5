// FP64 vector kernels for the Krylov solvers: fixed-order two-stage
// reductions (reproducible run to run) built on wavefront shuffles, and the
// streaming updates of classical Gram-Schmidt.
#include "common.hpp"
#include "krylov.hpp"

namespace stkkt {

namespace {

constexpr int kThreads = 256;
constexpr int kGroup = 8;   // vectors per pass of the multi-dot

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// partial[i * G + b] = sum over block b's elements of V_i[e] * w[e], i < k.
__global__ void __launch_bounds__(kThreads) multidot_kernel(const double *__restrict__ V, long long ldv, int k,
                                                            const double *__restrict__ w, long long n,
                                                            double *__restrict__ partial) {
  __shared__ double red[kGroup][kThreads / 64];
  const int G = gridDim.x;
  const long long per = (n + G - 1) / G;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = lo + per < n ? lo + per : n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i0 = 0; i0 < k; i0 += kGroup) {
    const int gk = k - i0 < kGroup ? k - i0 : kGroup;
    double acc[kGroup];
#pragma unroll
    for (int g = 0; g < kGroup; ++g) acc[g] = 0.0;
    for (long long e = lo + threadIdx.x; e < hi; e += kThreads) {
      const double we = w[e];
#pragma unroll
      for (int g = 0; g < kGroup; ++g)
        if (g < gk) acc[g] += V[(long long)(i0 + g) * ldv + e] * we;
    }
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
      const double s = wave_sum(acc[g]);
      if (lane == 0) red[g][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < gk) {
      double s = 0.0;
      for (int wv = 0; wv < kThreads / 64; ++wv) s += red[threadIdx.x][wv];
      partial[(long long)(i0 + threadIdx.x) * G + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// out[i] = sum_b partial[i * G + b] (fixed order), one block per i.
__global__ void __launch_bounds__(kThreads) reduce_kernel(const double *__restrict__ partial, int G,
                                                          double *__restrict__ out) {
  __shared__ double red[kThreads / 64];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < G; b += kThreads) s += partial[(long long)i * G + b];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int wv = 0; wv < kThreads / 64; ++wv) t += red[wv];
    out[i] = t;
  }
}

// w[e] -= sum_i h[i] V_i[e]   (h in device memory, i ascending)
__global__ void __launch_bounds__(kThreads) update_kernel(double *__restrict__ w, const double *__restrict__ V,
                                                          long long ldv, int k, const double *__restrict__ h,
                                                          long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += h[i] * V[(long long)i * ldv + e];
    w[e] -= s;
  }
}

// out[e] = sum_i y[i] V_i[e]  (+ out[e] if accumulate)
__global__ void __launch_bounds__(kThreads) combine_kernel(double *__restrict__ out, const double *__restrict__ V,
                                                           long long ldv, int k, const double *__restrict__ y,
                                                           long long n, int accumulate) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += y[i] * V[(long long)i * ldv + e];
    out[e] = accumulate ? out[e] + s : s;
  }
}

// out = a * x + b * y
__global__ void __launch_bounds__(kThreads) axpby_kernel(double *__restrict__ out, double a, const double *__restrict__ x,
                                                         double b, const double *__restrict__ y, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    out[e] = a * x[e] + b * y[e];
}

__global__ void scale_kernel(double *__restrict__ out, const double *__restrict__ x, double a, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    out[e] = a * x[e];
}

// Second CGS pass fused with the first update: with h the first-pass
// coefficients, w <- w - sum_g h[g] V_g and partial[g * G + b] = sum over
// block b's elements of V_g[e] w_new[e], g < k <= 64.  The block's element
// range is walked in tiles of 64 whose k basis entries are staged in LDS, so
// V is read from memory once for both the update and the new dots.
constexpr int kTile = 64;
constexpr int kFuseMax = 64;

__global__ void __launch_bounds__(kThreads) update_dot_kernel(double *__restrict__ w, const double *__restrict__ V,
                                                              long long ldv, int k, const double *__restrict__ h,
                                                              long long n, double *__restrict__ partial) {
  __shared__ double Vs[kFuseMax][kTile + 1];   // padded: the dots read down a column
  __shared__ double Ws[kTile];
  __shared__ double part[kThreads / 64][kTile];
  __shared__ double red[kThreads / 64][kFuseMax];
  const int G = gridDim.x;
  const long long per = (n + G - 1) / G;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = lo + per < n ? lo + per : n;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double acc = 0.0;   // dot of basis vector g = lane over this wave's quarter of every tile
  // the next tile's basis entries are loaded into registers while the current
  // tile is processed (entry q = t + 256 r of the k x 64 tile)
  constexpr int kPre = kFuseMax * kTile / kThreads;
  double pre[kPre];
  auto fetch = [&](long long e0) {
    const int m = (int)(hi - e0 < kTile ? hi - e0 : kTile);
#pragma unroll
    for (int r = 0; r < kPre; ++r) {
      const int q = t + kThreads * r, g = q / kTile, e = q % kTile;
      pre[r] = (g < k && e < m) ? V[(long long)g * ldv + e0 + e] : 0.0;
    }
  };
  if (lo < hi) fetch(lo);
  for (long long e0 = lo; e0 < hi; e0 += kTile) {
    const int m = (int)(hi - e0 < kTile ? hi - e0 : kTile);
#pragma unroll
    for (int r = 0; r < kPre; ++r) {
      const int q = t + kThreads * r, g = q / kTile, e = q % kTile;
      if (g < k) Vs[g][e] = pre[r];
    }
    if (e0 + kTile < hi) fetch(e0 + kTile);
    __syncthreads();
    // update: each wave sums a quarter of the basis vectors for every element of the tile
    {
      double s = 0.0;
      for (int g = wave; g < k; g += kThreads / 64) s += h[g] * Vs[g][lane];
      part[wave][lane] = s;
    }
    __syncthreads();
    if (t < kTile) {
      double s = 0.0;
#pragma unroll
      for (int wv = 0; wv < kThreads / 64; ++wv) s += part[wv][t];
      const double wn = t < m ? w[e0 + t] - s : 0.0;
      if (t < m) w[e0 + t] = wn;
      Ws[t] = wn;
    }
    __syncthreads();
    // dots: lane g, this wave's 16 elements of the tile
    if (lane < k) {
#pragma unroll 4
      for (int e = wave * (kTile / 4); e < (wave + 1) * (kTile / 4); ++e) acc += Vs[lane][e] * Ws[e];
    }
    __syncthreads();
  }
  red[wave][lane] = acc;
  __syncthreads();
  if (t < k) {
    double s = 0.0;
#pragma unroll
    for (int wv = 0; wv < kThreads / 64; ++wv) s += red[wv][t];
    partial[(long long)t * G + blockIdx.x] = s;
  }
}

// Last CGS update fused with the norm: w <- w - sum_g h[g] V_g and
// partial[b] = sum over block b's elements of w_new[e]^2.
__global__ void __launch_bounds__(kThreads) update_norm_kernel(double *__restrict__ w, const double *__restrict__ V,
                                                               long long ldv, int k, const double *__restrict__ h,
                                                               long long n, double *__restrict__ partial) {
  __shared__ double red[kThreads / 64];
  const int G = gridDim.x;
  const long long per = (n + G - 1) / G;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = lo + per < n ? lo + per : n;
  double acc = 0.0;
  for (long long e = lo + threadIdx.x; e < hi; e += kThreads) {
    double s = 0.0;
    for (int g = 0; g < k; ++g) s += h[g] * V[(long long)g * ldv + e];
    const double wn = w[e] - s;
    w[e] = wn;
    acc += wn * wn;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int wv = 0; wv < kThreads / 64; ++wv) s += red[wv];
    partial[blockIdx.x] = s;
  }
}

}  // namespace

bool cgs2_fused_ok(int k) { return k <= kFuseMax; }

void update_dot(double *w, const double *V, long long ldv, int k, const double *h, long long n, double *partial,
                double *out, hipStream_t s) {
  const int G = reduction_blocks(n);
  hipLaunchKernelGGL(update_dot_kernel, dim3(G), dim3(kThreads), 0, s, w, V, ldv, k, h, n, partial);
  STKKT_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_kernel, dim3(k), dim3(kThreads), 0, s, partial, G, out);
  STKKT_HIP(hipGetLastError());
}

void update_norm(double *w, const double *V, long long ldv, int k, const double *h, long long n, double *partial,
                 double *out, hipStream_t s) {
  const int G = reduction_blocks(n);
  hipLaunchKernelGGL(update_norm_kernel, dim3(G), dim3(kThreads), 0, s, w, V, ldv, k, h, n, partial);
  STKKT_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, s, partial, G, out);
  STKKT_HIP(hipGetLastError());
}

int reduction_blocks(long long n) {
  long long g = (n + 4095) / 4096;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (int)g;
}

void multidot(const double *V, long long ldv, int k, const double *w, long long n, double *partial, double *out,
              hipStream_t s) {
  const int G = reduction_blocks(n);
  hipLaunchKernelGGL(multidot_kernel, dim3(G), dim3(kThreads), 0, s, V, ldv, k, w, n, partial);
  STKKT_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_kernel, dim3(k), dim3(kThreads), 0, s, partial, G, out);
  STKKT_HIP(hipGetLastError());
}

void gs_update(double *w, const double *V, long long ldv, int k, const double *h, long long n, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel, dim3(blocks_for(n, kThreads, 16384)), dim3(kThreads), 0, s, w, V, ldv, k, h, n);
  STKKT_HIP(hipGetLastError());
}

void combine(double *out, const double *V, long long ldv, int k, const double *y, long long n, bool accumulate,
             hipStream_t s) {
  hipLaunchKernelGGL(combine_kernel, dim3(blocks_for(n, kThreads, 16384)), dim3(kThreads), 0, s, out, V, ldv, k, y,
                     n, accumulate ? 1 : 0);
  STKKT_HIP(hipGetLastError());
}

void axpby(double *out, double a, const double *x, double b, const double *y, long long n, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(blocks_for(n, kThreads, 16384)), dim3(kThreads), 0, s, out, a, x, b, y, n);
  STKKT_HIP(hipGetLastError());
}

void scale(double *out, const double *x, double a, long long n, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(n, kThreads, 16384)), dim3(kThreads), 0, s, out, x, a, n);
  STKKT_HIP(hipGetLastError());
}

}  // namespace stkkt
