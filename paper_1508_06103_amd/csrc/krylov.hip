// FP64 vector kernels for the Krylov solvers: fixed-order two-stage
// reductions (reproducible run to run) built on wavefront shuffles, and the
// streaming updates of classical Gram-Schmidt.
#include "common.hpp"
#include "krylov.hpp"
#include "cgs2_dev.hpp"

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
    if ((int)threadIdx.x < gk) {
      double s = 0.0;
      for (int wv = 0; wv < kThreads / 64; ++wv) s += red[threadIdx.x][wv];
      partial[(long long)(i0 + threadIdx.x) * G + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// The first CGS pass for k <= 64 vectors on the register tiles of the fused
// passes (partial[i * G + b] as above).
template <int KR>
__global__ void __launch_bounds__(kCgsThreads) multidot_tiles_kernel(const double *__restrict__ V, long long ldv,
                                                                     int k, const double *__restrict__ w, long long n,
                                                                     double *__restrict__ partial) {
  const int G = gridDim.x;
  const long long per = (n + G - 1) / G;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = lo + per < n ? lo + per : n;
  dot_range<KR>(w, V, ldv, k, lo, hi > lo ? hi : lo, partial + blockIdx.x, G);
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

// Second CGS pass fused with the first update (w <- w - V h, partial[g * G +
// b] = block b's part of V_g . w_new) and the last update fused with the norm
// (partial[b] = block b's part of |w_new|^2); the bodies are shared with the
// batched solver.
template <int KR>
__global__ void __launch_bounds__(kCgsThreads) update_dot_kernel(double *__restrict__ w, const double *__restrict__ V,
                                                                 long long ldv, int k, const double *__restrict__ h,
                                                                 long long n, double *__restrict__ partial) {
  const int G = gridDim.x;
  const long long per = (n + G - 1) / G;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = lo + per < n ? lo + per : n;
  update_dot_range<KR>(w, V, ldv, k, h, lo, hi > lo ? hi : lo, partial + blockIdx.x, G);
}

template <int KR>
__global__ void __launch_bounds__(kCgsThreads) update_norm_kernel(double *__restrict__ w, const double *__restrict__ V,
                                                                  long long ldv, int k, const double *__restrict__ h,
                                                                  long long n, double *__restrict__ partial) {
  const int G = gridDim.x;
  const long long per = (n + G - 1) / G;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = lo + per < n ? lo + per : n;
  const double s = update_norm_range<KR>(w, V, ldv, k, h, lo, hi > lo ? hi : lo);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

}  // namespace

bool cgs2_fused_ok(int k) { return k <= kCgsMaxK; }

void update_dot(double *w, const double *V, long long ldv, int k, const double *h, long long n, double *partial,
                double *out, hipStream_t s) {
  const int G = reduction_blocks(n);
  if (k <= kCgsHalf)
    hipLaunchKernelGGL(update_dot_kernel<kCgsHalf>, dim3(G), dim3(kThreads), 0, s, w, V, ldv, k, h, n, partial);
  else if (k <= 48)
    hipLaunchKernelGGL(update_dot_kernel<48>, dim3(G), dim3(kThreads), 0, s, w, V, ldv, k, h, n, partial);
  else if (k <= 56)
    hipLaunchKernelGGL(update_dot_kernel<56>, dim3(G), dim3(kThreads), 0, s, w, V, ldv, k, h, n, partial);
  else
    hipLaunchKernelGGL(update_dot_kernel<kCgsMaxK>, dim3(G), dim3(kThreads), 0, s, w, V, ldv, k, h, n, partial);
  STKKT_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_kernel, dim3(k), dim3(kThreads), 0, s, partial, G, out);
  STKKT_HIP(hipGetLastError());
}

void update_norm(double *w, const double *V, long long ldv, int k, const double *h, long long n, double *partial,
                 double *out, hipStream_t s) {
  const int G = reduction_blocks(n);
  if (k <= kCgsHalf)
    hipLaunchKernelGGL(update_norm_kernel<kCgsHalf>, dim3(G), dim3(kThreads), 0, s, w, V, ldv, k, h, n, partial);
  else if (k <= 48)
    hipLaunchKernelGGL(update_norm_kernel<48>, dim3(G), dim3(kThreads), 0, s, w, V, ldv, k, h, n, partial);
  else
    hipLaunchKernelGGL(update_norm_kernel<kCgsMaxK>, dim3(G), dim3(kThreads), 0, s, w, V, ldv, k, h, n, partial);
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
  if (k <= kCgsHalf)
    hipLaunchKernelGGL(multidot_tiles_kernel<kCgsHalf>, dim3(G), dim3(kCgsThreads), 0, s, V, ldv, k, w, n, partial);
  else if (k <= 48)
    hipLaunchKernelGGL(multidot_tiles_kernel<48>, dim3(G), dim3(kCgsThreads), 0, s, V, ldv, k, w, n, partial);
  else if (k <= 56)
    hipLaunchKernelGGL(multidot_tiles_kernel<56>, dim3(G), dim3(kCgsThreads), 0, s, V, ldv, k, w, n, partial);
  else if (k <= kCgsMaxK)
    hipLaunchKernelGGL(multidot_tiles_kernel<kCgsMaxK>, dim3(G), dim3(kCgsThreads), 0, s, V, ldv, k, w, n, partial);
  else
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
