// FP64 Krylov vector operations (device).
#pragma once

#include "common.hpp"

namespace stkkt {

// Number of first-stage blocks used by multidot for vectors of length n
// (partial buffers need k * reduction_blocks(n) doubles).
int reduction_blocks(long long n);

// out[i] = V_i . w for i < k (out: device), V_i = V + i * ldv.
void multidot(const double *V, long long ldv, int k, const double *w, long long n, double *partial, double *out,
              hipStream_t s);
// w -= sum_i h[i] V_i  (h: device)
void gs_update(double *w, const double *V, long long ldv, int k, const double *h, long long n, hipStream_t s);
// out = sum_i y[i] V_i (+ out if accumulate)  (y: device)
void combine(double *out, const double *V, long long ldv, int k, const double *y, long long n, bool accumulate,
             hipStream_t s);
// Fused CGS2 passes (k <= 64 basis vectors, cgs2_fused_ok):
//   update_dot:  w -= sum_i h[i] V_i, then out[i] = V_i . w   (V read once)
//   update_norm: w -= sum_i h[i] V_i, then out[0] = w . w
bool cgs2_fused_ok(int k);
void update_dot(double *w, const double *V, long long ldv, int k, const double *h, long long n, double *partial,
                double *out, hipStream_t s);
void update_norm(double *w, const double *V, long long ldv, int k, const double *h, long long n, double *partial,
                 double *out, hipStream_t s);
void axpby(double *out, double a, const double *x, double b, const double *y, long long n, hipStream_t s);
void scale(double *out, const double *x, double a, long long n, hipStream_t s);

}  // namespace stkkt
