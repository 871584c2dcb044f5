// 3x3 block helpers shared by the ILU factorisations.
#pragma once

#include <hip/hip_runtime.h>

namespace stkkt {

// Inverse of a row-major 3x3 block by Gauss-Jordan elimination with partial
// pivoting on [a | I]; ok = false for a singular block.
__device__ inline void inv33_pivot(const double *a, double *out, bool &ok) {
  double m[3][6];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      m[r][c] = a[3 * r + c];
      m[r][3 + c] = (r == c) ? 1.0 : 0.0;
    }
  ok = true;
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (fabs(m[r][col]) > fabs(m[piv][col])) piv = r;
    if (!(fabs(m[piv][col]) > 0.0)) {
      ok = false;
      return;
    }
    if (piv != col)
      for (int c = 0; c < 6; ++c) {
        double t = m[col][c];
        m[col][c] = m[piv][c];
        m[piv][c] = t;
      }
    const double dinv = 1.0 / m[col][col];
    for (int c = 0; c < 6; ++c) m[col][c] *= dinv;
    for (int r = 0; r < 3; ++r) {
      if (r == col) continue;
      const double f = m[r][col];
      for (int c = 0; c < 6; ++c) m[r][c] -= f * m[col][c];
    }
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) out[3 * r + c] = m[r][3 + c];
}

}  // namespace stkkt
