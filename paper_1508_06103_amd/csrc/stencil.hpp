// Coefficients of the space-time KKT operator, evaluated on the fly.
//
// Space: Q1 hexahedra on a uniform mesh, exact integration; 1-D assembled
// entries on an axis with nn nodes and spacing h (row i, column i+d):
//   mass  M[i,i+d]  = h/6 (d = +-1), 2h/3 inside / h/3 at an end (d = 0)
//   stiff K[i,i+d]  = -1/h (d = +-1), 2/h inside / 1/h at an end (d = 0)
//   conv  D[i,i+d]  = int phi_i phi_{i+d}' = +-1/2 (d = +-1), 0 inside,
//                     -1/2 at the first node, +1/2 at the last (d = 0)
// 3-D: B = Mz Mx My products, K = sum of one stiffness and two masses,
// N[j,i] = (v.grad phi_i, phi_j) = vx Dx My Mz + vy Mx Dy Mz + vz Mx My Dz,
// A[j,i] = sum over the elements shared by j and i of a_e times the element
// stiffness entry.  Time: hat functions on t^n = n tau, mass Tt and
// stiffness St with the same 1-D rules, trapezoid weights w_n.
//
// The block formula kkt_block() is the (n, j) x (n+dt, j+d) 3x3 block of F_h
// in the (C, G, f) slot order (Section 3.2 point-block ordering; Appendix A
// block structure; variant conventions in stkkt.h).
#pragma once

#include "common.hpp"

namespace stkkt {

__host__ __device__ inline double mass1(double h, int i, int d, int nn) {
  if (d != 0) return h / 6.0;
  return (i == 0 || i == nn - 1) ? h / 3.0 : 2.0 * h / 3.0;
}
__host__ __device__ inline double stiff1(double h, int i, int d, int nn) {
  if (d != 0) return -1.0 / h;
  return (i == 0 || i == nn - 1) ? 1.0 / h : 2.0 / h;
}
__host__ __device__ inline double conv1(int i, int d, int nn) {
  if (d == -1) return -0.5;
  if (d == 1) return 0.5;
  if (i == 0) return -0.5;
  if (i == nn - 1) return 0.5;
  return 0.0;
}
__host__ __device__ inline double tmass(double tau, int n, int dt, int M) {
  if (dt != 0) return tau / 6.0;
  return (n == 0 || n == M) ? tau / 3.0 : 2.0 * tau / 3.0;
}
__host__ __device__ inline double tstiff(double tau, int n, int dt, int M) {
  if (dt != 0) return -1.0 / tau;
  return (n == 0 || n == M) ? 1.0 / tau : 2.0 / tau;
}
__host__ __device__ inline double wtrap(double tau, int n, int M) {
  return (n == 0 || n == M) ? 0.5 * tau : tau;
}

__host__ __device__ inline bool on_dirichlet(const OpDev &op, int x, int y, int z) {
  unsigned f = op.faces;
  return ((f & 1u) && x == 0) || ((f & 2u) && x == op.nn[0] - 1) || ((f & 4u) && y == 0) ||
         ((f & 8u) && y == op.nn[1] - 1) || ((f & 16u) && z == 0) || ((f & 32u) && z == op.nn[2] - 1);
}

// A[j, j+d]: diffusion stiffness with element coefficients.
__host__ __device__ inline double stiff_var(const OpDev &op, int jx, int jy, int jz, int dx, int dy, int dz) {
  int lo[3], hi[3];
  const int j[3] = {jx, jy, jz};
  const int d[3] = {dx, dy, dz};
  for (int a = 0; a < 3; ++a) {
    int l = j[a] - 1, u = j[a];
    if (d[a] == 1) l = j[a];
    if (d[a] == -1) u = j[a] - 1;
    lo[a] = l < 0 ? 0 : l;
    hi[a] = u > op.n[a] - 1 ? op.n[a] - 1 : u;
  }
  double s = 0.0;
  for (int ez = lo[2]; ez <= hi[2]; ++ez)
    for (int ey = lo[1]; ey <= hi[1]; ++ey)
      for (int ex = lo[0]; ex <= hi[0]; ++ex) {
        const int e[3] = {ex, ey, ez};
        double me[3], ke[3];
        for (int a = 0; a < 3; ++a) {
          int lj = j[a] - e[a], li = j[a] + d[a] - e[a];
          me[a] = (lj == li ? 2.0 : 1.0) * op.h[a] / 6.0;
          ke[a] = (lj == li ? 1.0 : -1.0) / op.h[a];
        }
        double ae = op.a_elem[(long long)ex + (long long)op.n[0] * (ey + (long long)op.n[1] * ez)];
        s += ae * (ke[0] * me[1] * me[2] + me[0] * ke[1] * me[2] + me[0] * me[1] * ke[2]);
      }
  return s;
}

// Spatial coefficients between node j and its neighbour j + d.
struct SpatialCoef {
  double B, K, A, N, Nt;  // N = N[j, j+d], Nt = N[j+d, j]
};

__host__ __device__ inline SpatialCoef spatial_coef(const OpDev &op, int jx, int jy, int jz, int dx, int dy,
                                                    int dz) {
  const double mx = mass1(op.h[0], jx, dx, op.nn[0]);
  const double my = mass1(op.h[1], jy, dy, op.nn[1]);
  const double mz = mass1(op.h[2], jz, dz, op.nn[2]);
  const double kx = stiff1(op.h[0], jx, dx, op.nn[0]);
  const double ky = stiff1(op.h[1], jy, dy, op.nn[1]);
  const double kz = stiff1(op.h[2], jz, dz, op.nn[2]);
  SpatialCoef c;
  c.B = mx * my * mz;
  c.K = kx * my * mz + mx * ky * mz + mx * my * kz;
  c.N = op.v[0] * conv1(jx, dx, op.nn[0]) * my * mz + op.v[1] * mx * conv1(jy, dy, op.nn[1]) * mz +
        op.v[2] * mx * my * conv1(jz, dz, op.nn[2]);
  c.Nt = op.v[0] * conv1(jx + dx, -dx, op.nn[0]) * my * mz +
         op.v[1] * mx * conv1(jy + dy, -dy, op.nn[1]) * mz +
         op.v[2] * mx * my * conv1(jz + dz, -dz, op.nn[2]);
  c.A = stiff_var(op, jx, jy, jz, dx, dy, dz);
  return c;
}

// 3x3 block F_h[(n, j), (n+dt, j+d)] in row-major (row slot, column slot),
// given the spatial coefficients c between j and j + d.
// The neighbour must exist (inside the mesh and 0 <= n+dt <= M).
__host__ __device__ inline void kkt_block_c(const OpDev &op, const SpatialCoef &c, int jx, int jy, int jz, int n,
                                            int dx, int dy, int dz, int dt, double *out) {
  for (int e = 0; e < 9; ++e) out[e] = 0.0;
  const bool same = (dx == 0 && dy == 0 && dz == 0);
  const double Pj = on_dirichlet(op, jx, jy, jz) ? 0.0 : 1.0;
  const double Qj = 1.0 - Pj;
  const double Pi = on_dirichlet(op, jx + dx, jy + dy, jz + dz) ? 0.0 : 1.0;
  const double tau = op.tau;
  const int M = op.M;
  const double ht = 0.5 * tau;
  const double sens = same ? op.sensor[(long long)jx + (long long)op.nn[0] * (jy + (long long)op.nn[1] * jz)] : 0.0;
  const double A1 = c.B + ht * (c.A + c.N), A2 = -c.B + ht * (c.A + c.N);
  const double A1t = c.B + ht * (c.A + c.Nt), A2t = -c.B + ht * (c.A + c.Nt);
  const double idn = (same && dt == 0) ? 1.0 : 0.0;
  // C-slot row: state equation
  if (n == 0) {
    out[0] = idn;
  } else {
    out[0] = Qj * idn + Pj * Pi * (dt == 0 ? A1 : (dt == -1 ? A2 : 0.0));
    if (dt == 0 || dt == -1) out[2] = -Pj * ht * c.B;
  }
  // f-slot row: regularisation block W (beta2 with K, or with B for H1-L2)
  out[8] = op.beta1 * tstiff(tau, n, dt, M) * c.B +
           op.beta2 * tmass(tau, n, dt, M) * (op.reg == STKKT_REG_H1L2 ? c.B : c.K);
  if (op.variant == STKKT_DTO) {
    if (dt == 0) out[3] = wtrap(tau, n, M) * sens;
    double g = Qj * idn;
    if (dt == 0) g += (n >= 1) ? Pj * Pi * A1t : Pj * idn;
    if (dt == 1 && n <= M - 1) g += Pj * Pi * A2t;
    out[4] = g;
    if ((dt == 0 && n >= 1) || (dt == 1 && n <= M - 1)) out[7] = -ht * c.B * Pi;
  } else {
    if (n <= M - 1) {
      if (dt == 0 || dt == 1) out[3] = ht * sens;
      double g = 0.0;
      if (dt == 0) g = Pj * Pi * A1t + Qj * idn;
      if (dt == 1) g = Pj * Pi * A2t;
      out[4] = g;
    } else {
      out[4] = idn;
    }
    out[7] = -tmass(tau, n, dt, M) * c.B * Pi;
  }
}

__host__ __device__ inline void kkt_block(const OpDev &op, int jx, int jy, int jz, int n, int dx, int dy, int dz,
                                          int dt, double *out) {
  const SpatialCoef c = spatial_coef(op, jx, jy, jz, dx, dy, dz);
  kkt_block_c(op, c, jx, jy, jz, n, dx, dy, dz, dt, out);
}

}  // namespace stkkt
