// Exact block-tridiagonal-in-time solve of the coarse KKT system.
#pragma once

#include "common.hpp"

namespace stkkt {

class CoarseLU {
 public:
  // Forms and inverts every Schur complement of the coarse operator `cop`
  // (FP64 setup); the inverses and E_k are kept in `precision`.
  CoarseLU(const Allocator *al, const kkt_op *cop, int precision, hipStream_t s);
  // x = F_c^{-1} r (device vectors of 3 N_c (M_c + 1) doubles, no aliasing)
  void solve(const double *r, double *x, hipStream_t s) const;
  // x_c = F_c^{-1} r_c for c < q right-hand sides at r + c ldr and x + c ldx
  // (no aliasing): every dense block is read once per 16 right-hand sides
  // and multiplied on the FP64 matrix cores.
  void solve_multi(int q, const double *r, long long ldr, double *x, long long ldx, hipStream_t s) const;
  // bytes of dense blocks streamed by one solve
  size_t bytes_per_solve() const;
  // whether one vector is faster through the matrix-core pass than through
  // the GEMV sweeps (FP64 blocks: the 16-byte row loads of the matrix-core
  // pass stream them faster; FP32 blocks: the GEMV is faster)
  bool one_vector_on_mfma() const { return prec_ == STKKT_F64; }

 private:
  template <typename T> void solve_t(const double *r, double *x, hipStream_t s) const;
  template <typename T>
  void solve_multi_t(int q, const double *r, long long ldr, double *x, long long ldx, hipStream_t s) const;
  int prec_;
  int nb_ = 0, nlev_ = 0;
  int ld_ = 0;       // leading dimension of the stored blocks (nb_ rounded up to 64, zero rows below nb_)
  int nsplit_ = 1;   // column chunks of one multi-RHS block product
  DevBuf Sinv_, E_, Lidx_, Lval_, partial_, t_, mpartial_, mt_;
};

}  // namespace stkkt
