// Two-level space-time preconditioner (Section 3.2, two-level paragraph):
// nested coarse space-time mesh, linear interpolation I_c^h and its transpose
// (or injection) as transfers, and the coarse KKT system rediscretised on the
// coarse mesh.  F_c^{-1} is applied either as in the paper's experiments
// (Section 4): a few steps of restarted GMRES from zero, right-preconditioned
// by the one-level space-time RAS of the coarse mesh; or exactly, by block
// elimination in time with explicitly inverted Schur complements (CoarseLU).
#include <cmath>
#include <memory>

#include "coarse.hpp"
#include "coarse_lu.hpp"
#include "ras.hpp"

struct coarse {
  stkkt::Allocator al;
  const kkt_op *fine_op = nullptr;   // identity only
  stkkt::OpDev fine{};
  int fac[4] = {1, 1, 1, 1};
  coarse_params_t params{};
  kkt_op *cop = nullptr;    // owned coarse operator
  ras *cras = nullptr;      // owned coarse preconditioner
  stkkt::DevBuf xc, yc;     // coarse vectors
  std::unique_ptr<stkkt::GmresWork> work;   // inner GMRES workspace
  std::unique_ptr<stkkt::CoarseLU> lu;       // exact coarse solve (method LU)
  ~coarse() {
    lu.reset();
    work.reset();
    delete cras;
    delete cop;
  }
};

namespace stkkt {

namespace {

// 1-D linear interpolation weight of coarse node I at fine node i (factor f).
__device__ inline double hat(int i, int I, int f) {
  const int d = i - I * f;
  const int ad = d < 0 ? -d : d;
  return ad >= f ? 0.0 : 1.0 - (double)ad / f;
}

// y_fine = I_c^h x_coarse: every fine node interpolates the (up to 16) coarse
// nodes of the coarse space-time cell that contains it.
__global__ void prolong_kernel(OpDev fo, OpDev co, int fx, int fy, int fz, int ft, const double *__restrict__ xc,
                               double *__restrict__ y) {
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < fo.V;
       g += (long long)gridDim.x * blockDim.x) {
    const int n = (int)(g / fo.N);
    const long long j = g - (long long)n * fo.N;
    const int i0 = (int)(j % fo.nn[0]), i1 = (int)((j / fo.nn[0]) % fo.nn[1]), i2 = (int)(j / ((long long)fo.nn[0] * fo.nn[1]));
    const int f[4] = {fx, fy, fz, ft};
    const int p[4] = {i0, i1, i2, n};
    int lo[4], cnt[4];
    for (int d = 0; d < 4; ++d) {
      lo[d] = p[d] / f[d];
      cnt[d] = (p[d] % f[d] == 0) ? 1 : 2;
    }
    double a0 = 0, a1 = 0, a2 = 0;
    for (int b3 = 0; b3 < cnt[3]; ++b3)
      for (int b2 = 0; b2 < cnt[2]; ++b2)
        for (int b1 = 0; b1 < cnt[1]; ++b1)
          for (int b0 = 0; b0 < cnt[0]; ++b0) {
            const int I0 = lo[0] + b0, I1 = lo[1] + b1, I2 = lo[2] + b2, I3 = lo[3] + b3;
            const double w = hat(p[0], I0, f[0]) * hat(p[1], I1, f[1]) * hat(p[2], I2, f[2]) * hat(p[3], I3, f[3]);
            const long long cg = 3 * ((long long)I3 * co.N + I0 + (long long)co.nn[0] * (I1 + (long long)co.nn[1] * I2));
            a0 += w * xc[cg];
            a1 += w * xc[cg + 1];
            a2 += w * xc[cg + 2];
          }
    y[3 * g] = a0;
    y[3 * g + 1] = a1;
    y[3 * g + 2] = a2;
  }
}

// x_coarse = (I_c^h)^T x_fine (transpose: every coarse node gathers the fine
// nodes of its support) or injection (the fine value at the coarse node).
__global__ void restrict_kernel(OpDev fo, OpDev co, int fx, int fy, int fz, int ft, int injection,
                                const double *__restrict__ x, double *__restrict__ xc) {
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < co.V;
       g += (long long)gridDim.x * blockDim.x) {
    const int n = (int)(g / co.N);
    const long long j = g - (long long)n * co.N;
    const int I[4] = {(int)(j % co.nn[0]), (int)((j / co.nn[0]) % co.nn[1]), (int)(j / ((long long)co.nn[0] * co.nn[1])), n};
    const int f[4] = {fx, fy, fz, ft};
    const int L[4] = {fo.nn[0], fo.nn[1], fo.nn[2], fo.M + 1};
    if (injection) {
      const long long fg = 3 * ((long long)(I[3] * f[3]) * fo.N + I[0] * f[0] +
                                (long long)fo.nn[0] * (I[1] * f[1] + (long long)fo.nn[1] * (I[2] * f[2])));
      xc[3 * g] = x[fg];
      xc[3 * g + 1] = x[fg + 1];
      xc[3 * g + 2] = x[fg + 2];
      continue;
    }
    int lo[4], hi[4];
    for (int d = 0; d < 4; ++d) {
      lo[d] = max(0, I[d] * f[d] - f[d] + 1);
      hi[d] = min(L[d] - 1, I[d] * f[d] + f[d] - 1);
    }
    double a0 = 0, a1 = 0, a2 = 0;
    for (int p3 = lo[3]; p3 <= hi[3]; ++p3) {
      const double w3 = hat(p3, I[3], f[3]);
      for (int p2 = lo[2]; p2 <= hi[2]; ++p2) {
        const double w2 = w3 * hat(p2, I[2], f[2]);
        for (int p1 = lo[1]; p1 <= hi[1]; ++p1) {
          const double w1 = w2 * hat(p1, I[1], f[1]);
          const long long base = 3 * ((long long)p3 * fo.N + (long long)fo.nn[0] * (p1 + (long long)fo.nn[1] * p2));
          for (int p0 = lo[0]; p0 <= hi[0]; ++p0) {
            const double w = w1 * hat(p0, I[0], f[0]);
            const long long fg = base + 3LL * p0;
            a0 += w * x[fg];
            a1 += w * x[fg + 1];
            a2 += w * x[fg + 2];
          }
        }
      }
    }
    xc[3 * g] = a0;
    xc[3 * g + 1] = a1;
    xc[3 * g + 2] = a2;
  }
}

}  // namespace

coarse *coarse_create(const kkt_op *fine, const coarse_params_t *cp, hipStream_t s) {
  STKKT_REQUIRE(cp->method == STKKT_COARSE_GMRES_RAS || cp->method == STKKT_COARSE_LU,
                "coarse_setup: unknown coarse solver");
  STKKT_REQUIRE(cp->precision == STKKT_F64 || cp->precision == STKKT_F32, "coarse_setup: bad precision");
  STKKT_REQUIRE(cp->restrict_kind == STKKT_RESTRICT_TRANSPOSE || cp->restrict_kind == STKKT_RESTRICT_INJECTION,
                "coarse_setup: bad restriction");
  if (cp->method == STKKT_COARSE_GMRES_RAS)
    STKKT_REQUIRE(cp->maxit >= 1 && cp->rtol > 0 && cp->rtol < 1, "coarse_setup: bad coarse solver settings");
  const OpDev &fd = fine->d;
  const int nf[4] = {fd.n[0], fd.n[1], fd.n[2], fd.M};
  for (int d = 0; d < 4; ++d)
    STKKT_REQUIRE(cp->factor[d] >= 1 && nf[d] % cp->factor[d] == 0,
                  "coarse_setup: coarsening factors must divide the element counts and nt");
  auto C = std::make_unique<coarse>();
  C->al = fine->al;
  C->fine = fd;
  C->fine_op = fine;
  C->params = *cp;
  for (int d = 0; d < 4; ++d) C->fac[d] = cp->factor[d];
  // coarse problem: same model, coarse mesh, averaged element coefficients
  kkt_problem_t p{};
  const int nc[3] = {fd.n[0] / cp->factor[0], fd.n[1] / cp->factor[1], fd.n[2] / cp->factor[2]};
  for (int d = 0; d < 3; ++d) {
    p.n[d] = nc[d];
    p.len[d] = fine->len[d];
    p.v[d] = fd.v[d];
  }
  p.nt = fd.M / cp->factor[3];
  p.T = fine->T;
  std::vector<double> ac((size_t)nc[0] * nc[1] * nc[2], 0.0);
  const int f0 = cp->factor[0], f1 = cp->factor[1], f2 = cp->factor[2];
  for (int ez = 0; ez < fd.n[2]; ++ez)
    for (int ey = 0; ey < fd.n[1]; ++ey)
      for (int ex = 0; ex < fd.n[0]; ++ex)
        ac[(ex / f0) + (size_t)nc[0] * ((ey / f1) + (size_t)nc[1] * (ez / f2))] +=
            fine->a_host[ex + (size_t)fd.n[0] * (ey + (size_t)fd.n[1] * ez)];
  for (double &v : ac) v /= (double)(f0 * f1 * f2);
  p.a_elem = ac.data();
  p.beta1 = fd.beta1;
  p.beta2 = fd.beta2;
  std::vector<int32_t> cs;
  for (int32_t j : fine->sensor_node) {
    const int i0 = j % fd.nn[0], i1 = (j / fd.nn[0]) % fd.nn[1], i2 = j / (fd.nn[0] * fd.nn[1]);
    STKKT_REQUIRE(i0 % f0 == 0 && i1 % f1 == 0 && i2 % f2 == 0,
                  "coarse_setup: every sensor must sit on a coarse node");
    cs.push_back((i0 / f0) + (nc[0] + 1) * ((i1 / f1) + (nc[1] + 1) * (i2 / f2)));
  }
  std::vector<double> zeros((size_t)(p.nt + 1) * cs.size(), 0.0);
  p.n_sensors = (int32_t)cs.size();
  p.sensor_node = cs.data();
  p.data = zeros.data();
  p.dirichlet_faces = fd.faces;
  p.variant = fd.variant;
  kkt_alloc_t al = fine->al.cb;
  C->cop = op_create(&p, al.alloc ? &al : nullptr, s);
  const size_t nvc = 3 * (size_t)C->cop->d.V;
  C->xc = DevBuf(&C->al, sizeof(double) * nvc);
  C->yc = DevBuf(&C->al, sizeof(double) * nvc);
  if (cp->method == STKKT_COARSE_LU) {
    C->lu = std::make_unique<CoarseLU>(&C->al, C->cop, cp->precision, s);
  } else {
    ras_params_t rp{};
    for (int d = 0; d < 4; ++d) rp.p[d] = cp->p[d];
    rp.overlap = cp->overlap;
    rp.precision = cp->precision;
    rp.ilu_level = 0;
    C->cras = ras_create(C->cop, &rp, s);
    C->work = std::make_unique<GmresWork>(&C->cop->al, (long long)nvc, cp->maxit, false, false);
  }
  return C.release();
}

void coarse_apply_device(const coarse *C, const double *x, double *y, hipStream_t s) {
  const OpDev &fo = C->fine, &co = C->cop->d;
  hipLaunchKernelGGL(restrict_kernel, dim3(blocks_for(co.V, 256, 8192)), dim3(256), 0, s, fo, co, C->fac[0],
                     C->fac[1], C->fac[2], C->fac[3], C->params.restrict_kind == STKKT_RESTRICT_INJECTION ? 1 : 0, x,
                     C->xc.as<double>());
  STKKT_HIP(hipGetLastError());
  if (C->lu) {
    C->lu->solve(C->xc.as<double>(), C->yc.as<double>(), s);
  } else {
    fill_zero(C->yc.as<double>(), 3 * co.V, s);
    solve_params_t sp{};
    sp.restart = C->params.maxit;
    sp.maxit = C->params.maxit;
    sp.rtol = C->params.rtol;
    sp.flexible = 0;
    sp.fixed_iters = 0;
    const int st = gmres_solve(C->cop, C->cras, nullptr, sp, C->xc.as<double>(), C->yc.as<double>(), s, nullptr,
                               C->work.get());
    if (st != STKKT_OK && st != STKKT_NOT_CONVERGED) throw Error(st, "coarse solve failed");
  }
  hipLaunchKernelGGL(prolong_kernel, dim3(blocks_for(fo.V, 256, 1 << 16)), dim3(256), 0, s, fo, co, C->fac[0],
                     C->fac[1], C->fac[2], C->fac[3], C->yc.as<double>(), y);
  STKKT_HIP(hipGetLastError());
}

void coarse_free(coarse *c) { delete c; }

bool coarse_built_for(const coarse *c, const kkt_op *op) { return c->fine_op == op; }

}  // namespace stkkt
