// Restarted right-preconditioned GMRES / FGMRES driver (Sections 3.2 and 4 of
// the paper: F_h M^{-1} U' = b, U = M^{-1} U', x0 = 0, relative tolerance,
// restarts).  Orthogonalisation is classical Gram-Schmidt applied twice
// (CGS2) on the device; the small Hessenberg least-squares problem is solved
// on the host with Givens rotations, one device-to-host copy per step.
// Stopping rule: the Givens estimate |g_{j+1}| <= rtol ||b|| ends a cycle,
// the true residual ||b - F x|| <= rtol ||b|| decides convergence.
#include <chrono>
#include <cmath>

#include "coarse.hpp"
#include "krylov.hpp"
#include "ras.hpp"

namespace stkkt {

PinnedHost::PinnedHost(size_t n) {
  if (hipHostMalloc((void **)&p, n * sizeof(double), hipHostMallocDefault) != hipSuccess) p = nullptr;
  if (!p) throw Error(STKKT_ENOMEM, "kkt_solve: pinned host allocation failed");
}

PinnedHost::~PinnedHost() {
  if (p) (void)hipHostFree(p);
}

GmresWork::GmresWork(const Allocator *al, long long n_, int m_, bool flex_, bool two_level)
    : n(n_), m(m_), flex(flex_), coarse(two_level), G(reduction_blocks(n_)), hlen(2 * (m_ + 1) + 2),
      V(al, sizeof(double) * (size_t)(m_ + 1) * n_), Z(al, flex_ ? sizeof(double) * (size_t)m_ * n_ : 0),
      rb(al, sizeof(double) * n_), wb(al, sizeof(double) * n_), tb(al, sizeof(double) * n_),
      ub(al, sizeof(double) * n_), yb(al, two_level ? sizeof(double) * n_ : 0),
      t2(al, two_level ? sizeof(double) * n_ : 0), partial(al, sizeof(double) * (size_t)(m_ + 1) * G),
      hdev(al, sizeof(double) * (size_t)(hlen + m_ + 1)), hh((size_t)(hlen + m_ + 1)) {}

bool GmresWork::fits(long long n_, int m_, bool flex_, bool two_level) const {
  return n == n_ && m >= m_ && (flex || !flex_) && (coarse || !two_level);
}

void precond_apply(const kkt_op *op, const ras *R, const coarse *C, const double *v, double *z, double *y,
                   double *t, hipStream_t s) {
  const long long n = 3 * op->d.V;
  if (!C) {
    ras_apply_device(R, v, z, s);
    return;
  }
  // y = I_c^h F_c^{-1} I_h^c v;  z = y + M_one^{-1} (v - F_h y)
  coarse_apply_device(C, v, y, s);
  matvec_device(op, y, t, s);
  axpby(t, 1.0, v, -1.0, t, n, s);
  ras_apply_device(R, t, z, s);
  axpby(z, 1.0, z, 1.0, y, n, s);
}

int gmres_solve(const kkt_op *op, const ras *R, const coarse *C, const solve_params_t &sp, const double *b,
                double *x, hipStream_t s, kkt_stats_t *st, GmresWork *work) {
  const auto t0 = std::chrono::steady_clock::now();
  const long long n = 3 * op->d.V;
  const int m = sp.restart;
  // Both forms keep the preconditioned vectors z_j = M^{-1} v_j (one more
  // n-vector per step in device memory) and update x from them, so a restart
  // needs no further preconditioner application.  With a fixed preconditioner
  // (sp.flexible == 0) this gives the iterates of right-preconditioned GMRES
  // up to rounding (M^{-1} is linear); with a varying one it is FGMRES.
  const bool flex = true;
  std::unique_ptr<GmresWork> own;
  if (!work || !work->fits(n, m, flex, C != nullptr)) {
    own = std::make_unique<GmresWork>(&op->al, n, m, flex, C != nullptr);
    work = own.get();
  }
  GmresWork &W = *work;
  DevBuf &V = W.V, &Z = W.Z, &rb = W.rb, &wb = W.wb, &tb = W.tb, &ub = W.ub, &yb = W.yb, &t2 = W.t2,
         &partial = W.partial, &hdev = W.hdev;
  PinnedHost &hh = W.hh;
  const int hlen = 2 * (m + 1) + 2;
  double *Vd = V.as<double>(), *Zd = Z.as<double>(), *r = rb.as<double>(), *w = wb.as<double>(),
         *t = tb.as<double>(), *u = ub.as<double>(), *hd = hdev.as<double>();
  double *ydev = hd + hlen;

  auto dot = [&](const double *a, const double *c) {
    multidot(a, 0, 1, c, n, partial.as<double>(), hd, s);
    STKKT_HIP(hipMemcpyAsync(hh.p, hd, sizeof(double), hipMemcpyDeviceToHost, s));
    STKKT_HIP(hipStreamSynchronize(s));
    return hh.p[0];
  };
  auto precond = [&](const double *v, double *z) {
    precond_apply(op, R, C, v, z, yb.as<double>(), t2.as<double>(), s);
  };

  kkt_stats_t stats{};
  int status = STKKT_OK;
  const double bnorm = std::sqrt(dot(b, b));
  stats.bnorm = bnorm;
  if (!std::isfinite(bnorm)) throw Error(STKKT_EINVAL, "kkt_solve: non-finite right-hand side");
  if (bnorm == 0.0) {
    fill_zero(x, n, s);
    STKKT_HIP(hipStreamSynchronize(s));
    stats.converged = 1;
    if (st) *st = stats;
    return STKKT_OK;
  }
  const double target = sp.rtol * bnorm;
  const int limit = sp.fixed_iters > 0 ? sp.fixed_iters : sp.maxit;
  matvec_device(op, x, t, s);
  axpby(r, 1.0, b, -1.0, t, n, s);
  double beta = std::sqrt(dot(r, r));
  stats.rel_res_true = beta / bnorm;
  stats.rel_res_est = beta / bnorm;
  if (sp.fixed_iters == 0 && beta <= target) {
    stats.converged = 1;
    if (st) *st = stats;
    return STKKT_OK;
  }
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), col(m + 1), y(m);
  for (;;) {
    if (beta == 0.0) {
      stats.converged = 1;
      break;
    }
    if (!std::isfinite(beta)) {
      status = STKKT_EBREAKDOWN;
      break;
    }
    scale(Vd, r, 1.0 / beta, n, s);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    bool breakdown = false;
    for (int j = 0; j < m; ++j) {
      const double *vj = Vd + (long long)j * n;
      double *zj = flex ? Zd + (long long)j * n : u;
      precond(vj, zj);
      matvec_device(op, zj, w, s);
      // CGS2: h1 = V^T w; w -= V h1; h2 = V^T w; w -= V h2; |w|^2
      multidot(Vd, n, j + 1, w, n, partial.as<double>(), hd, s);
      if (cgs2_fused_ok(j + 1)) {
        update_dot(w, Vd, n, j + 1, hd, n, partial.as<double>(), hd + (m + 1), s);
        update_norm(w, Vd, n, j + 1, hd + (m + 1), n, partial.as<double>(), hd + 2 * (m + 1), s);
      } else {
        gs_update(w, Vd, n, j + 1, hd, n, s);
        multidot(Vd, n, j + 1, w, n, partial.as<double>(), hd + (m + 1), s);
        gs_update(w, Vd, n, j + 1, hd + (m + 1), n, s);
        multidot(w, 0, 1, w, n, partial.as<double>(), hd + 2 * (m + 1), s);
      }
      STKKT_HIP(hipMemcpyAsync(hh.p, hd, sizeof(double) * hlen, hipMemcpyDeviceToHost, s));
      STKKT_HIP(hipStreamSynchronize(s));
      const double hn = std::sqrt(hh.p[2 * (m + 1)]);
      std::fill(col.begin(), col.end(), 0.0);
      for (int i = 0; i <= j; ++i) col[i] = hh.p[i] + hh.p[(m + 1) + i];
      col[j + 1] = hn;
      for (int i = 0; i < j; ++i) {
        const double tmp = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = tmp;
      }
      const double d = std::hypot(col[j], col[j + 1]);
      double c = 1.0, sgn = 0.0;
      if (d != 0.0) {
        c = col[j] / d;
        sgn = col[j + 1] / d;
      }
      cs[j] = c;
      sn[j] = sgn;
      col[j] = d;
      col[j + 1] = 0.0;
      for (int i = 0; i <= m; ++i) H[(size_t)i * m + j] = col[i];
      g[j + 1] = -sgn * g[j];
      g[j] = c * g[j];
      stats.iters += 1;
      k = j + 1;
      const double est = std::fabs(g[j + 1]);
      if (!std::isfinite(est) || !std::isfinite(hn)) {
        breakdown = true;
        break;
      }
      bool done = stats.iters >= limit;
      if (sp.fixed_iters == 0 && (est <= target || hn == 0.0)) done = true;
      if (done || hn == 0.0) break;
      scale(Vd + (long long)(j + 1) * n, w, 1.0 / hn, n, s);
    }
    if (breakdown) {
      status = STKKT_EBREAKDOWN;
      break;
    }
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[i];
      for (int l = i + 1; l < k; ++l) acc -= H[(size_t)i * m + l] * y[l];
      y[i] = acc / H[(size_t)i * m + i];
    }
    for (int i = 0; i < k; ++i) hh.p[hlen + i] = y[i];
    STKKT_HIP(hipMemcpyAsync(ydev, hh.p + hlen, sizeof(double) * k, hipMemcpyHostToDevice, s));
    if (flex) {
      combine(x, Zd, n, k, ydev, n, true, s);
    } else {
      combine(u, Vd, n, k, ydev, n, false, s);
      precond(u, t);
      axpby(x, 1.0, x, 1.0, t, n, s);
    }
    matvec_device(op, x, t, s);
    axpby(r, 1.0, b, -1.0, t, n, s);
    beta = std::sqrt(dot(r, r));
    stats.rel_res_est = std::fabs(g[k]) / bnorm;
    stats.rel_res_true = beta / bnorm;
    if (sp.fixed_iters > 0) {
      stats.converged = beta <= target ? 1 : 0;
      if (stats.iters >= sp.fixed_iters) break;
    } else if (beta <= target) {
      stats.converged = 1;
      break;
    }
    if (stats.iters >= limit) break;
    stats.restarts += 1;
  }
  STKKT_HIP(hipStreamSynchronize(s));
  if (status == STKKT_OK && !stats.converged && sp.fixed_iters == 0) status = STKKT_NOT_CONVERGED;
  stats.status = status;
  stats.t_ms[0] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = stats;
  return status;
}

}  // namespace stkkt
