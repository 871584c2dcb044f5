// Batched solves: many independent KKT systems advanced together by one
// restarted FGMRES (Sections 3.2 and 4 of the paper: right-preconditioned
// FGMRES, x0 given, relative tolerance per instance), with every device step
// issued once for the whole batch.
//
// The instances' vectors are concatenated (instance i at element voff_i,
// 256-aligned).  Each Arnoldi step is one batched preconditioner launch over
// the (instance, subdomain) work list, one batched matvec over the (instance,
// tile) work list, and CGS2 passes whose reductions are per instance: every
// instance's elements are cut into fixed chunks, each chunk reduced by one
// block and the chunk sums of an instance added in a fixed order, so an
// instance's arithmetic does not depend on which other instances share the
// batch.  The host reads back all instances' Hessenberg columns with one copy
// per step and runs the Givens updates.
//
// Instances run in lockstep inside a cycle.  An instance whose residual
// estimate meets its tolerance (or that reaches maxit) leaves the cycle; at
// the end of the cycle every instance that took part updates its iterate and
// computes its true residual; those that have not converged start the next
// cycle together.  Finished instances are masked out of every launch.
#include <chrono>
#include <cmath>
#include <memory>

#include "coarse.hpp"
#include "ras.hpp"

namespace stkkt {

namespace {

constexpr int kBT = 256;          // threads per block
constexpr long long kChunk = 4096;   // elements per reduction chunk
constexpr int kGroup = 8;         // basis vectors per pass of the multi-dot

struct Chunk {
  int32_t inst, pad;
  int64_t lo, hi;   // element range in the concatenated vectors
};

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// partial[g * nch + c] = sum over chunk c of V_g[e] w[e], g < k.
__global__ void __launch_bounds__(kBT) bmultidot_kernel(const double *__restrict__ V, long long ldv, int k,
                                                        const double *__restrict__ w, const Chunk *__restrict__ ch,
                                                        int nch, const int *__restrict__ act,
                                                        double *__restrict__ partial) {
  __shared__ double red[kGroup][kBT / 64];
  const Chunk c = load_uniform(ch + blockIdx.x);
  if (!as_const(act)[c.inst]) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i0 = 0; i0 < k; i0 += kGroup) {
    const int gk = k - i0 < kGroup ? k - i0 : kGroup;
    double acc[kGroup];
#pragma unroll
    for (int g = 0; g < kGroup; ++g) acc[g] = 0.0;
    for (long long e = c.lo + threadIdx.x; e < c.hi; e += kBT) {
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
      for (int wv = 0; wv < kBT / 64; ++wv) s += red[threadIdx.x][wv];
      partial[(long long)(i0 + threadIdx.x) * nch + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// out[inst * ostride + g] = sum of the instance's chunk partials (fixed order);
// grid (count, k).
__global__ void __launch_bounds__(kBT) breduce_kernel(const double *__restrict__ partial, int nch,
                                                      const int *__restrict__ cfirst, const int *__restrict__ act,
                                                      int ostride, double *__restrict__ out) {
  __shared__ double red[kBT / 64];
  const int inst = blockIdx.x, g = blockIdx.y;
  if (!as_const(act)[inst]) return;
  const int c0 = as_const(cfirst)[inst], c1 = as_const(cfirst)[inst + 1];
  double s = 0.0;
  for (int c = c0 + threadIdx.x; c < c1; c += kBT) s += partial[(long long)g * nch + c];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int wv = 0; wv < kBT / 64; ++wv) t += red[wv];
    out[(long long)inst * ostride + g] = t;
  }
}

// w[e] -= sum_g h[inst][g] V_g[e]
__global__ void __launch_bounds__(kBT) bupdate_kernel(double *__restrict__ w, const double *__restrict__ V,
                                                      long long ldv, int k, const double *__restrict__ h,
                                                      int hstride, const Chunk *__restrict__ ch,
                                                      const int *__restrict__ act) {
  const Chunk c = load_uniform(ch + blockIdx.x);
  if (!as_const(act)[c.inst]) return;
  const double *hi = h + (long long)c.inst * hstride;
  for (long long e = c.lo + threadIdx.x; e < c.hi; e += kBT) {
    double s = 0.0;
    for (int g = 0; g < k; ++g) s += hi[g] * V[(long long)g * ldv + e];
    w[e] -= s;
  }
}

// out[e] = x[e] / sqrt(nrm2[inst])  (0 when the norm is 0)
__global__ void __launch_bounds__(kBT) bnormalize_kernel(double *__restrict__ out, const double *__restrict__ x,
                                                         const double *__restrict__ nrm2, int nstride,
                                                         const Chunk *__restrict__ ch, const int *__restrict__ act) {
  const Chunk c = load_uniform(ch + blockIdx.x);
  if (!as_const(act)[c.inst]) return;
  const double q = nrm2[(long long)c.inst * nstride];
  const double inv = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  for (long long e = c.lo + threadIdx.x; e < c.hi; e += kBT) out[e] = x[e] * inv;
}

// out = x - y
__global__ void __launch_bounds__(kBT) bsub_kernel(double *__restrict__ out, const double *__restrict__ x,
                                                   const double *__restrict__ y, const Chunk *__restrict__ ch,
                                                   const int *__restrict__ act) {
  const Chunk c = load_uniform(ch + blockIdx.x);
  if (!as_const(act)[c.inst]) return;
  for (long long e = c.lo + threadIdx.x; e < c.hi; e += kBT) out[e] = x[e] - y[e];
}

// x[e] += sum_{g < kcnt[inst]} y[inst][g] Z_g[e]
__global__ void __launch_bounds__(kBT) bcombine_kernel(double *__restrict__ x, const double *__restrict__ Z,
                                                       long long ldz, const double *__restrict__ y, int ystride,
                                                       const int *__restrict__ kcnt, const Chunk *__restrict__ ch,
                                                       const int *__restrict__ act) {
  const Chunk c = load_uniform(ch + blockIdx.x);
  if (!as_const(act)[c.inst]) return;
  const int k = as_const(kcnt)[c.inst];
  const double *yi = y + (long long)c.inst * ystride;
  for (long long e = c.lo + threadIdx.x; e < c.hi; e += kBT) {
    double s = 0.0;
    for (int g = 0; g < k; ++g) s += yi[g] * Z[(long long)g * ldz + e];
    x[e] += s;
  }
}

struct PinnedBuf {
  void *p = nullptr;
  explicit PinnedBuf(size_t bytes) {
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) p = nullptr;
    if (!p) throw Error(STKKT_ENOMEM, "kkt_solve_batch: pinned host allocation failed");
  }
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  template <class T> T *as() const { return static_cast<T *>(p); }
};

}  // namespace

int gmres_solve_batch(int count, const kkt_op *const *ops, const ras *const *R, const solve_params_t &sp,
                      const double *const *b, double *const *x, hipStream_t s, kkt_stats_t *stats) {
  const auto t0 = std::chrono::steady_clock::now();
  const int m = sp.restart;
  const Allocator *al = &ops[0]->al;
  // layout of the concatenated vectors and the reduction chunks
  std::vector<long long> voff(count), nloc(count);
  std::vector<Chunk> chunks;
  std::vector<int> cfirst(count + 1);
  long long Ntot = 0;
  for (int i = 0; i < count; ++i) {
    nloc[i] = 3 * ops[i]->d.V;
    voff[i] = Ntot;
    cfirst[i] = (int)chunks.size();
    for (long long lo = 0; lo < nloc[i]; lo += kChunk)
      chunks.push_back(Chunk{i, 0, Ntot + lo, Ntot + std::min(nloc[i], lo + kChunk)});
    Ntot += (nloc[i] + 255) / 256 * 256;
  }
  cfirst[count] = (int)chunks.size();
  const int nch = (int)chunks.size();
  const int hs = 2 * (m + 1) + 2;   // per instance: h1[m+1], h2[m+1], |w|^2, spare
  DevBuf V(al, sizeof(double) * (size_t)(m + 1) * Ntot), Z(al, sizeof(double) * (size_t)m * Ntot);
  DevBuf Bv(al, sizeof(double) * Ntot), X(al, sizeof(double) * Ntot), Rv(al, sizeof(double) * Ntot),
      Wv(al, sizeof(double) * Ntot), Tv(al, sizeof(double) * Ntot);
  DevBuf partial(al, sizeof(double) * (size_t)(m + 1) * nch);
  DevBuf hdev(al, sizeof(double) * (size_t)count * hs), ydev(al, sizeof(double) * (size_t)count * m);
  DevBuf d_chunks(al, sizeof(Chunk) * (size_t)nch), d_cfirst(al, sizeof(int) * (count + 1));
  DevBuf act_step(al, sizeof(int) * count), act_cyc(al, sizeof(int) * count), d_kcnt(al, sizeof(int) * count);
  PinnedBuf hh(sizeof(double) * (size_t)count * hs), hy(sizeof(double) * (size_t)count * m),
      hflags(sizeof(int) * 3 * (size_t)count);
  STKKT_HIP(hipMemcpyAsync(d_chunks.ptr, chunks.data(), sizeof(Chunk) * nch, hipMemcpyHostToDevice, s));
  STKKT_HIP(hipMemcpyAsync(d_cfirst.ptr, cfirst.data(), sizeof(int) * (count + 1), hipMemcpyHostToDevice, s));
  fill_zero(V.as<double>(), (long long)(m + 1) * Ntot, s);
  fill_zero(Z.as<double>(), (long long)m * Ntot, s);
  fill_zero(Bv.as<double>(), Ntot, s);
  fill_zero(X.as<double>(), Ntot, s);
  fill_zero(Rv.as<double>(), Ntot, s);
  fill_zero(Wv.as<double>(), Ntot, s);
  fill_zero(Tv.as<double>(), Ntot, s);
  for (int i = 0; i < count; ++i) {
    STKKT_HIP(hipMemcpyAsync(Bv.as<double>() + voff[i], b[i], sizeof(double) * nloc[i], hipMemcpyDeviceToDevice, s));
    STKKT_HIP(hipMemcpyAsync(X.as<double>() + voff[i], x[i], sizeof(double) * nloc[i], hipMemcpyDeviceToDevice, s));
  }
  MvBatch mv;
  matvec_batch_prepare(ops, voff.data(), count, al, mv, s);
  RasBatch rb;
  ras_batch_prepare(R, voff.data(), count, al, rb, s);

  double *Vd = V.as<double>(), *Zd = Z.as<double>(), *Bd = Bv.as<double>(), *Xd = X.as<double>(),
         *Rd = Rv.as<double>(), *Wd = Wv.as<double>(), *Td = Tv.as<double>(), *hd = hdev.as<double>();
  const Chunk *chd = d_chunks.as<Chunk>();
  const int *cfd = d_cfirst.as<int>();
  int *hf = hflags.as<int>();
  int *h_step = hf, *h_cyc = hf + count, *h_k = hf + 2 * count;
  auto upload_flags = [&](int *host, DevBuf &dev) {
    STKKT_HIP(hipMemcpyAsync(dev.ptr, host, sizeof(int) * count, hipMemcpyHostToDevice, s));
  };
  // per-instance reductions: out[i * ostride + g] = V_g . w over instance i, g < k
  auto bdot = [&](const double *Vb, long long ldv, int k, const double *w, const int *act, int ostride, double *out) {
    hipLaunchKernelGGL(bmultidot_kernel, dim3(nch), dim3(kBT), 0, s, Vb, ldv, k, w, chd, nch, act,
                       partial.as<double>());
    hipLaunchKernelGGL(breduce_kernel, dim3(count, k), dim3(kBT), 0, s, partial.as<double>(), nch, cfd, act, ostride,
                       out);
    STKKT_HIP(hipGetLastError());
  };
  auto fetch = [&](int n_doubles) {
    STKKT_HIP(hipMemcpyAsync(hh.p, hd, sizeof(double) * (size_t)n_doubles, hipMemcpyDeviceToHost, s));
    STKKT_HIP(hipStreamSynchronize(s));
  };
  const double *H = hh.as<double>();

  std::vector<kkt_stats_t> st(count);
  std::vector<double> bnorm(count), target(count), beta(count);
  std::vector<int> state(count, 0);   // 0 running, 1 converged, 2 stopped (maxit), 3 breakdown
  const int limit = sp.fixed_iters > 0 ? sp.fixed_iters : sp.maxit;
  for (int i = 0; i < count; ++i) h_cyc[i] = 1;
  upload_flags(h_cyc, act_cyc);
  // ||b|| and the initial residual
  bdot(Bd, 0, 1, Bd, act_cyc.as<int>(), hs, hd);
  fetch(count * hs);
  for (int i = 0; i < count; ++i) {
    bnorm[i] = std::sqrt(H[(size_t)i * hs]);
    st[i].bnorm = bnorm[i];
    target[i] = sp.rtol * bnorm[i];
    if (!std::isfinite(bnorm[i])) throw Error(STKKT_EINVAL, "kkt_solve_batch: non-finite right-hand side");
  }
  matvec_batch_run(mv, Xd, Td, act_cyc.as<int>(), s);
  hipLaunchKernelGGL(bsub_kernel, dim3(nch), dim3(kBT), 0, s, Rd, Bd, Td, chd, act_cyc.as<int>());
  bdot(Rd, 0, 1, Rd, act_cyc.as<int>(), hs, hd);
  fetch(count * hs);
  for (int i = 0; i < count; ++i) {
    beta[i] = std::sqrt(H[(size_t)i * hs]);
    st[i].rel_res_true = st[i].rel_res_est = bnorm[i] > 0 ? beta[i] / bnorm[i] : 0.0;
    if (bnorm[i] == 0.0 || (sp.fixed_iters == 0 && beta[i] <= target[i]) || beta[i] == 0.0) {
      state[i] = 1;
      st[i].converged = 1;
    }
  }
  std::vector<std::vector<double>> Hm(count), g(count), cs(count), sn(count);
  for (int i = 0; i < count; ++i) {
    Hm[i].assign((size_t)(m + 1) * m, 0.0);
    g[i].assign(m + 1, 0.0);
    cs[i].assign(m, 0.0);
    sn[i].assign(m, 0.0);
  }
  std::vector<int> kdone(count);
  for (;;) {
    int ncyc = 0;
    for (int i = 0; i < count; ++i) {
      h_cyc[i] = state[i] == 0 ? 1 : 0;
      h_step[i] = h_cyc[i];
      ncyc += h_cyc[i];
      kdone[i] = 0;
      std::fill(g[i].begin(), g[i].end(), 0.0);
      g[i][0] = beta[i];
    }
    if (ncyc == 0) break;
    upload_flags(h_cyc, act_cyc);
    upload_flags(h_step, act_step);
    // v_0 = r / beta (the squared norm is still in hd from the last residual)
    hipLaunchKernelGGL(bnormalize_kernel, dim3(nch), dim3(kBT), 0, s, Vd, Rd, hd, hs, chd, act_step.as<int>());
    STKKT_HIP(hipGetLastError());
    int nstep = ncyc;
    for (int j = 0; j < m && nstep > 0; ++j) {
      const int *act = act_step.as<int>();
      double *zj = Zd + (long long)j * Ntot;
      ras_batch_run(rb, Vd + (long long)j * Ntot, zj, act, h_step, s);
      matvec_batch_run(mv, zj, Wd, act, s);
      bdot(Vd, Ntot, j + 1, Wd, act, hs, hd);
      hipLaunchKernelGGL(bupdate_kernel, dim3(nch), dim3(kBT), 0, s, Wd, Vd, Ntot, j + 1, hd, hs, chd, act);
      bdot(Vd, Ntot, j + 1, Wd, act, hs, hd + (m + 1));
      hipLaunchKernelGGL(bupdate_kernel, dim3(nch), dim3(kBT), 0, s, Wd, Vd, Ntot, j + 1, hd + (m + 1), hs, chd,
                         act);
      bdot(Wd, 0, 1, Wd, act, hs, hd + 2 * (m + 1));
      fetch(count * hs);
      bool changed = false;
      for (int i = 0; i < count; ++i) {
        if (!h_step[i]) continue;
        const double *hi = H + (size_t)i * hs;
        const double hn = std::sqrt(hi[2 * (m + 1)]);
        std::vector<double> col(m + 1, 0.0);
        for (int q = 0; q <= j; ++q) col[q] = hi[q] + hi[(m + 1) + q];
        col[j + 1] = hn;
        for (int q = 0; q < j; ++q) {
          const double tmp = cs[i][q] * col[q] + sn[i][q] * col[q + 1];
          col[q + 1] = -sn[i][q] * col[q] + cs[i][q] * col[q + 1];
          col[q] = tmp;
        }
        const double d = std::hypot(col[j], col[j + 1]);
        double c = 1.0, sg = 0.0;
        if (d != 0.0) {
          c = col[j] / d;
          sg = col[j + 1] / d;
        }
        cs[i][j] = c;
        sn[i][j] = sg;
        col[j] = d;
        col[j + 1] = 0.0;
        for (int q = 0; q <= m; ++q) Hm[i][(size_t)q * m + j] = col[q];
        g[i][j + 1] = -sg * g[i][j];
        g[i][j] = c * g[i][j];
        st[i].iters += 1;
        kdone[i] = j + 1;
        const double est = std::fabs(g[i][j + 1]);
        bool leave = st[i].iters >= limit || hn == 0.0 || j + 1 == m;
        if (!std::isfinite(est) || !std::isfinite(hn)) {
          leave = true;
          state[i] = 3;
        }
        if (sp.fixed_iters == 0 && est <= target[i]) leave = true;
        if (leave) {
          h_step[i] = 0;
          changed = true;
          --nstep;
        }
      }
      if (changed) upload_flags(h_step, act_step);
      if (nstep > 0) {
        // v_{j+1} = w / |w| for the instances still in the cycle
        hipLaunchKernelGGL(bnormalize_kernel, dim3(nch), dim3(kBT), 0, s, Vd + (long long)(j + 1) * Ntot, Wd,
                           hd + 2 * (m + 1), hs, chd, act_step.as<int>());
        STKKT_HIP(hipGetLastError());
      }
    }
    // end of cycle: x += Z y for every instance that took part
    double *Y = hy.as<double>();
    for (int i = 0; i < count; ++i) {
      h_k[i] = 0;
      if (!h_cyc[i] || state[i] == 3) {
        h_cyc[i] = state[i] == 3 ? 0 : h_cyc[i];
        continue;
      }
      const int k = kdone[i];
      std::vector<double> y(k);
      for (int q = k - 1; q >= 0; --q) {
        double acc = g[i][q];
        for (int l = q + 1; l < k; ++l) acc -= Hm[i][(size_t)q * m + l] * y[l];
        y[q] = acc / Hm[i][(size_t)q * m + q];
      }
      for (int q = 0; q < k; ++q) Y[(size_t)i * m + q] = y[q];
      h_k[i] = k;
      st[i].rel_res_est = std::fabs(g[i][k]) / bnorm[i];
    }
    upload_flags(h_cyc, act_cyc);
    STKKT_HIP(hipMemcpyAsync(d_kcnt.ptr, h_k, sizeof(int) * count, hipMemcpyHostToDevice, s));
    STKKT_HIP(hipMemcpyAsync(ydev.ptr, Y, sizeof(double) * (size_t)count * m, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(bcombine_kernel, dim3(nch), dim3(kBT), 0, s, Xd, Zd, Ntot, ydev.as<double>(), m,
                       d_kcnt.as<int>(), chd, act_cyc.as<int>());
    STKKT_HIP(hipGetLastError());
    matvec_batch_run(mv, Xd, Td, act_cyc.as<int>(), s);
    hipLaunchKernelGGL(bsub_kernel, dim3(nch), dim3(kBT), 0, s, Rd, Bd, Td, chd, act_cyc.as<int>());
    bdot(Rd, 0, 1, Rd, act_cyc.as<int>(), hs, hd);
    fetch(count * hs);
    for (int i = 0; i < count; ++i) {
      if (!h_cyc[i]) continue;
      beta[i] = std::sqrt(H[(size_t)i * hs]);
      st[i].rel_res_true = beta[i] / bnorm[i];
      const bool ok = beta[i] <= target[i];
      if (!std::isfinite(beta[i])) {
        state[i] = 3;
      } else if (sp.fixed_iters > 0) {
        st[i].converged = ok ? 1 : 0;
        if (st[i].iters >= sp.fixed_iters) state[i] = 2;
        else st[i].restarts += 1;
      } else if (ok) {
        st[i].converged = 1;
        state[i] = 1;
      } else if (st[i].iters >= limit) {
        state[i] = 2;
      } else {
        st[i].restarts += 1;
      }
    }
  }
  for (int i = 0; i < count; ++i)
    STKKT_HIP(hipMemcpyAsync(x[i], Xd + voff[i], sizeof(double) * nloc[i], hipMemcpyDeviceToDevice, s));
  STKKT_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  int worst = STKKT_OK;
  for (int i = 0; i < count; ++i) {
    int status = STKKT_OK;
    if (state[i] == 3) status = STKKT_EBREAKDOWN;
    else if (!st[i].converged && sp.fixed_iters == 0) status = STKKT_NOT_CONVERGED;
    st[i].status = status;
    st[i].t_ms[0] = ms;
    if (status < 0) worst = status;
    else if (worst == STKKT_OK) worst = status;
    if (stats) stats[i] = st[i];
  }
  return worst;
}

}  // namespace stkkt
