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
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>

#include "batch.hpp"
#include "cgs2_dev.hpp"
#include "krylov.hpp"

namespace stkkt {

namespace {

constexpr int kBT = 256;          // threads per block
constexpr long long kChunk = 4096;   // elements per reduction chunk
constexpr int kGroup = 8;         // basis vectors per pass of the multi-dot
constexpr int kGraphSteps = 8;    // Arnoldi steps per captured graph (one host check each)

struct Chunk {
  int32_t inst, pad;
  int64_t lo, hi;   // element range in the concatenated vectors
};

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// The same for k <= 64 on the register tiles of the fused passes.
template <int KR>
__global__ void __launch_bounds__(kCgsThreads) bmultidot_tiles_kernel(const double *__restrict__ V, long long ldv,
                                                                      int k, const double *__restrict__ w,
                                                                      const Chunk *__restrict__ ch, int nch,
                                                                      const int *__restrict__ act,
                                                                      double *__restrict__ partial) {
  const Chunk c = load_uniform(ch + blockIdx.x);
  if (!as_const(act)[c.inst]) return;
  dot_range<KR>(w, V, ldv, k, c.lo, c.hi, partial + blockIdx.x, nch);
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
    if ((int)threadIdx.x < gk) {
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

// The fused CGS passes over the chunk work list (bodies shared with the single
// solve): w -= V h_inst with partial[g * nch + chunk] = chunk part of V_g . w_new,
// and w -= V h_inst with partial[chunk] = chunk part of |w_new|^2.
template <int KR>
__global__ void __launch_bounds__(kCgsThreads) bupdate_dot_kernel(double *__restrict__ w,
                                                                  const double *__restrict__ V, long long ldv, int k,
                                                                  const double *__restrict__ h, int hstride,
                                                                  const Chunk *__restrict__ ch, int nch,
                                                                  const int *__restrict__ act,
                                                                  double *__restrict__ partial) {
  const Chunk c = load_uniform(ch + blockIdx.x);
  if (!as_const(act)[c.inst]) return;
  update_dot_range<KR>(w, V, ldv, k, h + (long long)c.inst * hstride, c.lo, c.hi, partial + blockIdx.x, nch);
}

template <int KR>
__global__ void __launch_bounds__(kCgsThreads) bupdate_norm_kernel(double *__restrict__ w,
                                                                   const double *__restrict__ V, long long ldv, int k,
                                                                   const double *__restrict__ h, int hstride,
                                                                   const Chunk *__restrict__ ch,
                                                                   const int *__restrict__ act,
                                                                   double *__restrict__ partial) {
  const Chunk c = load_uniform(ch + blockIdx.x);
  if (!as_const(act)[c.inst]) return;
  const double s = update_norm_range<KR>(w, V, ldv, k, h + (long long)c.inst * hstride, c.lo, c.hi);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
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

// Givens arithmetic shared by the host (one check per step) and the device
// (graph form), written out with no fused multiply-adds so that both give
// the same bits: a member's result does not depend on which form ran it.
__host__ __device__ inline void rot_apply(double c, double s, double a, double b, double &na, double &nb) {
#pragma clang fp contract(off)
  na = c * a + s * b;
  nb = -s * a + c * b;
}

// c, s, d with c x + s y = d, -s x + c y = 0 (d = sqrt(x^2 + y^2), scaled)
__host__ __device__ inline void rot_make(double x, double y, double &c, double &s, double &d) {
#pragma clang fp contract(off)
  const double ax = x < 0 ? -x : x, ay = y < 0 ? -y : y;
  const double big = ax > ay ? ax : ay, small = ax > ay ? ay : ax;
  if (big == 0.0) {
    c = 1.0, s = 0.0, d = 0.0;
    return;
  }
  const double r = small / big;
  d = big * sqrt(1.0 + r * r);
  c = x / d;
  s = y / d;
}

// Arnoldi step j of every member still in its cycle (one thread per member):
// the new Hessenberg column from the two CGS passes, the member's previous
// Givens rotations applied to it, the new rotation, the residual estimate
// |g[j+1]|.  A member leaves the cycle (its flag in act cleared) when the
// estimate meets its target, at its step limit, at the end of the cycle, or
// on a zero or non-finite norm (non-finite: breakdown flag).  Per member, st
// holds cs[m], sn[m], g[m+1], H[(m+1) m] (H[q m + j]); in: iters, kdone,
// breakdown.
__global__ void bgivens_kernel(int j, int m, int S, const double *__restrict__ hd, int hs, double *__restrict__ st,
                               long long stride, int *__restrict__ in, const double *__restrict__ tgt, int limit,
                               int fixed, int *__restrict__ act) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S || !act[i]) return;
  const double *h = hd + (long long)i * hs;
  double *cs = st + i * stride, *sn = cs + m, *g = sn + m, *H = g + (m + 1);
  int *ci = in + 4 * i;
  const double hn = sqrt(h[2 * (m + 1)]);
  // the column is rotated top down with one carried entry: entry q is final
  // once rotation q has been applied
  double a = h[0] + h[m + 1];
  for (int q = 0; q < j; ++q) {
    const double b = h[q + 1] + h[(m + 1) + q + 1];
    double na, nb;
    rot_apply(cs[q], sn[q], a, b, na, nb);
    H[(long long)q * m + j] = na;
    a = nb;
  }
  double c, sg, d;
  rot_make(a, hn, c, sg, d);
  cs[j] = c;
  sn[j] = sg;
  H[(long long)j * m + j] = d;
  H[(long long)(j + 1) * m + j] = 0.0;
  g[j + 1] = -sg * g[j];
  g[j] = c * g[j];
  ci[0] += 1;
  ci[1] = j + 1;
  const double est = fabs(g[j + 1]);
  bool leave = ci[0] >= limit || hn == 0.0 || j + 1 == m;
  if (!isfinite(est) || !isfinite(hn)) {
    leave = true;
    ci[2] = 1;
  }
  if (fixed == 0 && est <= tgt[i]) leave = true;
  if (leave) act[i] = 0;
}

// start of a cycle: g = (beta, 0, ..., 0) for the members in act
__global__ void bcycle_init_kernel(int m, int S, double *__restrict__ st, long long stride,
                                   const double *__restrict__ beta, const int *__restrict__ act) {
  const int i = blockIdx.y;
  if (i >= S || !act[i]) return;
  double *g = st + i * stride + 2 * m;
  for (int q = threadIdx.x; q <= m; q += blockDim.x) g[q] = q == 0 ? beta[i] : 0.0;
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


}  // namespace


PinnedBlock::PinnedBlock(size_t bytes) {
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) p = nullptr;
  if (!p) throw Error(STKKT_ENOMEM, "batch: pinned host allocation failed");
}

PinnedBlock::~PinnedBlock() {
  if (p) (void)hipHostFree(p);
}

BatchEngine::BatchEngine(const Allocator *al, const solve_params_t &sp, long long capacity, int slots,
                         hipStream_t s)
    : al_(al), sp_(sp), s_(s), cap_((capacity + 255) / 256 * 256), m_(sp.restart), hs_(2 * (sp.restart + 1) + 2),
      slots_(slots) {
  STKKT_REQUIRE(slots >= 1 && cap_ >= 256, "batch: empty engine");
  const size_t m = (size_t)m_, N = (size_t)cap_;
  V_ = DevBuf(al, sizeof(double) * (m + 1) * N);
  Z_ = DevBuf(al, sizeof(double) * m * N);
  B_ = DevBuf(al, sizeof(double) * N);
  X_ = DevBuf(al, sizeof(double) * N);
  R_ = DevBuf(al, sizeof(double) * N);
  W_ = DevBuf(al, sizeof(double) * N);
  T_ = DevBuf(al, sizeof(double) * N);
  const long long max_chunks = cap_ / kChunk + slots;
  partial_ = DevBuf(al, sizeof(double) * (m + 1) * (size_t)max_chunks);
  hdev_ = DevBuf(al, sizeof(double) * (size_t)slots * hs_);
  ydev_ = DevBuf(al, sizeof(double) * (size_t)slots * m);
  chunks_ = DevBuf(al, sizeof(Chunk) * (size_t)max_chunks);
  cfirst_ = DevBuf(al, sizeof(int) * (size_t)(slots + 1));
  kcnt_ = DevBuf(al, sizeof(int) * (size_t)slots);
  act_a_ = DevBuf(al, sizeof(int) * (size_t)slots);
  act_b_ = DevBuf(al, sizeof(int) * (size_t)slots);
  act_c_ = DevBuf(al, sizeof(int) * (size_t)slots);
  hh_ = std::make_unique<PinnedBlock>(sizeof(double) * (size_t)slots * hs_);
  hy_ = std::make_unique<PinnedBlock>(sizeof(double) * (size_t)slots * m);
  hflags_ = std::make_unique<PinnedBlock>(sizeof(int) * 4 * (size_t)slots);
  gstride_ = 2 * (long long)m + (m + 1) + (long long)(m + 1) * m;
  gst_ = DevBuf(al, sizeof(double) * (size_t)slots * gstride_);
  gin_ = DevBuf(al, sizeof(int) * 4 * (size_t)slots);
  gtg_ = DevBuf(al, sizeof(double) * 2 * (size_t)slots);
  hg_ = std::make_unique<PinnedBlock>(sizeof(double) * ((size_t)slots * gstride_ + 2 * (size_t)slots) +
                                      sizeof(int) * 4 * (size_t)slots);
  fill_zero(V_.as<double>(), (long long)((m + 1) * N), s);
  fill_zero(Z_.as<double>(), (long long)(m * N), s);
  fill_zero(B_.as<double>(), cap_, s);
  fill_zero(X_.as<double>(), cap_, s);
  fill_zero(R_.as<double>(), cap_, s);
  fill_zero(W_.as<double>(), cap_, s);
  fill_zero(T_.as<double>(), cap_, s);
  free_[0] = cap_;
}

BatchEngine::~BatchEngine() {
  drop_graphs();
  if (cs_) (void)hipStreamDestroy(cs_);
}

void BatchEngine::drop_graphs() {
  for (hipGraphExec_t e : graphs_) (void)hipGraphExecDestroy(e);
  graphs_.clear();
}

long long BatchEngine::free_elems() const {
  long long f = 0;
  for (auto &kv : free_) f += kv.second;
  return f;
}

size_t BatchEngine::member_bytes(const kkt_op *op, const ras *R, const coarse *C) {
  size_t b = ras_local_bytes(R);
  if (C) b += sizeof(double) * 3 * (size_t)op->d.V;   // the coarse correction y
  return b;
}

int BatchEngine::admit(const kkt_op *op, const ras *R, const coarse *C) {
  STKKT_REQUIRE(op && R && R->op == op, "batch: preconditioner built for another operator");
  STKKT_REQUIRE(!C || coarse_built_for(C, op), "batch: coarse level built for another operator");
  int slot = -1;
  for (int i = 0; i < (int)slots_.size(); ++i)
    if (!slots_[i].used) {
      slot = i;
      break;
    }
  if (slot < 0) return -1;
  const long long n = 3 * op->d.V, need = (n + 255) / 256 * 256;
  auto it = free_.begin();
  for (; it != free_.end(); ++it)
    if (it->second >= need) break;
  if (it == free_.end()) return -1;
  // everything that can fail (allocations, host vectors) is done before the
  // slot and the vector range are taken, so a failure leaves the engine as it was
  DevBuf local(al_, ras_local_bytes(R));
  DevBuf y2 = C ? DevBuf(al_, sizeof(double) * n) : DevBuf();
  std::vector<double> Hm((size_t)(m_ + 1) * m_, 0.0), g(m_ + 1, 0.0), cs(m_, 0.0), sn(m_, 0.0);
  STKKT_HIP(hipMemsetAsync(local.ptr, 0, local.bytes, s_));
  const long long off = it->first, len = it->second;
  free_.erase(it);
  if (len > need) free_[off + need] = len - need;
  Slot &sl = slots_[slot];
  sl = Slot{};
  sl.used = true;
  sl.op = op;
  sl.R = R;
  sl.C = C;
  sl.voff = off;
  sl.n = n;
  sl.local = std::move(local);
  sl.y2 = std::move(y2);
  sl.Hm = std::move(Hm);
  sl.g = std::move(g);
  sl.cs = std::move(cs);
  sl.sn = std::move(sn);
  sl.t0 = std::chrono::steady_clock::now();
  ++nused_;
  dirty_ = true;
  return slot;
}

void BatchEngine::release(int slot) {
  Slot &sl = slots_[slot];
  if (!sl.used) return;
  STKKT_HIP(hipStreamSynchronize(s_));   // nothing in flight may still use the slot's buffers
  const long long need = (sl.n + 255) / 256 * 256;
  long long off = sl.voff, len = need;
  // coalesce with the neighbouring free ranges
  auto nx = free_.lower_bound(off);
  if (nx != free_.end() && nx->first == off + len) {
    len += nx->second;
    free_.erase(nx);
  }
  auto pv = free_.lower_bound(off);
  if (pv != free_.begin()) {
    --pv;
    if (pv->first + pv->second == off) {
      off = pv->first;
      len += pv->second;
      free_.erase(pv);
    }
  }
  free_[off] = len;
  sl = Slot{};
  --nused_;
  dirty_ = true;
}

void BatchEngine::rebuild() {
  const int S = (int)slots_.size();
  std::vector<Chunk> ch;
  std::vector<int> cf(S + 1);
  std::vector<const kkt_op *> ops(S, nullptr);
  std::vector<const ras *> rs(S, nullptr);
  std::vector<void *> loc(S, nullptr);
  std::vector<long long> voff(S, 0);
  for (int i = 0; i < S; ++i) {
    cf[i] = (int)ch.size();
    const Slot &sl = slots_[i];
    if (!sl.used) continue;
    for (long long lo = 0; lo < sl.n; lo += kChunk)
      ch.push_back(Chunk{i, 0, sl.voff + lo, sl.voff + std::min(sl.n, lo + kChunk)});
    ops[i] = sl.op;
    rs[i] = sl.R;
    loc[i] = sl.local.ptr;
    voff[i] = sl.voff;
  }
  cf[S] = (int)ch.size();
  nch_ = (int)ch.size();
  if (nch_) STKKT_HIP(hipMemcpyAsync(chunks_.ptr, ch.data(), sizeof(Chunk) * ch.size(), hipMemcpyHostToDevice, s_));
  STKKT_HIP(hipMemcpyAsync(cfirst_.ptr, cf.data(), sizeof(int) * cf.size(), hipMemcpyHostToDevice, s_));
  matvec_batch_prepare(ops.data(), voff.data(), S, al_, mv_, s_);   // synchronises: ch, cf may go
  ras_batch_prepare(rs.data(), voff.data(), loc.data(), S, al_, rb_, s_);
  drop_graphs();   // captured with the previous composition's work lists
  dirty_ = false;
}

void BatchEngine::upload(int *host, DevBuf &dev) {
  STKKT_HIP(hipMemcpyAsync(dev.ptr, host, sizeof(int) * slots_.size(), hipMemcpyHostToDevice, s_));
}

void BatchEngine::bdot(const double *V, long long ldv, int k, const double *w, const int *act, double *out) {
  if (nch_ == 0) return;
  const Chunk *chd = chunks_.as<Chunk>();
  double *part = partial_.as<double>();
  if (k <= kCgsHalf)
    hipLaunchKernelGGL(bmultidot_tiles_kernel<kCgsHalf>, dim3(nch_), dim3(kCgsThreads), 0, s_, V, ldv, k, w, chd, nch_,
                       act, part);
  else if (k <= 48)
    hipLaunchKernelGGL(bmultidot_tiles_kernel<48>, dim3(nch_), dim3(kCgsThreads), 0, s_, V, ldv, k, w, chd, nch_, act,
                       part);
  else if (k <= 56)
    hipLaunchKernelGGL(bmultidot_tiles_kernel<56>, dim3(nch_), dim3(kCgsThreads), 0, s_, V, ldv, k, w, chd, nch_, act,
                       part);
  else if (k <= kCgsMaxK)
    hipLaunchKernelGGL(bmultidot_tiles_kernel<kCgsMaxK>, dim3(nch_), dim3(kCgsThreads), 0, s_, V, ldv, k, w, chd, nch_,
                       act, part);
  else
    hipLaunchKernelGGL(bmultidot_kernel, dim3(nch_), dim3(kBT), 0, s_, V, ldv, k, w, chd, nch_, act, part);
  hipLaunchKernelGGL(breduce_kernel, dim3((unsigned)slots_.size(), k), dim3(kBT), 0, s_, partial_.as<double>(), nch_,
                     cfirst_.as<int>(), act, hs_, out);
  STKKT_HIP(hipGetLastError());
}

void BatchEngine::fetch() {
  STKKT_HIP(hipMemcpyAsync(hh_->p, hdev_.ptr, sizeof(double) * slots_.size() * hs_, hipMemcpyDeviceToHost, s_));
  STKKT_HIP(hipStreamSynchronize(s_));
}

// z_j = M^{-1} v_j for the members flagged in act.  Two-level members first
// get their coarse corrections y (one multi-right-hand-side coarse
// application per coarse level) and t = v - F y (in T_ at their offsets);
// then one batched RAS launch applies M_one^{-1} to v (one-level members)
// and to t (two-level members), and z += y finishes the two-level members.
void BatchEngine::precondition(int j, const int *act_dev) {
  const long long N = cap_;
  const double *v = V_.as<double>() + (long long)j * N;
  double *z = Z_.as<double>() + (long long)j * N;
  int *hf = hflags_->as<int>();
  const int S = (int)slots_.size();
  int *h_ras = hf + 3 * S;
  bool any_two = false;
  for (int i = 0; i < S; ++i) {
    h_ras[i] = hf[i] && slots_[i].C == nullptr;
    any_two = any_two || (hf[i] && slots_[i].C != nullptr);
  }
  if (!any_two) {
    ras_batch_run(rb_, v, z, act_dev, hf, s_);
    return;
  }
  // y = I_c^h F_c^{-1} I_h^c v, grouped by coarse level
  std::vector<const coarse *> seen;
  std::vector<const double *> xs;
  std::vector<double *> ys;
  for (int i = 0; i < S; ++i) {
    const coarse *C = slots_[i].C;
    if (!hf[i] || !C || std::find(seen.begin(), seen.end(), C) != seen.end()) continue;
    seen.push_back(C);
    xs.clear();
    ys.clear();
    for (int k = i; k < S; ++k)
      if (hf[k] && slots_[k].C == C) {
        xs.push_back(v + slots_[k].voff);
        ys.push_back(slots_[k].y2.as<double>());
      }
    coarse_apply_multi_device(C, (int)xs.size(), xs.data(), ys.data(), s_);
  }
  // z = y + M_one^{-1} (v - F y)
  double *T = T_.as<double>();
  for (int i = 0; i < S; ++i) {
    const Slot &sl = slots_[i];
    if (!hf[i] || !sl.C) continue;
    double *t = T + sl.voff;
    matvec_device(sl.op, sl.y2.as<double>(), t, s_);
    axpby(t, 1.0, v + sl.voff, -1.0, t, sl.n, s_);
    h_ras[i] = 2;
  }
  upload(h_ras, act_c_);
  ras_batch_run(rb_, v, z, act_c_.as<int>(), h_ras, s_, T);
  for (int i = 0; i < S; ++i) {
    const Slot &sl = slots_[i];
    if (!hf[i] || !sl.C) continue;
    double *zi = z + sl.voff;
    axpby(zi, 1.0, zi, 1.0, sl.y2.as<double>(), sl.n, s_);
  }
}

// CGS2 of step j for the members in act: h1 = V^T w; w -= V h1 with
// h2 = V^T w; w -= V h2 with |w|^2 (into hd at 0, m+1 and 2(m+1))
void BatchEngine::cgs2(int j, const int *act) {
  const int m = m_, hs = hs_;
  const long long N = cap_;
  double *hd = hdev_.as<double>(), *Vd = V_.as<double>(), *Wd = W_.as<double>();
  const Chunk *chd = chunks_.as<Chunk>();
  bdot(Vd, N, j + 1, Wd, act, hd);
  if (cgs2_fused_ok(j + 1) && nch_ > 0) {
    double *part = partial_.as<double>();
    const int *cf = cfirst_.as<int>();
    const unsigned S = (unsigned)slots_.size();
    if (j + 1 <= kCgsHalf)
      hipLaunchKernelGGL(bupdate_dot_kernel<kCgsHalf>, dim3(nch_), dim3(kCgsThreads), 0, s_, Wd, Vd, N, j + 1, hd, hs,
                         chd, nch_, act, part);
    else if (j + 1 <= 48)
      hipLaunchKernelGGL(bupdate_dot_kernel<48>, dim3(nch_), dim3(kCgsThreads), 0, s_, Wd, Vd, N, j + 1, hd, hs, chd,
                         nch_, act, part);
    else if (j + 1 <= 56)
      hipLaunchKernelGGL(bupdate_dot_kernel<56>, dim3(nch_), dim3(kCgsThreads), 0, s_, Wd, Vd, N, j + 1, hd, hs, chd,
                         nch_, act, part);
    else
      hipLaunchKernelGGL(bupdate_dot_kernel<kCgsMaxK>, dim3(nch_), dim3(kCgsThreads), 0, s_, Wd, Vd, N, j + 1, hd, hs,
                         chd, nch_, act, part);
    hipLaunchKernelGGL(breduce_kernel, dim3(S, j + 1), dim3(kBT), 0, s_, part, nch_, cf, act, hs, hd + (m + 1));
    if (j + 1 <= kCgsHalf)
      hipLaunchKernelGGL(bupdate_norm_kernel<kCgsHalf>, dim3(nch_), dim3(kCgsThreads), 0, s_, Wd, Vd, N, j + 1,
                         hd + (m + 1), hs, chd, act, part);
    else if (j + 1 <= 48)
      hipLaunchKernelGGL(bupdate_norm_kernel<48>, dim3(nch_), dim3(kCgsThreads), 0, s_, Wd, Vd, N, j + 1, hd + (m + 1),
                         hs, chd, act, part);
    else
      hipLaunchKernelGGL(bupdate_norm_kernel<kCgsMaxK>, dim3(nch_), dim3(kCgsThreads), 0, s_, Wd, Vd, N, j + 1,
                         hd + (m + 1), hs, chd, act, part);
    hipLaunchKernelGGL(breduce_kernel, dim3(S, 1), dim3(kBT), 0, s_, part, nch_, cf, act, hs, hd + 2 * (m + 1));
    STKKT_HIP(hipGetLastError());
  } else {
    hipLaunchKernelGGL(bupdate_kernel, dim3(nch_), dim3(kBT), 0, s_, Wd, Vd, N, j + 1, hd, hs, chd, act);
    bdot(Vd, N, j + 1, Wd, act, hd + (m + 1));
    hipLaunchKernelGGL(bupdate_kernel, dim3(nch_), dim3(kBT), 0, s_, Wd, Vd, N, j + 1, hd + (m + 1), hs, chd, act);
    bdot(Wd, 0, 1, Wd, act, hd + 2 * (m + 1));
  }
}

// Step j with no host involvement: z_j, w = F z_j, CGS2, the rotations on
// the device (members leaving the cycle drop out of act_a_), v_{j+1}.
void BatchEngine::arnoldi_step(int j) {
  const int S = (int)slots_.size(), m = m_, hs = hs_;
  const long long N = cap_;
  int *act = act_a_.as<int>();
  double *hd = hdev_.as<double>(), *Vd = V_.as<double>(), *Zd = Z_.as<double>(), *Wd = W_.as<double>();
  ras_batch_run(rb_, Vd + (long long)j * N, Zd + (long long)j * N, act, hflags_->as<int>(), s_);
  matvec_batch_run(mv_, Zd + (long long)j * N, Wd, act, s_);
  cgs2(j, act);
  const int limit = sp_.fixed_iters > 0 ? sp_.fixed_iters : sp_.maxit;
  hipLaunchKernelGGL(bgivens_kernel, dim3((S + 63) / 64), dim3(64), 0, s_, j, m, S, hd, hs, gst_.as<double>(), gstride_,
                     gin_.as<int>(), gtg_.as<double>(), limit, sp_.fixed_iters, act);
  if (j + 1 < m)
    hipLaunchKernelGGL(bnormalize_kernel, dim3(nch_), dim3(kBT), 0, s_, Vd + (long long)(j + 1) * N, Wd,
                       hd + 2 * (m + 1), hs, chunks_.as<Chunk>(), act);
  STKKT_HIP(hipGetLastError());
}

// One cycle of the running members (flags run[], already in act_a_, v_0
// formed) from captured graphs of kGraphSteps steps each, captured once per
// composition on an engine stream and replayed on the engine's stream; one
// host check of the flags per graph.  Afterwards each member's rotations,
// Hessenberg columns and step counts are copied back to its slot.
void BatchEngine::cycle_graph(const int *run, int S) {
  const int m = m_;
  double *hgd = hg_->as<double>();
  int *hgi = reinterpret_cast<int *>(hgd + (size_t)S * gstride_ + 2 * (size_t)S);
  double *tg = hgd + (size_t)S * gstride_;
  for (int i = 0; i < S; ++i) {
    tg[i] = slots_[i].target;
    tg[S + i] = slots_[i].beta;
    hgi[4 * i] = slots_[i].st.iters;
    hgi[4 * i + 1] = hgi[4 * i + 2] = hgi[4 * i + 3] = 0;
  }
  STKKT_HIP(hipMemcpyAsync(gtg_.ptr, tg, sizeof(double) * 2 * S, hipMemcpyHostToDevice, s_));
  STKKT_HIP(hipMemcpyAsync(gin_.ptr, hgi, sizeof(int) * 4 * S, hipMemcpyHostToDevice, s_));
  hipLaunchKernelGGL(bcycle_init_kernel, dim3(1, S), dim3(64), 0, s_, m, S, gst_.as<double>(), gstride_,
                     gtg_.as<double>() + S, act_a_.as<int>());
  STKKT_HIP(hipGetLastError());
  if (graphs_.empty()) {
    if (!cs_) STKKT_HIP(hipStreamCreateWithFlags(&cs_, hipStreamNonBlocking));
    for (int j0 = 0; j0 < m; j0 += kGraphSteps) {
      hipGraph_t g = nullptr;
      STKKT_HIP(hipStreamBeginCapture(cs_, hipStreamCaptureModeThreadLocal));
      std::swap(s_, cs_);
      try {
        for (int j = j0; j < std::min(m, j0 + kGraphSteps); ++j) arnoldi_step(j);
      } catch (...) {
        std::swap(s_, cs_);
        (void)hipStreamEndCapture(cs_, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      std::swap(s_, cs_);
      STKKT_HIP(hipStreamEndCapture(cs_, &g));
      hipGraphExec_t e = nullptr;
      const hipError_t rc = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      STKKT_HIP(rc);
      graphs_.push_back(e);
    }
  }
  int *hact = hflags_->as<int>() + 3 * S;
  for (hipGraphExec_t e : graphs_) {
    STKKT_HIP(hipGraphLaunch(e, s_));
    STKKT_HIP(hipMemcpyAsync(hact, act_a_.ptr, sizeof(int) * S, hipMemcpyDeviceToHost, s_));
    STKKT_HIP(hipStreamSynchronize(s_));
    bool any = false;
    for (int i = 0; i < S; ++i) any = any || hact[i] != 0;
    if (!any) break;
  }
  STKKT_HIP(hipMemcpyAsync(hgd, gst_.ptr, sizeof(double) * (size_t)S * gstride_, hipMemcpyDeviceToHost, s_));
  STKKT_HIP(hipMemcpyAsync(hgi, gin_.ptr, sizeof(int) * 4 * S, hipMemcpyDeviceToHost, s_));
  STKKT_HIP(hipStreamSynchronize(s_));
  for (int i = 0; i < S; ++i) {
    if (!run[i]) continue;
    Slot &sl = slots_[i];
    const double *st = hgd + (size_t)i * gstride_;
    std::copy(st + 2 * m, st + 3 * m + 1, sl.g.begin());
    std::copy(st + 3 * m + 1, st + 3 * m + 1 + (size_t)(m + 1) * m, sl.Hm.begin());
    sl.st.iters = hgi[4 * i];
    sl.kdone = hgi[4 * i + 1];
    if (hgi[4 * i + 2]) sl.breakdown = true;
  }
}

void BatchEngine::cycle(std::vector<int> &finished) {
  if (dirty_) rebuild();
  const int S = (int)slots_.size(), m = m_, hs = hs_;
  const long long N = cap_;
  int *hf = hflags_->as<int>();
  int *h_step = hf, *h_cyc = hf + S, *h_k = hf + 2 * S;
  const double *H = hh_->as<double>();
  double *hd = hdev_.as<double>(), *Vd = V_.as<double>(), *Zd = Z_.as<double>(), *Bd = B_.as<double>(),
         *Xd = X_.as<double>(), *Rd = R_.as<double>(), *Wd = W_.as<double>(), *Td = T_.as<double>();
  const Chunk *chd = chunks_.as<Chunk>();
  const int limit = sp_.fixed_iters > 0 ? sp_.fixed_iters : sp_.maxit;
  auto finish = [&](int i) {
    Slot &sl = slots_[i];
    sl.state = 2;
    int status = STKKT_OK;
    if (sl.breakdown) status = STKKT_EBREAKDOWN;
    else if (!sl.st.converged && sp_.fixed_iters == 0) status = STKKT_NOT_CONVERGED;
    sl.st.status = status;
    sl.st.t_ms[0] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - sl.t0).count();
    finished.push_back(i);
  };

  // newly admitted members: ||b||, r = b - F x0, ||r||
  int nnew = 0;
  for (int i = 0; i < S; ++i) {
    h_cyc[i] = slots_[i].used && slots_[i].state == 0;
    nnew += h_cyc[i];
  }
  if (nnew) {
    upload(h_cyc, act_b_);
    const int *act = act_b_.as<int>();
    bdot(Bd, 0, 1, Bd, act, hd);
    fetch();
    for (int i = 0; i < S; ++i) {
      if (!h_cyc[i]) continue;
      Slot &sl = slots_[i];
      sl.bnorm = std::sqrt(H[(size_t)i * hs]);
      sl.st.bnorm = sl.bnorm;
      sl.target = sp_.rtol * sl.bnorm;
    }
    matvec_batch_run(mv_, Xd, Td, act, s_);
    hipLaunchKernelGGL(bsub_kernel, dim3(nch_), dim3(kBT), 0, s_, Rd, Bd, Td, chd, act);
    bdot(Rd, 0, 1, Rd, act, hd);
    fetch();
    for (int i = 0; i < S; ++i) {
      if (!h_cyc[i]) continue;
      Slot &sl = slots_[i];
      sl.beta = std::sqrt(H[(size_t)i * hs]);
      sl.st.rel_res_true = sl.st.rel_res_est = sl.bnorm > 0 ? sl.beta / sl.bnorm : 0.0;
      sl.state = 1;
      if (!std::isfinite(sl.bnorm) || !std::isfinite(sl.beta)) {
        sl.breakdown = true;
        finish(i);
      } else if (sl.bnorm == 0.0) {
        // F x = 0 has the solution x = 0 whatever x0 was (as kkt_solve returns)
        fill_zero(Xd + sl.voff, sl.n, s_);
        sl.st.rel_res_true = sl.st.rel_res_est = 0.0;
        sl.st.converged = 1;
        finish(i);
      } else if (sl.beta == 0.0 || (sp_.fixed_iters == 0 && sl.beta <= sl.target)) {
        sl.st.converged = 1;
        finish(i);
      }
    }
  }
  // one cycle of every running member
  int ncyc = 0;
  for (int i = 0; i < S; ++i) {
    Slot &sl = slots_[i];
    h_cyc[i] = sl.used && sl.state == 1;
    h_step[i] = h_cyc[i];
    ncyc += h_cyc[i];
    if (h_cyc[i]) {
      sl.kdone = 0;
      std::fill(sl.g.begin(), sl.g.end(), 0.0);
      sl.g[0] = sl.beta;
    }
  }
  if (ncyc == 0) return;
  upload(h_cyc, act_b_);
  upload(h_step, act_a_);
  // v_0 = r / beta: |r|^2 of every running member is in hd (last residual)
  hipLaunchKernelGGL(bnormalize_kernel, dim3(nch_), dim3(kBT), 0, s_, Vd, Rd, hd, hs, chd, act_a_.as<int>());
  STKKT_HIP(hipGetLastError());
  bool graph = sp_.graph != 0 && ras_batch_single_launch(rb_);
  for (int i = 0; i < S && graph; ++i)
    if (h_cyc[i] && slots_[i].C) graph = false;
  int nstep = graph ? 0 : ncyc;
  if (graph) cycle_graph(h_cyc, S);
  std::vector<double> col(m + 1);
  for (int j = 0; j < m && nstep > 0; ++j) {
    const int *act = act_a_.as<int>();
    double *zj = Zd + (long long)j * N;
    precondition(j, act);
    matvec_batch_run(mv_, zj, Wd, act, s_);
    cgs2(j, act);
    fetch();
    bool changed = false;
    for (int i = 0; i < S; ++i) {
      if (!h_step[i]) continue;
      Slot &sl = slots_[i];
      const double *hi = H + (size_t)i * hs;
      const double hn = std::sqrt(hi[2 * (m + 1)]);
      std::fill(col.begin(), col.end(), 0.0);
      for (int q = 0; q <= j; ++q) col[q] = hi[q] + hi[(m + 1) + q];
      col[j + 1] = hn;
      for (int q = 0; q < j; ++q) rot_apply(sl.cs[q], sl.sn[q], col[q], col[q + 1], col[q], col[q + 1]);
      double c, sg, d;
      rot_make(col[j], col[j + 1], c, sg, d);
      sl.cs[j] = c;
      sl.sn[j] = sg;
      col[j] = d;
      col[j + 1] = 0.0;
      for (int q = 0; q <= m; ++q) sl.Hm[(size_t)q * m + j] = col[q];
      sl.g[j + 1] = -sg * sl.g[j];
      sl.g[j] = c * sl.g[j];
      sl.st.iters += 1;
      sl.kdone = j + 1;
      const double est = std::fabs(sl.g[j + 1]);
      bool leave = sl.st.iters >= limit || hn == 0.0 || j + 1 == m;
      if (!std::isfinite(est) || !std::isfinite(hn)) {
        leave = true;
        sl.breakdown = true;
      }
      if (sp_.fixed_iters == 0 && est <= sl.target) leave = true;
      if (leave) {
        h_step[i] = 0;
        changed = true;
        --nstep;
      }
    }
    if (changed) upload(h_step, act_a_);
    if (nstep > 0) {
      hipLaunchKernelGGL(bnormalize_kernel, dim3(nch_), dim3(kBT), 0, s_, Vd + (long long)(j + 1) * N, Wd,
                         hd + 2 * (m + 1), hs, chd, act_a_.as<int>());
      STKKT_HIP(hipGetLastError());
    }
  }
  // end of cycle: x += Z y, true residual
  double *Y = hy_->as<double>();
  for (int i = 0; i < S; ++i) {
    h_k[i] = 0;
    if (!h_cyc[i]) continue;
    Slot &sl = slots_[i];
    if (sl.breakdown) {
      h_cyc[i] = 0;
      finish(i);
      continue;
    }
    const int k = sl.kdone;
    for (int q = k - 1; q >= 0; --q) {
      double acc = sl.g[q];
      for (int l = q + 1; l < k; ++l) acc -= sl.Hm[(size_t)q * m + l] * Y[(size_t)i * m + l];
      Y[(size_t)i * m + q] = acc / sl.Hm[(size_t)q * m + q];
    }
    h_k[i] = k;
    sl.st.rel_res_est = std::fabs(sl.g[k]) / sl.bnorm;
  }
  upload(h_cyc, act_b_);
  STKKT_HIP(hipMemcpyAsync(kcnt_.ptr, h_k, sizeof(int) * S, hipMemcpyHostToDevice, s_));
  STKKT_HIP(hipMemcpyAsync(ydev_.ptr, Y, sizeof(double) * (size_t)S * m, hipMemcpyHostToDevice, s_));
  const int *actb = act_b_.as<int>();
  hipLaunchKernelGGL(bcombine_kernel, dim3(nch_), dim3(kBT), 0, s_, Xd, Zd, N, ydev_.as<double>(), m,
                     kcnt_.as<int>(), chd, actb);
  STKKT_HIP(hipGetLastError());
  matvec_batch_run(mv_, Xd, Td, actb, s_);
  hipLaunchKernelGGL(bsub_kernel, dim3(nch_), dim3(kBT), 0, s_, Rd, Bd, Td, chd, actb);
  bdot(Rd, 0, 1, Rd, actb, hd);
  fetch();
  for (int i = 0; i < S; ++i) {
    if (!h_cyc[i]) continue;
    Slot &sl = slots_[i];
    sl.beta = std::sqrt(H[(size_t)i * hs]);
    sl.st.rel_res_true = sl.beta / sl.bnorm;
    const bool ok = sl.beta <= sl.target;
    if (!std::isfinite(sl.beta)) {
      sl.breakdown = true;
      finish(i);
    } else if (sp_.fixed_iters > 0) {
      sl.st.converged = ok ? 1 : 0;
      if (sl.st.iters >= sp_.fixed_iters) finish(i);
      else sl.st.restarts += 1;
    } else if (ok) {
      sl.st.converged = 1;
      finish(i);
    } else if (sl.st.iters >= limit) {
      finish(i);
    } else {
      sl.st.restarts += 1;
    }
  }
}

int gmres_solve_batch(int count, const kkt_op *const *ops, const ras *const *R, const solve_params_t &sp,
                      const double *const *b, double *const *x, hipStream_t s, kkt_stats_t *stats) {
  long long cap = 0;
  for (int i = 0; i < count; ++i) cap += (3 * ops[i]->d.V + 255) / 256 * 256;
  BatchEngine eng(&ops[0]->al, sp, cap, count, s);
  std::vector<int> slot(count), member(count);
  for (int i = 0; i < count; ++i) {
    slot[i] = eng.admit(ops[i], R[i], nullptr);
    STKKT_REQUIRE(slot[i] >= 0, "kkt_solve_batch: internal capacity error");
    member[slot[i]] = i;
    const long long n = eng.size_of(slot[i]);
    STKKT_HIP(hipMemcpyAsync(eng.b_of(slot[i]), b[i], sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    STKKT_HIP(hipMemcpyAsync(eng.x_of(slot[i]), x[i], sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  }
  std::vector<int> done;
  int worst = STKKT_OK, left = count;
  while (left > 0) {
    done.clear();
    eng.cycle(done);
    for (int sl : done) {
      const int i = member[sl];
      STKKT_HIP(hipMemcpyAsync(x[i], eng.x_of(sl), sizeof(double) * eng.size_of(sl), hipMemcpyDeviceToDevice, s));
      const kkt_stats_t &st = eng.stats(sl);
      if (stats) stats[i] = st;
      if (st.status < 0) worst = st.status;
      else if (worst == STKKT_OK) worst = st.status;
      eng.release(sl);   // synchronises the stream first
      --left;
    }
  }
  STKKT_HIP(hipStreamSynchronize(s));
  return worst;
}

}  // namespace stkkt
