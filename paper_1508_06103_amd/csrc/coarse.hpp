// Two-level space-time preconditioner: coarse operator and transfers.
#pragma once

#include <memory>

#include "common.hpp"

struct coarse;
struct ras;

namespace stkkt {

struct PinnedHost {
  double *p = nullptr;
  explicit PinnedHost(size_t n);
  ~PinnedHost();
  PinnedHost(const PinnedHost &) = delete;
  PinnedHost &operator=(const PinnedHost &) = delete;
};

// Device workspace of one GMRES/FGMRES run: the Krylov basis V (m+1 vectors),
// the preconditioned basis Z (FGMRES, m vectors), five work vectors, two more
// for the two-level combination, reduction partials and the Hessenberg
// column; plus a pinned host mirror of the column.
struct GmresWork {
  long long n;
  int m;
  bool flex, coarse;
  int G, hlen;
  DevBuf V, Z, rb, wb, tb, ub, yb, t2, partial, hdev;
  PinnedHost hh;
  GmresWork(const Allocator *al, long long n, int m, bool flex, bool two_level);
  bool fits(long long n, int m, bool flex, bool two_level) const;
};

int gmres_solve_batch(int count, const kkt_op *const *ops, const ras *const *R, const solve_params_t &sp,
                      const double *const *b, double *const *x, hipStream_t s, kkt_stats_t *stats);
struct kkt_server *server_create(const server_params_t *p, const kkt_alloc_t *al, hipStream_t s);
int64_t server_submit(struct kkt_server *srv, const kkt_op *op, const ras *R, const coarse *C, const double *data,
                      double *x_out);
void server_step(struct kkt_server *srv, int32_t *n_running, int32_t *n_pending);
int server_poll(struct kkt_server *srv, int64_t ticket, kkt_stats_t *st);
void server_free(struct kkt_server *srv);
void coarse_apply_device(const coarse *C, const double *x, double *y, hipStream_t s);
// y[i] = coarse_apply(x[i]) for i < q (host arrays of device pointers); with
// the exact coarse solve the q coarse right-hand sides share one pass over
// the dense blocks.  Calls on one handle must be ordered on one stream.
void coarse_apply_multi_device(const coarse *C, int q, const double *const *x, double *const *y, hipStream_t s);
// the same for x_i = x + i ldx, y_i = y + i ldy (checked: strides, overlap)
void coarse_apply_strided(const coarse *C, int q, const double *x, long long ldx, double *y, long long ldy,
                          hipStream_t s);
coarse *coarse_create(const kkt_op *fine, const coarse_params_t *cp, hipStream_t s);
void coarse_free(coarse *c);
bool coarse_built_for(const coarse *c, const kkt_op *op);
ras *ras_create(const kkt_op *op, const ras_params_t *rp, hipStream_t s);
int gmres_solve(const kkt_op *op, const ras *R, const coarse *C, const solve_params_t &sp, const double *b,
                double *x, hipStream_t s, kkt_stats_t *st, GmresWork *work = nullptr);
}  // namespace stkkt
