// Request server: source-identification requests (an operator with its
// preconditioner, plus new sensor data) are admitted into the batch engine
// as slots and device memory allow, advanced together one FGMRES cycle per
// step, and retired as they finish, so requests that arrive while others
// are on the GPU join them at the next cycle (continuous batching).  F_h
// does not depend on the data, so a request only forms its right-hand side;
// operators and factors stay on the device across requests (the caller
// keeps the handles).
#include <chrono>
#include <deque>
#include <map>
#include <memory>

#include "batch.hpp"

using stkkt::Allocator;
using stkkt::BatchEngine;
using stkkt::Error;

struct kkt_server {
  Allocator al;
  solve_params_t sp{};
  hipStream_t s = nullptr;
  std::unique_ptr<BatchEngine> eng;
  size_t member_budget = 0, member_used = 0;
  struct Req {
    int64_t ticket = 0;
    const kkt_op *op = nullptr;
    const ras *R = nullptr;
    const coarse *C = nullptr;
    std::vector<double> data;
    double *x_out = nullptr;
    size_t bytes = 0;
    std::chrono::steady_clock::time_point t_submit, t_admit;
  };
  std::deque<Req> pending;
  std::map<int, Req> running;   // by engine slot
  std::map<int64_t, kkt_stats_t> done;
  std::map<int64_t, int> state;   // 0 pending, 1 running, 2 done
  int64_t next_ticket = 1;
};

namespace stkkt {

kkt_server *server_create(const server_params_t *p, const kkt_alloc_t *al, hipStream_t s) {
  STKKT_REQUIRE(p != nullptr, "kkt_server_create: params is NULL");
  STKKT_REQUIRE(p->restart >= 1 && p->restart <= 1000, "kkt_server_create: restart must be in [1, 1000]");
  STKKT_REQUIRE(p->maxit >= 1, "kkt_server_create: maxit must be >= 1");
  STKKT_REQUIRE(p->rtol > 0 && p->rtol < 1, "kkt_server_create: rtol must be in (0, 1)");
  STKKT_REQUIRE(p->max_active >= 1, "kkt_server_create: max_active must be >= 1");
  STKKT_REQUIRE(p->device_bytes > 0, "kkt_server_create: device_bytes must be positive");
  auto srv = std::make_unique<kkt_server>();
  if (al) srv->al.cb = *al;
  srv->sp.restart = p->restart;
  srv->sp.maxit = p->maxit;
  srv->sp.rtol = p->rtol;
  srv->sp.flexible = 1;
  srv->sp.graph = 1;
  srv->s = s;
  // half of the budget for the concatenated Krylov vectors (2m + 6 of them),
  // half for the members' own buffers (RAS local vectors, two-level temporaries)
  const double vec_bytes = 0.5 * (double)p->device_bytes;
  const long long cap = (long long)(vec_bytes / (8.0 * (2.0 * p->restart + 6.0)));
  STKKT_REQUIRE(cap >= 256, "kkt_server_create: device_bytes too small");
  srv->member_budget = (size_t)(0.5 * (double)p->device_bytes);
  srv->eng = std::make_unique<BatchEngine>(&srv->al, srv->sp, cap, p->max_active, s);
  return srv.release();
}

int64_t server_submit(kkt_server *srv, const kkt_op *op, const ras *R, const coarse *C, const double *data,
                      double *x_out) {
  STKKT_REQUIRE(op && R && data && x_out, "kkt_server_submit: NULL argument");
  STKKT_REQUIRE(R->op == op, "kkt_server_submit: preconditioner built for another operator");
  STKKT_REQUIRE(!C || coarse_built_for(C, op), "kkt_server_submit: coarse level built for another operator");
  const long long n = 3 * op->d.V;
  STKKT_REQUIRE((n + 255) / 256 * 256 <= srv->eng->capacity(), "kkt_server_submit: request larger than the server");
  const size_t bytes = BatchEngine::member_bytes(op, R, C);
  STKKT_REQUIRE(bytes <= srv->member_budget, "kkt_server_submit: request larger than the server");
  const size_t nd = (size_t)(op->d.M + 1) * op->sensor_node.size();
  for (size_t k = 0; k < nd; ++k) STKKT_REQUIRE(std::isfinite(data[k]), "kkt_server_submit: non-finite sensor data");
  kkt_server::Req q;
  q.ticket = srv->next_ticket++;
  q.op = op;
  q.R = R;
  q.C = C;
  q.data.assign(data, data + nd);
  q.x_out = x_out;
  q.bytes = bytes;
  q.t_submit = std::chrono::steady_clock::now();
  srv->state[q.ticket] = 0;
  srv->pending.push_back(std::move(q));
  return srv->pending.back().ticket;
}

void server_step(kkt_server *srv, int32_t *n_running, int32_t *n_pending) {
  BatchEngine &e = *srv->eng;
  // admission, first come first served: stop at the first request that does not fit
  while (!srv->pending.empty()) {
    kkt_server::Req &q = srv->pending.front();
    if (srv->member_used + q.bytes > srv->member_budget) break;
    const int slot = e.admit(q.op, q.R, q.C);
    if (slot < 0) break;
    try {
      rhs_device(q.op, q.data.data(), srv->s, e.b_of(slot));
      fill_zero(e.x_of(slot), e.size_of(slot), srv->s);
    } catch (...) {
      e.release(slot);   // the request stays queued; the slot is free again
      throw;
    }
    q.t_admit = std::chrono::steady_clock::now();
    srv->member_used += q.bytes;
    srv->state[q.ticket] = 1;
    srv->running[slot] = std::move(q);
    srv->pending.pop_front();
  }
  std::vector<int> fin;
  if (e.active() > 0) e.cycle(fin);
  const auto now = std::chrono::steady_clock::now();
  for (int slot : fin) {
    kkt_server::Req &q = srv->running.at(slot);
    STKKT_HIP(hipMemcpyAsync(q.x_out, e.x_of(slot), sizeof(double) * e.size_of(slot), hipMemcpyDeviceToDevice,
                             srv->s));
    kkt_stats_t st = e.stats(slot);
    st.t_ms[0] = std::chrono::duration<double, std::milli>(now - q.t_submit).count();
    st.t_ms[1] = std::chrono::duration<double, std::milli>(q.t_admit - q.t_submit).count();
    e.release(slot);   // synchronises the stream: the copy above is complete
    srv->member_used -= q.bytes;
    srv->done[q.ticket] = st;
    srv->state[q.ticket] = 2;
    srv->running.erase(slot);
  }
  if (n_running) *n_running = (int32_t)srv->running.size();
  if (n_pending) *n_pending = (int32_t)srv->pending.size();
}

int server_poll(kkt_server *srv, int64_t ticket, kkt_stats_t *st) {
  auto it = srv->state.find(ticket);
  STKKT_REQUIRE(it != srv->state.end(), "kkt_server_poll: unknown ticket");
  if (it->second != 2) return 0;
  if (st) *st = srv->done[ticket];
  srv->done.erase(ticket);
  srv->state.erase(it);
  return 1;
}

void server_free(kkt_server *srv) { delete srv; }

}  // namespace stkkt
