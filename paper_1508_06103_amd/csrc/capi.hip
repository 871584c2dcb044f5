// C ABI entry points (include/stkkt.h): argument checks, error capture and
// the operator handle.  No exception crosses this boundary.
#include <cmath>
#include <memory>
#include <set>

#include "coarse.hpp"
#include "ras.hpp"
#include "stencil.hpp"

namespace stkkt {

void ras_export(const ras *R, int sub, double *out);
int64_t ras_sub_blocks(const ras *R, int sub);
void ras_export_csr(const ras *R, int sub, int32_t *indptr, int32_t *indices, double *blocks);

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string &msg) { g_last_error = msg; }

void *Allocator::alloc(size_t bytes) const {
  if (bytes == 0) return nullptr;
  if (cb.alloc) {
    void *p = cb.alloc(bytes, cb.ctx);
    if (!p) throw Error(STKKT_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
  }
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(STKKT_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}

void Allocator::free(void *p) const {
  if (!p) return;
  if (cb.free) cb.free(p, cb.ctx);
  else (void)hipFree(p);
}

template <class F> static int guarded(F &&f) {
  try {
    return f();
  } catch (const Error &e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc &) {
    set_last_error("host allocation failed");
    return STKKT_ENOMEM;
  } catch (const std::exception &e) {
    set_last_error(e.what());
    return STKKT_EINVAL;
  } catch (...) {
    set_last_error("unknown error");
    return STKKT_EINVAL;
  }
}

kkt_op *op_create(const kkt_problem_t *p, const kkt_alloc_t *al, hipStream_t s) {
  STKKT_REQUIRE(p != nullptr, "kkt_assemble: problem is NULL");
  for (int d = 0; d < 3; ++d) {
    STKKT_REQUIRE(p->n[d] >= 1 && p->n[d] < 65535, "kkt_assemble: n[d] must be in [1, 65534]");
    STKKT_REQUIRE(p->len[d] > 0 && std::isfinite(p->len[d]), "kkt_assemble: len must be positive");
    STKKT_REQUIRE(std::isfinite(p->v[d]), "kkt_assemble: velocity must be finite");
  }
  STKKT_REQUIRE(p->nt >= 1, "kkt_assemble: nt must be >= 1");
  STKKT_REQUIRE(p->T > 0 && std::isfinite(p->T), "kkt_assemble: T must be positive");
  STKKT_REQUIRE(p->beta1 > 0 && p->beta2 > 0 && std::isfinite(p->beta1) && std::isfinite(p->beta2),
                "kkt_assemble: beta1, beta2 must be positive");
  STKKT_REQUIRE(p->variant == STKKT_DTO || p->variant == STKKT_OTD, "kkt_assemble: unknown variant");
  STKKT_REQUIRE(p->regularization == STKKT_REG_H1H1 || p->regularization == STKKT_REG_H1L2,
                "kkt_assemble: unknown regularization");
  STKKT_REQUIRE(p->a_elem != nullptr, "kkt_assemble: a_elem is NULL");
  STKKT_REQUIRE(p->n_sensors >= 1 && p->sensor_node != nullptr && p->data != nullptr,
                "kkt_assemble: at least one sensor with data is required");
  STKKT_REQUIRE((p->dirichlet_faces & ~63u) == 0, "kkt_assemble: bad Dirichlet face mask");
  auto op = std::make_unique<kkt_op>();
  if (al) op->al.cb = *al;
  OpDev &d = op->d;
  for (int k = 0; k < 3; ++k) {
    d.n[k] = p->n[k];
    d.nn[k] = p->n[k] + 1;
    d.h[k] = p->len[k] / p->n[k];
    d.v[k] = p->v[k];
    op->len[k] = p->len[k];
  }
  d.M = p->nt;
  d.N = d.nn[0] * d.nn[1] * d.nn[2];
  STKKT_REQUIRE((long long)d.nn[0] * d.nn[1] * d.nn[2] < (1LL << 31), "kkt_assemble: mesh too large");
  d.V = (long long)d.N * (d.M + 1);
  d.tau = p->T / p->nt;
  d.beta1 = p->beta1;
  d.beta2 = p->beta2;
  d.faces = p->dirichlet_faces;
  d.variant = p->variant;
  d.reg = p->regularization;
  op->T = p->T;
  const long long ne = (long long)p->n[0] * p->n[1] * p->n[2];
  op->a_host.assign(p->a_elem, p->a_elem + ne);
  for (double a : op->a_host) STKKT_REQUIRE(a > 0 && std::isfinite(a), "kkt_assemble: a_elem must be positive");
  std::vector<double> sens(d.N, 0.0);
  std::set<int32_t> seen;
  for (int s_ = 0; s_ < p->n_sensors; ++s_) {
    const int32_t j = p->sensor_node[s_];
    STKKT_REQUIRE(j >= 0 && j < d.N, "kkt_assemble: sensor node out of range");
    STKKT_REQUIRE(seen.insert(j).second, "kkt_assemble: duplicate sensor node");
    const int jx = j % d.nn[0], jy = (j / d.nn[0]) % d.nn[1], jz = j / (d.nn[0] * d.nn[1]);
    STKKT_REQUIRE(!on_dirichlet(d, jx, jy, jz), "kkt_assemble: sensor on a Dirichlet face");
    sens[j] = 1.0;
    op->sensor_node.push_back(j);
  }
  for (long long k = 0; k < (long long)(p->nt + 1) * p->n_sensors; ++k)
    STKKT_REQUIRE(std::isfinite(p->data[k]), "kkt_assemble: non-finite sensor data");
  op->a_elem = DevBuf(&op->al, sizeof(double) * ne);
  op->sensor = DevBuf(&op->al, sizeof(double) * d.N);
  op->atab = DevBuf(&op->al, sizeof(double) * 27 * (size_t)d.N);
  STKKT_HIP(hipMemcpyAsync(op->a_elem.ptr, op->a_host.data(), sizeof(double) * ne, hipMemcpyHostToDevice, s));
  STKKT_HIP(hipMemcpyAsync(op->sensor.ptr, sens.data(), sizeof(double) * d.N, hipMemcpyHostToDevice, s));
  d.a_elem = op->a_elem.as<double>();
  d.sensor = op->sensor.as<double>();
  stiff_table(d, op->atab.as<double>(), s);
  op->mv = choose_matvec_tile(d);
  STKKT_HIP(hipStreamSynchronize(s));
  return op.release();
}

}  // namespace stkkt

using namespace stkkt;

extern "C" {

int kkt_assemble(const kkt_problem_t *p, const kkt_alloc_t *al, void *stream, kkt_op_t **op, double *b) {
  return guarded([&] {
    STKKT_REQUIRE(op != nullptr, "kkt_assemble: op is NULL");
    *op = nullptr;
    std::unique_ptr<kkt_op> h(op_create(p, al, as_stream(stream)));
    if (b) rhs_device(h.get(), p->data, as_stream(stream), b);
    *op = h.release();
    return STKKT_OK;
  });
}

int kkt_rhs(const kkt_op_t *op, const double *data_host, void *stream, double *b) {
  return guarded([&] {
    STKKT_REQUIRE(op && data_host && b, "kkt_rhs: NULL argument");
    for (long long k = 0; k < (long long)(op->d.M + 1) * (long long)op->sensor_node.size(); ++k)
      STKKT_REQUIRE(std::isfinite(data_host[k]), "kkt_rhs: non-finite sensor data");
    rhs_device(op, data_host, as_stream(stream), b);
    return STKKT_OK;
  });
}

int kkt_rhs_noalloc(const kkt_op_t *op, const double *data_host, void *stream, double *b) {
  return guarded([&] {
    STKKT_REQUIRE(op && data_host && b, "kkt_rhs_noalloc: NULL argument");
    for (long long k = 0; k < (long long)(op->d.M + 1) * (long long)op->sensor_node.size(); ++k)
      STKKT_REQUIRE(std::isfinite(data_host[k]), "kkt_rhs_noalloc: non-finite sensor data");
    rhs_device_noalloc(op, data_host, as_stream(stream), b);
    return STKKT_OK;
  });
}

int kkt_matvec(const kkt_op_t *op, const double *x, double *y, void *stream) {
  return guarded([&] {
    STKKT_REQUIRE(op && x && y, "kkt_matvec: NULL argument");
    STKKT_REQUIRE(x != y, "kkt_matvec: x and y must not alias");
    matvec_device(op, x, y, as_stream(stream));
    return STKKT_OK;
  });
}

int64_t kkt_size(const kkt_op_t *op) { return op ? 3 * op->d.V : -1; }

int ras_setup(const kkt_op_t *op, const ras_params_t *rp, void *stream, ras_t **out) {
  return guarded([&] {
    STKKT_REQUIRE(op && out, "ras_setup: NULL argument");
    *out = nullptr;
    *out = ras_create(op, rp, as_stream(stream));
    return STKKT_OK;
  });
}

int ras_apply(const ras_t *R, const double *r, double *z, void *stream) {
  return guarded([&] {
    STKKT_REQUIRE(R && r && z, "ras_apply: NULL argument");
    STKKT_REQUIRE(r != z, "ras_apply: r and z must not alias");
    ras_apply_device(R, r, z, as_stream(stream));
    return STKKT_OK;
  });
}

int ras_num_subdomains(const ras_t *R) { return R ? R->nsub : -1; }

int ras_query_boxes(const ras_t *R, int32_t *host_out) {
  return guarded([&] {
    STKKT_REQUIRE(R && host_out, "ras_query_boxes: NULL argument");
    std::copy(R->boxes.begin(), R->boxes.end(), host_out);
    return STKKT_OK;
  });
}

int64_t ras_factor_bytes(const ras_t *R) {
  if (!R) return -1;
  return R->total_blocks * 9 * (R->params.precision == STKKT_F32 ? 4 : 8);
}

int32_t ras_query_apply_rows(const ras_t *R) { return R ? stkkt::ras_apply_rows_per_phase(R) : -1; }

int ras_export_factors(const ras_t *R, int32_t sub, double *host_out) {
  return guarded([&] {
    STKKT_REQUIRE(R && host_out, "ras_export_factors: NULL argument");
    ras_export(R, sub, host_out);
    return STKKT_OK;
  });
}

int64_t ras_subdomain_blocks(const ras_t *R, int32_t sub) {
  if (!R || sub < 0 || sub >= R->nsub) return -1;
  return ras_sub_blocks(R, sub);
}

int ras_export_factors_csr(const ras_t *R, int32_t sub, int32_t *indptr, int32_t *indices, double *blocks) {
  return guarded([&] {
    STKKT_REQUIRE(R && indptr && indices && blocks, "ras_export_factors_csr: NULL argument");
    ras_export_csr(R, sub, indptr, indices, blocks);
    return STKKT_OK;
  });
}

int coarse_setup(const kkt_op_t *fine, const coarse_params_t *cp, void *stream, coarse_t **out) {
  return guarded([&] {
    STKKT_REQUIRE(fine && cp && out, "coarse_setup: NULL argument");
    *out = nullptr;
    *out = coarse_create(fine, cp, as_stream(stream));
    return STKKT_OK;
  });
}

int coarse_apply(const coarse_t *c, const double *x, double *y, void *stream) {
  return guarded([&] {
    STKKT_REQUIRE(c && x && y, "coarse_apply: NULL argument");
    STKKT_REQUIRE(x != y, "coarse_apply: x and y must not alias");
    coarse_apply_device(c, x, y, as_stream(stream));
    return STKKT_OK;
  });
}

int coarse_apply_multi(const coarse_t *c, int32_t q, const double *x, int64_t ldx, double *y, int64_t ldy,
                       void *stream) {
  return guarded([&] {
    STKKT_REQUIRE(c && (q == 0 || (x && y)), "coarse_apply_multi: NULL argument");
    coarse_apply_strided(c, q, x, ldx, y, ldy, as_stream(stream));
    return STKKT_OK;
  });
}

int kkt_solve(const kkt_op_t *op, const ras_t *R, const coarse_t *C, const solve_params_t *sp, const double *b,
              double *x, void *stream, kkt_stats_t *stats) {
  return guarded([&] {
    STKKT_REQUIRE(op && R && sp && b && x, "kkt_solve: NULL argument");
    STKKT_REQUIRE(R->op == op, "kkt_solve: preconditioner built for another operator");
    STKKT_REQUIRE(!C || coarse_built_for(C, op), "kkt_solve: coarse level built for another operator");
    STKKT_REQUIRE(sp->restart >= 1 && sp->restart <= 1000, "kkt_solve: restart must be in [1, 1000]");
    STKKT_REQUIRE(sp->maxit >= 1 || sp->fixed_iters > 0, "kkt_solve: maxit must be >= 1");
    STKKT_REQUIRE(sp->rtol > 0 && sp->rtol < 1, "kkt_solve: rtol must be in (0, 1)");
    STKKT_REQUIRE(sp->fixed_iters >= 0, "kkt_solve: fixed_iters must be >= 0");
    STKKT_REQUIRE(b != x, "kkt_solve: b and x must not alias");
    return gmres_solve(op, R, C, *sp, b, x, as_stream(stream), stats);
  });
}

int kkt_solve_batch(int32_t count, const kkt_op_t *const *ops, const ras_t *const *ras, const solve_params_t *sp,
                    const double *const *b, double *const *x, void *stream, kkt_stats_t *stats) {
  return guarded([&] {
    STKKT_REQUIRE(count >= 1 && ops && ras && sp && b && x, "kkt_solve_batch: NULL argument or empty batch");
    STKKT_REQUIRE(sp->restart >= 1 && sp->restart <= 1000, "kkt_solve_batch: restart must be in [1, 1000]");
    STKKT_REQUIRE(sp->maxit >= 1 || sp->fixed_iters > 0, "kkt_solve_batch: maxit must be >= 1");
    STKKT_REQUIRE(sp->rtol > 0 && sp->rtol < 1, "kkt_solve_batch: rtol must be in (0, 1)");
    STKKT_REQUIRE(sp->fixed_iters >= 0, "kkt_solve_batch: fixed_iters must be >= 0");
    std::set<const kkt_op *> seen;
    for (int i = 0; i < count; ++i) {
      STKKT_REQUIRE(ops[i] && ras[i] && b[i] && x[i], "kkt_solve_batch: NULL entry");
      STKKT_REQUIRE(ras[i]->op == ops[i], "kkt_solve_batch: preconditioner built for another operator");
      STKKT_REQUIRE(b[i] != x[i], "kkt_solve_batch: b and x must not alias");
    }
    return gmres_solve_batch(count, ops, ras, *sp, b, x, as_stream(stream), stats);
  });
}

int kkt_server_create(const server_params_t *p, const kkt_alloc_t *al, void *stream, kkt_server_t **out) {
  return guarded([&] {
    STKKT_REQUIRE(out != nullptr, "kkt_server_create: out is NULL");
    *out = nullptr;
    *out = server_create(p, al, as_stream(stream));
    return STKKT_OK;
  });
}

int kkt_server_submit(kkt_server_t *srv, const kkt_op_t *op, const ras_t *ras, const coarse_t *coarse,
                      const double *data_host, double *x_out, int64_t *ticket) {
  return guarded([&] {
    STKKT_REQUIRE(srv && ticket, "kkt_server_submit: NULL argument");
    *ticket = server_submit(srv, op, ras, coarse, data_host, x_out);
    return STKKT_OK;
  });
}

int kkt_server_step(kkt_server_t *srv, int32_t *n_running, int32_t *n_pending) {
  return guarded([&] {
    STKKT_REQUIRE(srv != nullptr, "kkt_server_step: NULL server");
    server_step(srv, n_running, n_pending);
    return STKKT_OK;
  });
}

int kkt_server_poll(kkt_server_t *srv, int64_t ticket, kkt_stats_t *stats) {
  return guarded([&] {
    STKKT_REQUIRE(srv != nullptr, "kkt_server_poll: NULL server");
    return server_poll(srv, ticket, stats);
  });
}

void kkt_server_destroy(kkt_server_t *srv) { server_free(srv); }

void kkt_op_destroy(kkt_op_t *op) { delete op; }
void ras_destroy(ras_t *R) { delete R; }
void coarse_destroy(coarse_t *c) { coarse_free(c); }

const char *kkt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
