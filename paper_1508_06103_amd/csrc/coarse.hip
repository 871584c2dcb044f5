// Two-level space-time preconditioner (placeholder until the coarse block LU lands).
#include "coarse.hpp"

struct coarse {
  int dummy = 0;
};

namespace stkkt {

void coarse_apply_device(const coarse *, const double *, double *, hipStream_t) {
  throw Error(STKKT_EINVAL, "coarse level not available");
}

coarse *coarse_create(const kkt_op *, const coarse_params_t *, hipStream_t) {
  throw Error(STKKT_EINVAL, "coarse level not available");
}

void coarse_free(coarse *c) { delete c; }

}  // namespace stkkt
