// Two-level space-time preconditioner: coarse operator and transfers.
#pragma once

#include "common.hpp"

struct coarse;

namespace stkkt {
void coarse_apply_device(const coarse *C, const double *x, double *y, hipStream_t s);
coarse *coarse_create(const kkt_op *fine, const coarse_params_t *cp, hipStream_t s);
void coarse_free(coarse *c);
}  // namespace stkkt
