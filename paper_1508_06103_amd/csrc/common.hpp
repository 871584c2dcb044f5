// Internal helpers shared by the library's translation units: error state,
// HIP checks, device memory through the caller's allocator, and the POD
// operator descriptor handed to kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/stkkt.h"

namespace stkkt {

// Error carried from the library internals to the C ABI wrappers.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);

#define STKKT_HIP(call)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      throw ::stkkt::Error(STKKT_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define STKKT_REQUIRE(cond, msg)                                                              \
  do {                                                                                        \
    if (!(cond)) throw ::stkkt::Error(STKKT_EINVAL, msg);                                     \
  } while (0)

// Allocation through the caller's callbacks (or hipMalloc).
struct Allocator {
  kkt_alloc_t cb{nullptr, nullptr, nullptr};
  void *alloc(size_t bytes) const;
  void free(void *p) const;
};

// Owning device buffer.
struct DevBuf {
  const Allocator *al = nullptr;
  void *ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const Allocator *a, size_t n) : al(a), bytes(n) { ptr = n ? a->alloc(n) : nullptr; }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : al(o.al), ptr(o.ptr), bytes(o.bytes) { o.ptr = nullptr; o.bytes = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) { reset(); al = o.al; ptr = o.ptr; bytes = o.bytes; o.ptr = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { reset(); }
  void reset() {
    if (ptr && al) al->free(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Operator descriptor passed by value to kernels.
struct OpDev {
  int n[3];        // elements per axis
  int nn[3];       // nodes per axis
  int M;           // time steps
  int N;           // spatial nodes
  long long V;     // space-time nodes N (M+1)
  double h[3];
  double tau;
  double v[3];
  double beta1, beta2;
  unsigned faces;  // Dirichlet face bitmask
  int variant;
  int reg;         // STKKT_REG_H1H1 or STKKT_REG_H1L2
  const double *a_elem;   // device [n2][n1][n0]
  const double *sensor;   // device [N], 1 at sensor nodes
};

// Launch shape of the matvec: spatial tiles of t[0] x t[1] x t[2] nodes
// (nt[] tiles per axis) marched over time chunks of clen levels.
struct MvTile {
  int t[3], nt[3];
  int ntiles, halo, clen, nchunks;
};

}  // namespace stkkt

struct kkt_op {
  stkkt::Allocator al;
  stkkt::OpDev d{};
  stkkt::MvTile mv{};
  stkkt::DevBuf a_elem, sensor, atab;   // atab: [N][27] diffusion stiffness rows
  std::vector<int32_t> sensor_node;   // host copy
  double T = 1.0, len[3] = {1, 1, 1};
  std::vector<double> a_host;         // host copy of a_elem (coarse setup)
};

namespace stkkt {
inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }
inline int blocks_for(long long n, int threads, int cap = 1 << 20) {
  long long b = (n + threads - 1) / threads;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return static_cast<int>(b);
}
// Read-only tables indexed by wave-uniform values are read through the
// constant address space, which lets the compiler use scalar loads (waited on
// with lgkmcnt) instead of vector loads that would drain the in-order vmcnt
// counter and with it every prefetch in flight.
template <class V> using cptr = const __attribute__((address_space(4))) V *;
template <class V> __device__ inline cptr<V> as_const(const V *p) { return (cptr<V>)p; }

// Copy a table entry (a struct of 32-bit words) through scalar loads.
template <class S> __device__ inline S load_uniform(const S *p) {
  static_assert(sizeof(S) % 4 == 0, "word-sized struct expected");
  S out;
  cptr<int32_t> src = (cptr<int32_t>)p;
  int32_t *dst = reinterpret_cast<int32_t *>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(S) / 4); ++i) dst[i] = src[i];
  return out;
}

kkt_op *op_create(const kkt_problem_t *p, const kkt_alloc_t *al, hipStream_t s);
void rhs_device(const kkt_op *op, const double *data_host, hipStream_t s, double *b);
// The same without allocation: staging in a static device array of
// kRhsScratchBytes (EINVAL when the data need more, see rhs_scratch_need).
constexpr size_t kRhsScratchBytes = STKKT_RHS_SCRATCH_BYTES;
size_t rhs_scratch_need(const kkt_op *op);
void rhs_device_noalloc(const kkt_op *op, const double *data_host, hipStream_t s, double *b);
void fill_zero(double *p, long long n, hipStream_t s);
void stiff_table(const OpDev &d, double *tab, hipStream_t s);
MvTile choose_matvec_tile(const OpDev &d);
void matvec_device(const kkt_op *op, const double *x, double *y, hipStream_t s);
// Batched matvec over operators whose vectors are concatenated: operator i
// reads x[voff_i ...] and writes y[voff_i ...]; one launch for all of them,
// operators with act[i] == 0 (device flags) skipped.
struct MvBatch {
  DevBuf desc;
  int count = 0;
  long long items = 0;
  int kh = 1;
  size_t lds = 0;
};
void matvec_batch_prepare(const kkt_op *const *ops, const long long *voff, int count, const Allocator *al,
                          MvBatch &out, hipStream_t s);
void matvec_batch_run(const MvBatch &b, const double *x, double *y, const int *act, hipStream_t s);
}  // namespace stkkt
