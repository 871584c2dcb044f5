// One-level space-time restricted additive Schwarz: data structures.
#pragma once

#include <memory>

#include "common.hpp"

namespace stkkt {

struct IlukData;

// Per subdomain (device table).
struct SubInfo {
  int32_t shape;
  int32_t org[4];        // box_lo in (x, y, z, t)
  int32_t olo[4], ohi[4];  // owned range in local coordinates [olo, ohi)
  int32_t pad_;
  int64_t fbase;         // element offset of this subdomain's factors
  int64_t sbase;         // element offset of its local vector (3 per row)
  int64_t wbase;         // element offset in the setup working buffer
};

// Per distinct box shape (device table).  Rows of a level are in ascending
// local lexicographic order rho = x + lx (y + ly (z + lz t)); the level of a
// node is x + 2y + 4z + 8t (every lower neighbour of the 81-point stencil has
// a strictly smaller level).
struct ShapeInfo {
  int32_t dims[4];
  int32_t nlev, nchunk, rmax, vol;
  int64_t lvl_off;     // into lvl_start (nlev + 1 entries, row offsets)
  int64_t coord_off;   // into coords (vol entries, packed 16-bit x|y|z|t)
  int64_t ct_off;      // into the chunk table (nlev*nchunk*81 (off9, cnt) pairs)
  int64_t tz_off;      // into tzpref (nlev*lt*lz entries)
};

struct ShapeHost {
  int dims[4];
  int nlev = 0, nchunk = 0, rmax = 0, vol = 0;
  std::vector<int32_t> lvl_start;
  std::vector<uint64_t> coords;
  std::vector<int32_t> ctab;   // (element offset, block count) per (level, chunk, slot)
  int64_t nblocks = 0;         // 3x3 blocks
  int64_t felems = 0;          // factor elements including group padding
  std::vector<int32_t> tzpref;
};

}  // namespace stkkt

struct ras {
  const kkt_op *op = nullptr;   // identity only; never dereferenced after setup
  stkkt::Allocator al;          // own copy: the handle may outlive its operator
  stkkt::OpDev d{};             // sizes of the operator (device pointers unused)
  ras_params_t params{};
  int nsub = 0;
  std::vector<stkkt::SubInfo> subs;
  std::vector<int> shape_of;
  std::vector<stkkt::ShapeHost> shapes;
  std::vector<int32_t> boxes;   // nsub x 16
  int64_t total_blocks = 0;    // 3x3 factor blocks of all subdomains
  int64_t factor_elems = 0;    // factor elements including group padding (zero block follows)
  int64_t scratch_elems = 0;
  int ring_rmax = 0, ring_ltlz = 0;   // LDS ring sizes of the apply kernel
  stkkt::DevBuf d_subs, d_shapes, d_lvl, d_coords, d_ctab, d_order, d_tz;
  stkkt::DevBuf factors;   // double or float, grouped (blk_pos), 16 zero elements at the end
  stkkt::DevBuf scratch;   // local vectors
  std::shared_ptr<stkkt::IlukData> iluk;   // ILU(k), k > 0: factors, tables and local vectors (else null)
};

namespace stkkt {
// local: device buffer for the subdomains' local vectors (ras_local_bytes(R)
// bytes, the last bytes zero), or NULL for the handle's own.
void ras_apply_device(const ras *R, const double *r, double *z, hipStream_t s, void *local = nullptr);
bool ras_uses_ring(const ras *R);   // the 256-row ring kernel (the one batched launches share)
// rows per phase of the kernel ras_apply runs: 256 or 64 (LDS ring), 0 (local vector in global memory)
int ras_apply_rows_per_phase(const ras *R);
size_t ras_local_bytes(const ras *R);

// Batched application over preconditioners whose vectors are concatenated
// (member i reads r[voff_i ...] and writes z[voff_i ...], its local vectors in
// local[i] when given): one launch over the (member, subdomain) work list
// when every member uses the LDS-ring kernel with the same precision, else
// one launch per member.  NULL members are empty slots.
struct RasBatch {
  DevBuf desc, work;
  int count = 0, blocks = 0, precision = STKKT_F64;
  bool ring = false;     // one launch over the (member, subdomain) work list of the ring members
  int kr = 256;          // rows per phase of that launch (the largest of 256, 128, 64 every member allows)
  std::vector<int> solo; // members launched on their own (no LDS ring, or ILU(k))
  size_t lds = 0;
  std::vector<const ras *> members;
  std::vector<long long> voff;
  std::vector<void *> local;
};
void ras_batch_prepare(const ras *const *R, const long long *voff, void *const *local, int count,
                       const Allocator *al, RasBatch &out, hipStream_t s);
// true when the whole batch is one launch (no member of its own)
inline bool ras_batch_single_launch(const RasBatch &b) { return b.ring && b.solo.empty(); }
// act: device flags (members with 0 are skipped; members with 2 read their
// input from r2 instead of r, at the same offset), act_host: the same flags on
// the host
void ras_batch_run(const RasBatch &b, const double *r, double *z, const int *act, const int *act_host,
                   hipStream_t s, const double *r2 = nullptr);
}
