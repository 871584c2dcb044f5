// Space-time RAS with ILU(k), k >= 1, subdomain solves (Section 4: ILU(k)
// with a fill level k; the paper's first table varies k): data structures.
//
// The level-k pattern of a box follows the usual symbolic rule on the
// 81-point block pattern (entries of the stencil have level 0; eliminating
// row k from row i offers entry (i, j) the level lev(i,k) + lev(k,j) + 1;
// entries of level <= k are kept).  Fill reaches node offsets beyond +-1, so
// the closed-form wavefront levels of ILU(0) no longer order the rows: here
// every row gets the dependency level 1 + max(level of the columns left of
// its diagonal), rows are stored level by level in 64-row chunks, and each
// chunk keeps its entries in an ELL layout (entry e of the chunk's row q at
// [e][9 entries of the block][64 rows]), so that a wavefront reads one entry
// of 64 rows with one coalesced load per block element.
#pragma once

#include <memory>

#include "common.hpp"

namespace stkkt {

// One 64-row chunk of a level: rows at level-order positions pos0 .. pos0+rows-1,
// lmax / umax entries left / right of the diagonal (padded to the chunk's
// longest row), factor values at element foff of the subdomain's block,
// column positions at coff of the shape's table.
struct IlukChunk {
  int32_t pos0, rows, lmax, umax;
  int64_t foff, coff;
};

struct IlukShapeDev {
  int32_t dims[4];
  int32_t nrows, nlev, nchunk, pad_;
  int64_t chunk_off;   // into the chunk table
  int64_t lvl_off;     // into the per-level first-chunk table (nlev + 1 entries)
  int64_t pos_off;     // into the per-position tables (coords, rho, nL, nU, pchunk)
  int64_t col_off;     // into the column table
};

struct IlukShapeHost {
  int dims[4] = {0, 0, 0, 0};
  int nrows = 0, nlev = 0;
  std::vector<int32_t> lvl_chunk;   // first chunk of every level, nlev + 1 entries
  std::vector<uint64_t> coords;     // packed x | y << 16 | z << 32 | t << 48 per position
  std::vector<int32_t> rho;         // natural index x + lx (y + ly (z + lz t)) per position
  std::vector<int32_t> pchunk;      // chunk of every position
  std::vector<int16_t> nL, nU;      // entries left / right of the diagonal per position
  std::vector<IlukChunk> chunks;
  std::vector<int32_t> cols;        // level-order positions of the entries (nrows for padding)
  int64_t felems = 0;               // factor elements of one subdomain (padded layout)
  int64_t nblocks = 0;              // 3x3 blocks of the pattern
  std::vector<int32_t> indptr, indices;   // the pattern as block CSR in natural order
};

struct IlukData {
  int level = 0;
  std::vector<IlukShapeHost> shapes;   // same order as the ILU(0) shape list of the handle
  int64_t factor_elems = 0, scratch_elems = 0, total_blocks = 0;
  DevBuf d_shapes, d_chunks, d_lvl, d_coords, d_rho, d_pchunk, d_nL, d_nU, d_cols;
  DevBuf factors;   // double or float, ELL layout per chunk
  DevBuf scratch;   // local vectors: (rows + 1) x 3 per subdomain
};

}  // namespace stkkt

struct ras;
struct kkt_op;

namespace stkkt {
// Build the ILU(k) factors of every subdomain of R (boxes, subdomain table
// and shape list already filled in by ras_create; fbase / sbase are
// rewritten for the ELL layout).
void iluk_create(ras *R, const kkt_op *op, hipStream_t s);
void iluk_apply(const ras *R, const double *r, double *z, void *local, hipStream_t s);
size_t iluk_local_bytes(const ras *R);
int64_t iluk_subdomain_blocks(const ras *R, int sub);
// natural-order block CSR: indptr[rows + 1], indices[blocks], blocks[9 x blocks]
// (L left of the diagonal, inv(U_ii) on it, U right of it)
void iluk_export_csr(const ras *R, int sub, int32_t *indptr, int32_t *indices, double *blocks);
}  // namespace stkkt
