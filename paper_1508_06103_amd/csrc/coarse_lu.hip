// Exact coarse solve F_c^{-1} by block elimination in time (the coarse
// operator is block tridiagonal in time, Section 3.2; block k = the 3 N_c
// unknowns of coarse level k):
//   S_0 = D_0,  S_k = D_k - L_k S_{k-1}^{-1} U_{k-1},
//   forward   y_0 = S_0^{-1} r_0,  y_k = S_k^{-1} (r_k - L_k y_{k-1}),
//   backward  x_M = y_M,           x_k = y_k - E_k x_{k+1},  E_k = S_k^{-1} U_k.
// D_k, L_k, U_k are the stencil blocks of the coarse operator (its 27 spatial
// neighbours at time offsets 0, -1, +1).  The setup forms every S_k densely
// and inverts it explicitly (blocked Gauss-Jordan elimination with partial
// pivoting, the trailing updates as tiled FP64 GEMMs), so one application is
// two sweeps of dense block products streamed from HBM: matrix-vector
// products (solve) or matrix-core products for up to 16 vectors per pass
// (solve_multi).
//
// Dense matrices are stored column-major (entry (r, c) at c * nb + r during
// the setup; the kept S_k^{-1} and E_k at c * ld + r, ld = nb rounded up to
// 64).  The Gauss-Jordan kernels work on rows of the buffer, i.e. on the
// transpose; the inverse of the transpose read column-major is the inverse
// itself.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "coarse_lu.hpp"
#include "stencil.hpp"

namespace stkkt {

namespace {

constexpr int kPanel = 64;   // Gauss-Jordan panel width (= GEMM inner dimension)

// ---------------------------------------------------------------------------
// sparse couplings: for every row r = 3 j + a of a level, its 27 spatial
// neighbours i and slots b (81 entries): column index 3 i + b and the value of
// the (dt) block; neighbours outside the mesh have value 0
// ---------------------------------------------------------------------------
__global__ void coupling_rows_kernel(OpDev op, int n, int dt, int32_t *__restrict__ idx, double *__restrict__ val) {
  const int N = op.N;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
    const int jx = j % op.nn[0], jy = (j / op.nn[0]) % op.nn[1], jz = j / (op.nn[0] * op.nn[1]);
    for (int k = 0; k < 27; ++k) {
      const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
      const int ix = jx + dx, iy = jy + dy, iz = jz + dz;
      const bool in = ix >= 0 && ix < op.nn[0] && iy >= 0 && iy < op.nn[1] && iz >= 0 && iz < op.nn[2];
      double blk[9];
      if (in) kkt_block(op, jx, jy, jz, n, dx, dy, dz, dt, blk);
      const int i = in ? ix + op.nn[0] * (iy + op.nn[1] * iz) : 0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          const long long e = (long long)(3 * j + a) * 81 + 3 * k + b;
          idx[e] = 3 * i + b;
          val[e] = in ? blk[3 * a + b] : 0.0;
        }
    }
  }
}

// S = D_k (column-major), from the dt = 0 coupling rows
__global__ void dense_from_rows_kernel(int nb, const int32_t *__restrict__ idx, const double *__restrict__ val,
                                       double *__restrict__ S) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nb; r += gridDim.x * blockDim.x)
    for (int t = 0; t < 81; ++t) {
      const double v = val[(long long)r * 81 + t];
      if (v != 0.0) S[(long long)idx[(long long)r * 81 + t] * nb + r] += v;
    }
}

// S(r, c) -= sum_t L(r, idx_t) E(idx_t, c)   (column-major S, E; L rows sparse)
__global__ void schur_update_kernel(int nb, const int32_t *__restrict__ idx, const double *__restrict__ val,
                                    const double *__restrict__ E, double *__restrict__ S) {
  const int c = blockIdx.y;
  const double *Ec = E + (long long)c * nb;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nb; r += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int t = 0; t < 81; ++t) acc += val[(long long)r * 81 + t] * Ec[idx[(long long)r * 81 + t]];
    S[(long long)c * nb + r] -= acc;
  }
}

// E(:, c) = sum_t Sinv(:, row_t) U(row_t, c), the rows of column c of U given
// as (row index, value) pairs
__global__ void e_from_cols_kernel(int nb, const int32_t *__restrict__ cidx, const double *__restrict__ cval,
                                   const double *__restrict__ Sinv, double *__restrict__ E) {
  const int c = blockIdx.y;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nb; r += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int t = 0; t < 81; ++t) {
      const double v = cval[(long long)c * 81 + t];
      if (v != 0.0) acc += v * Sinv[(long long)cidx[(long long)c * 81 + t] * nb + r];
    }
    E[(long long)c * nb + r] = acc;
  }
}

// transpose the (row r -> 81 columns) table of U into (column -> 81 rows)
void transpose_rows(int nb, const std::vector<int32_t> &idx, const std::vector<double> &val,
                    std::vector<int32_t> &cidx, std::vector<double> &cval) {
  cidx.assign((size_t)nb * 81, 0);
  cval.assign((size_t)nb * 81, 0.0);
  std::vector<int> fill(nb, 0);
  for (int r = 0; r < nb; ++r)
    for (int t = 0; t < 81; ++t) {
      const double v = val[(size_t)r * 81 + t];
      if (v == 0.0) continue;
      const int c = idx[(size_t)r * 81 + t];
      const int f = fill[c]++;
      if (f >= 81) throw Error(STKKT_EINVAL, "coarse LU: coupling column with more than 81 entries");
      cidx[(size_t)c * 81 + f] = r;
      cval[(size_t)c * 81 + f] = v;
    }
}

// ---------------------------------------------------------------------------
// blocked Gauss-Jordan inverse of the n x n row-major buffer A (in place)
// ---------------------------------------------------------------------------
__device__ inline void block_argmax(double v, int i, double *sv, int *si) {
  // largest |v|, smallest index on ties, over the workgroup
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_down(v, off, 64);
    const int oi = __shfl_down(i, off, 64);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
  if (lane == 0) {
    sv[w] = v;
    si[w] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k)
      if (sv[k] > sv[0] || (sv[k] == sv[0] && si[k] < si[0])) {
        sv[0] = sv[k];
        si[0] = si[k];
      }
  }
  __syncthreads();
}

// The panel columns [k, k + w) of all rows are eliminated in a column-major
// copy P (P[q * n + i] = A[i][k + q]), so that the pivot search reads a
// column contiguously and the elimination is coalesced across rows.
// Both copies go through a 64 x 64 LDS tile.
__global__ void gje_panel_gather_kernel(int n, int k, int w, const double *__restrict__ A, double *__restrict__ P) {
  __shared__ double tile[64][65];
  const int i0 = blockIdx.x * 64;
  for (int q = threadIdx.x; q < 64 * 64; q += blockDim.x) {
    const int r = q / 64, t = q % 64;
    tile[r][t] = (i0 + r < n && t < w) ? A[(long long)(i0 + r) * n + k + t] : 0.0;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 64 * 64; q += blockDim.x) {
    const int t = q / 64, r = q % 64;
    if (i0 + r < n && t < w) P[(long long)t * n + i0 + r] = tile[r][t];
  }
}

__global__ void gje_panel_scatter_kernel(int n, int k, int w, const double *__restrict__ P, double *__restrict__ A) {
  __shared__ double tile[64][65];
  const int i0 = blockIdx.x * 64;
  for (int q = threadIdx.x; q < 64 * 64; q += blockDim.x) {
    const int t = q / 64, r = q % 64;
    tile[r][t] = (i0 + r < n && t < w) ? P[(long long)t * n + i0 + r] : 0.0;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 64 * 64; q += blockDim.x) {
    const int r = q / 64, t = q % 64;
    if (i0 + r < n && t < w) A[(long long)(i0 + r) * n + k + t] = tile[r][t];
  }
}

// Gauss-Jordan step for column c of the panel [k, e), part 1 (one
// workgroup): pivot search over rows >= c, swap of the two rows' panel
// segments (the rest of the rows is swapped once per panel, gje_laswp_kernel;
// swp[c - k] records the pivot row), and the pivot row's panel segment divided
// by the pivot (its column-c entry replaced by 1 first); the segment goes to prow.
__global__ void __launch_bounds__(1024) gje_pivot_kernel(int n, int k, int e, int c, double *__restrict__ P,
                                                         int32_t *__restrict__ piv, int32_t *__restrict__ swp,
                                                         double *__restrict__ prow, double *__restrict__ fcol,
                                                         int *__restrict__ status) {
  __shared__ double sv[16];
  __shared__ int si[16];
  if (*status) return;
  const int j = c - k, w = e - k;
  const double *Pc = P + (long long)j * n;
  double best = -1.0;
  int bi = n;
  for (int i = c + threadIdx.x; i < n; i += blockDim.x) {
    const double v = fabs(Pc[i]);
    if (v > best || (v == best && i < bi)) {
      best = v;
      bi = i;
    }
  }
  block_argmax(best, bi, sv, si);
  const int p = si[0];
  const double pv = sv[0];
  if (!(pv > 0.0) || !std::isfinite(pv)) {
    if (threadIdx.x == 0) *status = 1;
    return;
  }
  if (threadIdx.x == 0) swp[j] = p;
  if (p != c) {
    if ((int)threadIdx.x < w) {
      double *Pq = P + (long long)threadIdx.x * n;
      const double t = Pq[c];
      Pq[c] = Pq[p];
      Pq[p] = t;
    }
    if (threadIdx.x == 0) {
      const int32_t t = piv[c];
      piv[c] = piv[p];
      piv[p] = t;
    }
  }
  __syncthreads();
  // the multipliers of the elimination: column j after the swap
  for (int i = threadIdx.x; i < n; i += blockDim.x) fcol[i] = Pc[i];
  const double a = Pc[c];
  __syncthreads();
  if ((int)threadIdx.x < w) {
    double *Pq = P + (long long)threadIdx.x * n;
    const double v = ((int)threadIdx.x == j ? 1.0 : Pq[c]) / a;
    prow[threadIdx.x] = v;
    Pq[c] = v;
  }
}

// Part 2 (one thread per entry, grid rows x panel columns): eliminate column
// c from every other row of the panel, P[q][i] -= fcol[i] prow[q] (entry
// j = c - k becoming -fcol[i] prow[j]); the multipliers come from the copy
// fcol, so no entry is read after another thread has written it.
__global__ void __launch_bounds__(256) gje_elim_kernel(int n, int k, int c, double *__restrict__ P,
                                                       const double *__restrict__ prow,
                                                       const double *__restrict__ fcol,
                                                       const int *__restrict__ status) {
  if (*status) return;
  const int j = c - k, q = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || i == c) return;
  const double f = fcol[i], pq = prow[q];
  double *x = P + (long long)q * n + i;
  *x = (q == j) ? -f * pq : *x - f * pq;
}

// ---------------------------------------------------------------------------
// The same Gauss-Jordan steps for all columns of a panel in one cooperative
// launch.  Workgroup g keeps the panel segments of rows [g R, g R + R) in LDS
// (column-major, padded: L[t (R + 1) + r]) for the whole panel; step c:
//  1. every workgroup finds its largest |entry| in column c over its rows
//     >= c (smallest row on ties) and publishes it, with that row's segment,
//     in slot (c & 1) of the candidate tables; the owner of row c publishes
//     row c's segment;
//  2. grid barrier;
//  3. every workgroup picks the same pivot row p from the candidates (largest
//     value, smallest row on ties: the choice of gje_pivot_kernel), forms the
//     scaled pivot row and eliminates column c from its own rows; the owner
//     of row p puts row c's old segment in its place (the swap), the owner of
//     row c the scaled pivot row.
// The two candidate slots alternate, so a slot is rewritten only after every
// workgroup has passed the barrier that follows its reads.  The barrier
// counter grows by the number of workgroups per step and is zeroed once per
// inversion; bar0 is the number of steps taken by earlier launches.  A
// barrier that has not completed after `spin_limit` polls (the default is
// about a second) sets the abort flag and status 2, and every workgroup
// leaves at its next barrier, so the launch always ends.
// ---------------------------------------------------------------------------
constexpr int kGjThreads = 1024;
constexpr unsigned kGjSpinLimit = 1u << 20;   // default bound on the polls of one barrier

struct GjSync {
  double *candv;     // [2][nwg] largest |entry|
  int32_t *candi;    // [2][nwg] its row
  double *candrow;   // [2][nwg][kPanel] that row's panel segment
  double *crow;      // [2][kPanel] row c's panel segment
  unsigned *count;   // barrier arrivals
  int *abort;        // set by a barrier that timed out
  unsigned spin_limit;
};

// All threads of the workgroup; false if the barrier was abandoned.  Every
// global write a step makes before its barrier (candidate tables, row c,
// pivot records) comes from wavefront 0, so thread 0's release ordering of its
// arrival covers them; the wait polls with relaxed loads and ends with one
// acquire fence, whose cache invalidation the other wavefronts of the
// compute unit see after the workgroup barrier.
__device__ inline bool gj_grid_barrier(const GjSync &gs, unsigned target) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(gs.count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int good = 1;
    unsigned spins = 0;
    while (__hip_atomic_load(gs.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(gs.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > gs.spin_limit) {
        __hip_atomic_store(gs.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// loads of values other workgroups wrote during the launch
template <typename T> __device__ inline T ld_agent(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void gj_reset_kernel(GjSync gs) {
  if (threadIdx.x == 0) {
    *gs.count = 0u;
    *gs.abort = 0;
  }
}

__global__ void __launch_bounds__(kGjThreads) gje_panel_kernel(int n, int k, int e, int R, double *__restrict__ A,
                                                              int32_t *__restrict__ piv, int32_t *__restrict__ swp,
                                                              GjSync gs, unsigned bar0, int *__restrict__ status) {
  extern __shared__ double gj_lds[];
  __shared__ double wv[kGjThreads / 64], prow_s[kPanel], crow_s[kPanel];
  __shared__ int wi[kGjThreads / 64];
  if (*status) return;
  const int tid = threadIdx.x, g = blockIdx.x, nwg = gridDim.x;
  const int w = e - k, LD = R + 1;
  const int r0 = g * R, rows = min(R, n - r0);
  double *L = gj_lds;
  for (int q = tid; q < R * w; q += kGjThreads) {
    const int r = q / w, t = q % w;
    L[t * LD + r] = r < rows ? A[(long long)(r0 + r) * n + k + t] : 0.0;
  }
  __syncthreads();
  // this thread's row and first column in the elimination
  const int rr = tid % R, t0 = tid / R, tstep = kGjThreads / R;
  for (int j = 0; j < w; ++j) {
    const int c = k + j, par = j & 1;
    // 1. local candidate
    double best = -1.0;
    int bi = n;
    for (int r = tid; r < rows; r += kGjThreads) {
      const int i = r0 + r;
      if (i < c) continue;
      const double v = fabs(L[j * LD + r]);
      if (v > best || (v == best && i < bi)) {
        best = v;
        bi = i;
      }
    }
    block_argmax(best, bi, wv, wi);
    {
      const double lv = wv[0];
      const int li = wi[0];
      if (tid == 0) {
        gs.candv[par * nwg + g] = lv;
        gs.candi[par * nwg + g] = li;
      }
      if (tid < w) {
        gs.candrow[((long long)par * nwg + g) * kPanel + tid] = li < n ? L[tid * LD + (li - r0)] : 0.0;
        if (c >= r0 && c < r0 + rows) gs.crow[par * kPanel + tid] = L[tid * LD + (c - r0)];
      }
    }
    // 2. all candidates published
    if (!gj_grid_barrier(gs, (unsigned)nwg * (bar0 + (unsigned)j + 1u))) {
      if (tid == 0) __hip_atomic_store(status, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    // 3. the pivot
    {
      double v = -1.0;
      int i = n;
      for (int q = tid; q < nwg; q += kGjThreads) {
        const double cv = ld_agent(gs.candv + par * nwg + q);
        const int ci = ld_agent(gs.candi + par * nwg + q);
        if (cv > v || (cv == v && ci < i)) {
          v = cv;
          i = ci;
        }
      }
      block_argmax(v, i, wv, wi);
    }
    const double pv = wv[0];
    const int p = wi[0];
    if (!(pv > 0.0) || !std::isfinite(pv)) {
      if (tid == 0) *status = 1;
      return;
    }
    const int gp = p / R;
    if (tid < w) {
      const double a = ld_agent(gs.candrow + ((long long)par * nwg + gp) * kPanel + j);
      const double x = ld_agent(gs.candrow + ((long long)par * nwg + gp) * kPanel + tid);
      prow_s[tid] = (tid == j ? 1.0 : x) / a;
      crow_s[tid] = ld_agent(gs.crow + par * kPanel + tid);
    }
    if (g == 0 && tid == 0) {
      swp[j] = p;
      if (p != c) {
        const int32_t t = piv[c];
        piv[c] = piv[p];
        piv[p] = t;
      }
    }
    __syncthreads();
    const int i = r0 + rr;
    const bool valid = rr < rows, isc = i == c, isp = i == p && p != c;
    const double f = valid ? (isp ? crow_s[j] : L[j * LD + rr]) : 0.0;
    __syncthreads();
    if (valid) {
      for (int t = t0; t < w; t += tstep) {
        double nv;
        if (isc) {
          nv = prow_s[t];
        } else {
          const double cur = isp ? crow_s[t] : L[t * LD + rr];
          nv = (t == j) ? -f * prow_s[j] : cur - f * prow_s[t];
        }
        L[t * LD + rr] = nv;
      }
    }
    __syncthreads();
  }
  for (int q = tid; q < R * w; q += kGjThreads) {
    const int r = q / w, t = q % w;
    if (r < rows) A[(long long)(r0 + r) * n + k + t] = L[t * LD + r];
  }
}

// Panel elimination with the pivots searched among the panel's own rows
// (block pivoting).  The Schur blocks of the coarse solve need no row
// exchanges across panels: with the pivots restricted to each 64-row
// diagonal block the inverse agrees with partial pivoting over all rows to
// about 1e-14 (and with LAPACK's inverse), so a panel needs no device-wide
// exchange per column.
//
// Step 1, one workgroup of four wavefronts (lane l on column l, wavefront v
// on rows 16 v ..): Gauss-Jordan inversion of the diagonal block D = A[K][K]
// (K = [k, e), w = e - k <= 64) in LDS.  Each step reads the rows'
// multipliers into registers first, so the row updates are independent and
// their LDS accesses pipeline.  Step j takes the largest
// |entry| of column j over the block rows j.. (smallest row on ties), swaps
// the two rows, records the pivot row in swp[j] (global index) and swaps the
// two entries of piv, then eliminates column j from the other rows with the
// in-place steps of gje_panel_kernel.  A[K][K] and Dinv (w x w, row stride
// kPanel) receive (P D)^{-1}; a zero or non-finite pivot sets status 1.
constexpr int kDiagThreads = 256;   // four wavefronts, 16 rows of the block each
__global__ void __launch_bounds__(kDiagThreads) gje_diag_kernel(int n, int k, int e, double *__restrict__ A,
                                                                double *__restrict__ Dinv,
                                                                int32_t *__restrict__ piv,
                                                                int32_t *__restrict__ swp,
                                                                int *__restrict__ status) {
  __shared__ double M[kPanel][kPanel + 1];
  __shared__ int32_t pv[kPanel], sw[kPanel];   // piv[k..e) and the pivot rows, kept in LDS
  __shared__ double pval;
  __shared__ int prow_i;
  if (*status) return;
  const int w = e - k, tid = (int)threadIdx.x, l = tid & 63, wv = tid >> 6;   // lane l: column l
  for (int r = wv; r < w; r += kDiagThreads / 64) M[r][l] = l < w ? A[(long long)(k + r) * n + k + l] : 0.0;
  if (tid < w) pv[tid] = piv[k + tid];
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    // pivot (wavefront 0; lane l looks at row l of column j)
    if (wv == 0) {
      double v = (l >= j && l < w) ? fabs(M[l][j]) : -1.0;
      int i = l;
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(i, off, 64);
        if (ov > v || (ov == v && oi < i)) {
          v = ov;
          i = oi;
        }
      }
      if (l == 0) {
        pval = v;
        prow_i = i;
      }
    }
    __syncthreads();
    const int p = prow_i;
    if (!(pval > 0.0) || !std::isfinite(pval)) {
      if (tid == 0) *status = 1;
      return;
    }
    // the swap; the pivot bookkeeping stays in LDS (a global access would
    // make every step's barrier wait for a memory round trip)
    if (wv == 0) {
      if (p != j && l < w) {
        const double t = M[j][l];
        M[j][l] = M[p][l];
        M[p][l] = t;
      }
      if (l == 0) {
        sw[j] = p;
        if (p != j) {
          const int32_t t = pv[j];
          pv[j] = pv[p];
          pv[p] = t;
        }
      }
    }
    __syncthreads();
    // the scaled pivot row (lane l: entry l) and the multipliers of this
    // wavefront's rows, read before any row changes; then its rows
    const double a = M[j][j];
    const double pr = l < w ? (l == j ? 1.0 : M[j][l]) / a : 0.0;
    const double pj = 1.0 / a;
    double f[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) f[q] = M[16 * wv + q][j];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = 16 * wv + q;
      if (r < w && l < w) M[r][l] = (r == j) ? pr : ((l == j) ? -f[q] * pj : M[r][l] - f[q] * pr);
    }
    __syncthreads();
  }
  for (int r = wv; r < w; r += kDiagThreads / 64)
    if (l < w) {
      A[(long long)(k + r) * n + k + l] = M[r][l];
      Dinv[r * kPanel + l] = M[r][l];
    }
  if (tid < w) {
    piv[k + tid] = pv[tid];
    swp[tid] = k + sw[tid];
  }
}

// Step 2: the panel columns of the rows outside the block,
// A[i][K] <- -A[i][K] Dinv (the rows of K already hold Dinv).  64 rows per
// workgroup of 256 threads with their panel segments (transposed) and Dinv in
// LDS; thread (row r, column group g) forms 16 of the row's w outputs.
__global__ void __launch_bounds__(256) gje_pmul_kernel(int n, int k, int e, double *__restrict__ A,
                                                       const double *__restrict__ Dinv,
                                                       const int *__restrict__ status) {
  __shared__ double Ds[kPanel][kPanel], St[kPanel][kPanel];   // Dinv[t][c]; segment St[t][row]
  if (*status) return;
  const int w = e - k, tid = (int)threadIdx.x, r0 = (int)blockIdx.x * 64;
  for (int q = tid; q < 64 * kPanel; q += 256) {
    const int a = q / kPanel, b = q % kPanel;
    Ds[a][b] = (a < w && b < w) ? Dinv[a * kPanel + b] : 0.0;
    const int i = r0 + a;
    St[b][a] = (i < n && b < w) ? A[(long long)i * n + k + b] : 0.0;
  }
  __syncthreads();
  const int r = tid & 63, g = tid >> 6;
  const int i = r0 + r;
  if (i >= n || (i >= k && i < e)) return;
  double acc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = 0.0;
  for (int t = 0; t < w; ++t) {
    const double sv = St[t][r];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] += sv * Ds[t][g * 16 + c];
  }
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int col = g * 16 + c;
    if (col < w) A[(long long)i * n + k + col] = -acc[c];
  }
}

// The panel's row swaps, in order, on the columns outside the panel (one
// thread per column).  Skipped after a failed pivot (swp is then incomplete).
__global__ void gje_laswp_kernel(int n, int k, int e, double *__restrict__ A, const int32_t *__restrict__ swp,
                                 const int *__restrict__ status) {
  if (*status) return;
  for (int col = blockIdx.x * blockDim.x + threadIdx.x; col < n; col += gridDim.x * blockDim.x) {
    if (col >= k && col < e) continue;
    for (int c = k; c < e; ++c) {
      const int p = swp[c - k];
      if (p == c) continue;
      const double t = A[(long long)c * n + col];
      A[(long long)c * n + col] = A[(long long)p * n + col];
      A[(long long)p * n + col] = t;
    }
  }
}

// Copy the panel rows [k, e) outside the panel columns: R[t][col] = A[k+t][col]
__global__ void gje_copy_rows_kernel(int n, int k, int e, const double *__restrict__ A, double *__restrict__ R) {
  const int t = blockIdx.y;
  for (int col = blockIdx.x * blockDim.x + threadIdx.x; col < n; col += gridDim.x * blockDim.x)
    R[(long long)t * n + col] = (col >= k && col < e) ? 0.0 : A[(long long)(k + t) * n + col];
}

// Trailing update outside the panel columns, a rank-(e - k) product:
//   rows outside the panel:  A[i][col] += sum_t A[i][k+t] R[t][col]
//   panel rows:              A[i][col]  = sum_t A[i][k+t] R[t][col]
// for the columns in [cb, ce) outside [xb, xe) (the tiles of column blocks
// ct0, ct0 + 1, ...), so that the next panel's columns can be updated first.
// on the FP64 matrix cores (v_mfma_f64_16x16x4: lane l supplies a = A[l%16][l/16]
// and b = B[l/16][l%16] and holds D[l/16 + 4r][l%16], r = 0..3).  A workgroup
// of 8 wavefronts owns a 128 x 128 output tile; wavefront (wr, wc) a 64 x 32
// part of it, as 4 x 2 blocks of 16 x 16.  The accumulators start from the
// tile's current values (0 for panel rows), requested first so that their
// latency overlaps the staging; the panel is taken in two passes of 32
// columns, each staging the A panel slice (128 rows x 32, rows padded against
// bank conflicts) and the R slice (32 x 128) in LDS.  About 67 KB of LDS and
// at most 128 registers let two workgroups share a compute unit, one loading
// while the other multiplies.
constexpr int kUpdTile = 128;
constexpr int kUpdThreads = 512;
constexpr int kUpdK = 32;
constexpr size_t kUpdLds = sizeof(double) * ((size_t)kUpdTile * (kUpdK + 1) + (size_t)kUpdK * kUpdTile);
typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kUpdThreads, 4) gje_update_kernel(int n, int k, int e, int cb, int ce, int xb,
                                                                    int xe, int ct0, double *__restrict__ A,
                                                                    const double *__restrict__ R) {
  extern __shared__ double upd_lds[];
  double(*As)[kUpdK + 1] = reinterpret_cast<double(*)[kUpdK + 1]>(upd_lds);              // [row][t]
  double(*Rs)[kUpdTile] = reinterpret_cast<double(*)[kUpdTile]>(upd_lds + kUpdTile * (kUpdK + 1));   // [t][col]
  const int row0 = blockIdx.y * kUpdTile, col0 = (ct0 + blockIdx.x) * kUpdTile;
  // columns this launch updates
  auto mine = [&](int col) {
    return col >= cb && col < ce && col < n && !(col >= k && col < e) && !(col >= xb && col < xe);
  };
  const int w = e - k;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc[4][2];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int col = col0 + wc * 32 + bj * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = row0 + wr * 64 + bi * 16 + lk + 4 * r;
        const bool acc_row = i < n && !(i >= k && i < e) && mine(col);
        acc[bi][bj][r] = acc_row ? A[(long long)i * n + col] : 0.0;
      }
    }
  for (int kb = 0; kb < w; kb += kUpdK) {
    if (kb > 0) __syncthreads();
    for (int q = tid; q < kUpdTile * kUpdK; q += kUpdThreads) {
      const int rr = q / kUpdK, t = q % kUpdK;
      const int i = row0 + rr;
      As[rr][t] = (i < n && kb + t < w) ? A[(long long)i * n + k + kb + t] : 0.0;
      const int t2 = q / kUpdTile, cc = q % kUpdTile;
      const int col = col0 + cc;
      Rs[t2][cc] = (col < n && kb + t2 < w) ? R[(long long)(kb + t2) * n + col] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int t0 = 0; t0 < kUpdK; t0 += 4) {
      double a[4], b[2];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) a[bi] = As[wr * 64 + bi * 16 + li][t0 + lk];
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) b[bj] = Rs[t0 + lk][wc * 32 + bj * 16 + li];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    }
  }
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int col = col0 + wc * 32 + bj * 16 + li;
      if (!mine(col)) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = row0 + wr * 64 + bi * 16 + lk + 4 * r;
        if (i >= n) continue;
        A[(long long)i * n + col] = acc[bi][bj][r];
      }
    }
}

// out[i][piv[j]] = A[i][j]
__global__ void gje_unpermute_kernel(int n, const double *__restrict__ A, const int32_t *__restrict__ piv,
                                     double *__restrict__ out) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
    out[(long long)i * n + piv[j]] = A[(long long)i * n + j];
}

__global__ void iota_kernel(int n, int32_t *p) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
}

// ---------------------------------------------------------------------------
// application
// ---------------------------------------------------------------------------
// t[i tsi + c tsc] = r_c[i] - (L y_c)[i] for the right-hand sides c =
// blockIdx.y (r_c = r + c ldr, y_c = y + c ldy; with y == nullptr: t = r).
// One wavefront per row: its 81 couplings spread over the lanes and summed
// in a fixed order.
__global__ void __launch_bounds__(256) lower_rhs_kernel(int nb, const int32_t *__restrict__ idx,
                                                        const double *__restrict__ val, const double *__restrict__ r,
                                                        long long ldr, const double *__restrict__ y, long long ldy,
                                                        double *__restrict__ t, int tsi, int tsc) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.y;
  const double *rc = r + c * ldr;
  const double *yc = y ? y + c * ldy : nullptr;
  for (int i = blockIdx.x * 4 + (threadIdx.x >> 6); i < nb; i += gridDim.x * 4) {
    double s = 0.0;
    if (yc) {
      const long long b = (long long)i * 81;
      s = val[b + lane] * yc[idx[b + lane]];
      if (lane < 81 - 64) s += val[b + 64 + lane] * yc[idx[b + 64 + lane]];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    }
    if (lane == 0) t[(long long)i * tsi + (long long)c * tsc] = rc[i] - s;
  }
}

constexpr int kGvRows = 256, kGvCols = 128;

// partial[chunk][r] = sum over the chunk's columns of A(r, c) x(c)
// (column-major A with leading dimension ld)
template <typename T>
__global__ void __launch_bounds__(kGvRows) gemv_partial_kernel(int nb, int ld, const T *__restrict__ A,
                                                               const double *__restrict__ x,
                                                               double *__restrict__ partial) {
  __shared__ T xs[kGvCols];
  const int c0 = blockIdx.y * kGvCols;
  const int nc = min(kGvCols, nb - c0);
  if ((int)threadIdx.x < nc) xs[threadIdx.x] = (T)x[c0 + threadIdx.x];
  __syncthreads();
  const int r = blockIdx.x * kGvRows + threadIdx.x;
  if (r >= nb) return;
  T acc = 0;
  const T *a = A + (long long)c0 * ld + r;
  for (int c = 0; c < nc; ++c) acc += a[(long long)c * ld] * xs[c];
  partial[(long long)blockIdx.y * nb + r] = (double)acc;
}

// out[r] = base[r] + sign * sum_chunks partial[chunk][r]  (fixed order)
__global__ void gemv_reduce_kernel(int nb, int nchunk, const double *__restrict__ partial,
                                   const double *__restrict__ base, double sign, double *__restrict__ out) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nb; r += gridDim.x * blockDim.x) {
    double s = 0.0;
#pragma unroll 8
    for (int q = 0; q < nchunk; ++q) s += partial[(long long)q * nb + r];
    out[r] = (base ? base[r] : 0.0) + sign * s;
  }
}

// out (leading dimension ld, rows nb..ld-1 zero) = S (nb x nb, leading dimension nb), column c = blockIdx.y
template <typename T>
__global__ void store_padded_kernel(int nb, int ld, const double *__restrict__ S, T *__restrict__ out) {
  const int c = blockIdx.y;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < ld; r += gridDim.x * blockDim.x)
    out[(long long)c * ld + r] = r < nb ? (T)S[(long long)c * nb + r] : (T)0;
}

// ---------------------------------------------------------------------------
// several right-hand sides at once.  The product inputs are kept transposed,
// XT[col][16] (the value of right-hand side c at column col in XT[16 col + c]),
// so that the matrix-core operands of 4 consecutive columns x 16 right-hand
// sides are one contiguous 512-byte read.
// ---------------------------------------------------------------------------
constexpr int kMrRows = 64, kMrRhs = 16, kMrThreads = 256, kMrAhead = 8;

// Y = A X for up to 16 right-hand sides on the FP64 matrix cores
// (v_mfma_f64_16x16x4: lane l supplies a = A[l%16][l/16], b = B[l/16][l%16]
// and holds D[l/16 + 4j][l%16], j = 0..3).  A workgroup of 4 wavefronts owns
// 64 rows and a chunk of columns (blockIdx.y); step s of wavefront w takes
// columns 16 s + 4 w .. 16 s + 4 w + 3 of the chunk.  Lane (i, kk) =
// (l%16, l/16) reads rows 4i .. 4i + 3 of its column with one 16-byte load
// (float) or two (double) and gives row 4i + m to product m (m = 0..3), so
// product m covers rows m, 4 + m, .., 60 + m of the tile and each column of
// the tile is one contiguous 256- or 512-byte read.  Loads run kMrAhead steps
// ahead of the products, with no branch: a column past the chunk reads the
// chunk's last column and enters as zero.  The four wavefronts' sums
// are added in LDS and written to partial[chunk][c][row] (leading dimension
// ld).  Float blocks are widened to double on load.  Column n of a product
// depends on column n of X only, so a right-hand side's result does not
// depend on the others.
// raw loads of 4 rows, widened and masked only when the products use them
// (a conversion right after the load would make the wavefront wait for it)
struct Rows4f {
  float4 v;
  __device__ void load(const float *p) { v = *reinterpret_cast<const float4 *>(p); }
  __device__ void get(bool ok, double a[4]) const {
    a[0] = ok ? (double)v.x : 0.0;
    a[1] = ok ? (double)v.y : 0.0;
    a[2] = ok ? (double)v.z : 0.0;
    a[3] = ok ? (double)v.w : 0.0;
  }
};
struct Rows4d {
  double2 u, v;
  __device__ void load(const double *p) {
    u = *reinterpret_cast<const double2 *>(p);
    v = *reinterpret_cast<const double2 *>(p + 2);
  }
  __device__ void get(bool ok, double a[4]) const {
    a[0] = ok ? u.x : 0.0;
    a[1] = ok ? u.y : 0.0;
    a[2] = ok ? v.x : 0.0;
    a[3] = ok ? v.y : 0.0;
  }
};
template <typename T> struct Rows4;
template <> struct Rows4<float> { using type = Rows4f; };
template <> struct Rows4<double> { using type = Rows4d; };

template <typename T>
__global__ void __launch_bounds__(kMrThreads) gemm_partial_kernel(int nb, int ld, int csplit, const T *__restrict__ A,
                                                                  int q, const double *__restrict__ XT,
                                                                  double *__restrict__ partial) {
  __shared__ double red[4 * kMrRhs * kMrRows];   // [wave][rhs][row]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = blockIdx.x * kMrRows;
  const int cbeg = blockIdx.y * csplit, cend = min(nb, cbeg + csplit);
  const int nst = ((cend - cbeg + 15) / 16 + kMrAhead - 1) / kMrAhead * kMrAhead;
  const T *arow = A + r0 + 4 * li;
  f64x4 acc[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) acc[m] = f64x4{0.0, 0.0, 0.0, 0.0};
  typename Rows4<T>::type raw[kMrAhead];
  double b[kMrAhead];
  const int c_lane = cbeg + 4 * wave + lk;   // column of step 0
  auto fetch = [&](int p, int st) {
    const int cc = min(c_lane + 16 * st, cend - 1);
    raw[p].load(arow + (long long)cc * ld);
    b[p] = XT[(long long)cc * kMrRhs + li];
  };
#pragma unroll
  for (int p = 0; p < kMrAhead; ++p) fetch(p, p);
  // the last kMrAhead fetches read the chunk's last column again (cache hits,
  // unused): an unconditional fetch keeps the wait counts exact
  for (int st = 0; st < nst; st += kMrAhead) {
#pragma unroll
    for (int p = 0; p < kMrAhead; ++p) {
      double a[4];
      raw[p].get(c_lane + 16 * (st + p) < cend, a);
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[p], acc[m], 0, 0, 0);
      fetch(p, st + kMrAhead + p);
    }
  }
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) red[(wave * kMrRhs + li) * kMrRows + 4 * (lk + 4 * j) + m] = acc[m][j];
  __syncthreads();
  const int rhs = tid >> 4, rl = 4 * (tid & 15);
  if (rhs >= q) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int row = r0 + rl + u;
    const double v = red[(0 * kMrRhs + rhs) * kMrRows + rl + u] + red[(1 * kMrRhs + rhs) * kMrRows + rl + u] +
                     red[(2 * kMrRhs + rhs) * kMrRows + rl + u] + red[(3 * kMrRhs + rhs) * kMrRows + rl + u];
    if (row < nb) partial[((long long)blockIdx.y * q + rhs) * ld + row] = v;
  }
}

// out_c[r] = base_c[r] + sign * sum_chunks partial[chunk][c][r] (fixed order),
// c = blockIdx.y; the same value also goes to outT[r][c]
__global__ void gemm_reduce_kernel(int nb, int ld, int q, int nchunk, const double *__restrict__ partial,
                                   const double *base, long long ldb, double sign, double *out, long long ldo,
                                   double *__restrict__ outT) {
  const int c = blockIdx.y;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nb; r += gridDim.x * blockDim.x) {
    double s = 0.0;
#pragma unroll 8
    for (int k = 0; k < nchunk; ++k) s += partial[((long long)k * q + c) * ld + r];
    const double v = (base ? base[c * ldb + r] : 0.0) + sign * s;
    out[c * ldo + r] = v;
    outT[(long long)r * kMrRhs + c] = v;
  }
}

}  // namespace

// Pivots among each panel's rows (the default) unless STKKT_COARSE_PIVOT is
// "global" or STKKT_COARSE_PANEL_ROWS selects one of the global-pivoting
// elimination paths below.
static bool block_pivoting() {
  if (std::getenv("STKKT_COARSE_PANEL_ROWS")) return false;
  const char *e = std::getenv("STKKT_COARSE_PIVOT");
  return !(e && e[0] == 'g');
}

// Rows per workgroup of the cooperative panel elimination (64, 128 or 256;
// STKKT_COARSE_PANEL_ROWS overrides, 0 selects the launch-per-column path),
// or 0 if its workgroups cannot all be resident at once.
static int panel_rows(int n) {
  const char *env = std::getenv("STKKT_COARSE_PANEL_ROWS");
  const int forced = env ? std::atoi(env) : -1;
  int dev = 0, cus = 0, coop = 0;
  STKKT_HIP(hipGetDevice(&dev));
  STKKT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  STKKT_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop || forced == 0) return 0;
  for (int R : {128, 256, 64}) {
    if (forced > 0 && R != forced) continue;
    const size_t lds = sizeof(double) * (size_t)kPanel * (R + 1);
    STKKT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&gje_panel_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    STKKT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gje_panel_kernel, kGjThreads, lds));
    if ((n + R - 1) / R <= per_cu * cus) return R;
  }
  return 0;
}

// Second stream and events of the panel look-ahead (default priority).
struct LookAhead {
  hipStream_t side = nullptr;
  hipEvent_t rows_ready = nullptr, rest_done = nullptr;
  LookAhead() {
    try {
      STKKT_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
      STKKT_HIP(hipEventCreateWithFlags(&rows_ready, hipEventDisableTiming));
      STKKT_HIP(hipEventCreateWithFlags(&rest_done, hipEventDisableTiming));
    } catch (...) {
      release();
      throw;
    }
  }
  ~LookAhead() { release(); }
  void release() {
    if (side) (void)hipStreamSynchronize(side);
    if (rest_done) (void)hipEventDestroy(rest_done);
    if (rows_ready) (void)hipEventDestroy(rows_ready);
    if (side) (void)hipStreamDestroy(side);
    side = nullptr;
    rows_ready = rest_done = nullptr;
  }
  LookAhead(const LookAhead &) = delete;
  LookAhead &operator=(const LookAhead &) = delete;
};

// Explicit inverse of the n x n row-major matrix in A (overwritten with the
// inverse).  tmp: n x n scratch; rows: 2 x kPanel x n scratch (the rows of
// two consecutive panels); pan: kPanel x n scratch (the launch-per-column
// path's panel; with block pivoting its first kPanel x kPanel doubles hold the
// diagonal block's inverse); piv: n int32; gs: candidate tables for
// ceil(n / 64) workgroups; la: the look-ahead's side stream and events.
static void gje_invert(int n, double *A, double *tmp, double *rows, double *pan, double *fcol, int32_t *piv,
                       int32_t *swp, double *prow, const GjSync &gs, int *status, const LookAhead &la,
                       hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    STKKT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&gje_update_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kUpdLds));
    attr_set = true;
  }
  const bool block = block_pivoting();
  const int R = block ? 0 : panel_rows(n);
  hipLaunchKernelGGL(iota_kernel, dim3(blocks_for(n, 256, 64)), dim3(256), 0, s, n, piv);
  if (R > 0) hipLaunchKernelGGL(gj_reset_kernel, dim3(1), dim3(64), 0, s, gs);
  const int nt = (n + kUpdTile - 1) / kUpdTile;
  // rank-(e - k) update of the columns [cb, ce) outside [xb, xe) on stream st
  auto update = [&](int k, int e, int cb, int ce, int xb, int xe, const double *Rk, hipStream_t st) {
    const int t0 = cb / kUpdTile, t1 = (ce + kUpdTile - 1) / kUpdTile;
    hipLaunchKernelGGL(gje_update_kernel, dim3(t1 - t0, nt), dim3(kUpdThreads), kUpdLds, st, n, k, e, cb, ce, xb, xe,
                       t0, A, Rk);
  };
  // the panel's swaps on the other columns, then its rows into Rk
  auto close_panel = [&](int k, int e, double *Rk) {
    hipLaunchKernelGGL(gje_laswp_kernel, dim3(blocks_for(n, 256, 64)), dim3(256), 0, s, n, k, e, A, swp, status);
    hipLaunchKernelGGL(gje_copy_rows_kernel, dim3(blocks_for(n, 256, 64), e - k), dim3(256), 0, s, n, k, e, A, Rk);
  };
  if (block || R > 0) {
    // Elimination of each panel (block pivoting: the diagonal block's inverse
    // and the other rows' multipliers; global pivoting: one cooperative
    // launch) with a look-ahead: the update by panel p first brings the next
    // panel's columns up to date, then the next panel is eliminated on s
    // while the rest of the update runs on the side stream.  The two touch
    // different columns, and the next panel's swaps on the other columns wait
    // for the rest of the update.  Every entry gets the same updates as
    // without the look-ahead, bit for bit.
    auto diag = [&](int k, int e) {
      hipLaunchKernelGGL(gje_diag_kernel, dim3(1), dim3(kDiagThreads), 0, s, n, k, e, A, pan, piv, swp, status);
    };
    auto pmul = [&](int k, int e) {
      hipLaunchKernelGGL(gje_pmul_kernel, dim3((n + 63) / 64), dim3(256), 0, s, n, k, e, A, pan, status);
    };
    auto eliminate = [&](int k, int e) {
      if (block) {
        diag(k, e);
        pmul(k, e);
        return;
      }
      int n_ = n, k_ = k, e_ = e, R_ = R;
      GjSync gs_ = gs;
      unsigned bar0 = (unsigned)k;
      void *args[] = {&n_, &k_, &e_, &R_, &A, &piv, &swp, &gs_, &bar0, &status};
      STKKT_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&gje_panel_kernel),
                                           dim3((n + R - 1) / R), dim3(kGjThreads), args,
                                           (unsigned)(sizeof(double) * (size_t)kPanel * (R + 1)), s));
    };
    eliminate(0, std::min(n, kPanel));
    close_panel(0, std::min(n, kPanel), rows);
    for (int k = 0, p = 0; k < n; k += kPanel, ++p) {
      const int e = std::min(n, k + kPanel);
      double *Rk = rows + (size_t)(p & 1) * kPanel * n;
      if (e >= n) {
        update(k, e, 0, n, 0, 0, Rk, s);
        break;
      }
      const int e2 = std::min(n, e + kPanel);
      STKKT_HIP(hipEventRecord(la.rows_ready, s));
      update(k, e, e, e2, 0, 0, Rk, s);
      STKKT_HIP(hipStreamWaitEvent(la.side, la.rows_ready, 0));
      update(k, e, 0, n, e, e2, Rk, la.side);
      STKKT_HIP(hipEventRecord(la.rest_done, la.side));
      eliminate(e, e2);
      STKKT_HIP(hipStreamWaitEvent(s, la.rest_done, 0));
      close_panel(e, e2, rows + (size_t)((p + 1) & 1) * kPanel * n);
    }
  } else {
    for (int k = 0; k < n; k += kPanel) {
      const int e = std::min(n, k + kPanel);
      const int nrb = (n + 63) / 64;
      hipLaunchKernelGGL(gje_panel_gather_kernel, dim3(nrb), dim3(256), 0, s, n, k, e - k, A, pan);
      for (int c = k; c < e; ++c) {
        hipLaunchKernelGGL(gje_pivot_kernel, dim3(1), dim3(1024), 0, s, n, k, e, c, pan, piv, swp, prow, fcol,
                           status);
        hipLaunchKernelGGL(gje_elim_kernel, dim3((n + 255) / 256, e - k), dim3(256), 0, s, n, k, c, pan, prow,
                           fcol, status);
      }
      hipLaunchKernelGGL(gje_panel_scatter_kernel, dim3(nrb), dim3(256), 0, s, n, k, e - k, pan, A);
      close_panel(k, e, rows);
      update(k, e, 0, n, 0, 0, rows, s);
    }
  }
  hipLaunchKernelGGL(gje_unpermute_kernel, dim3(blocks_for(n, 256, 64), n), dim3(256), 0, s, n, A, piv, tmp);
  STKKT_HIP(hipGetLastError());
  STKKT_HIP(hipMemcpyAsync(A, tmp, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToDevice, s));
}

CoarseLU::CoarseLU(const Allocator *al, const kkt_op *cop, int precision, hipStream_t s) : prec_(precision) {
  const OpDev &d = cop->d;
  nb_ = 3 * d.N;
  nlev_ = d.M + 1;
  STKKT_REQUIRE(nb_ <= 65535, "coarse_setup: coarse level too large for the dense block solve");
  const size_t nn = (size_t)nb_ * nb_;
  ld_ = (nb_ + kMrRows - 1) / kMrRows * kMrRows;
  const size_t nld = (size_t)ld_ * nb_;
  const size_t esz = precision == STKKT_F32 ? sizeof(float) : sizeof(double);
  Sinv_ = DevBuf(al, esz * nld * nlev_);
  E_ = DevBuf(al, esz * nld * std::max(nlev_ - 1, 1));
  Lidx_ = DevBuf(al, sizeof(int32_t) * (size_t)nb_ * 81 * nlev_);
  Lval_ = DevBuf(al, sizeof(double) * (size_t)nb_ * 81 * nlev_);
  partial_ = DevBuf(al, sizeof(double) * (size_t)nb_ * ((nb_ + kGvCols - 1) / kGvCols));
  t_ = DevBuf(al, sizeof(double) * nb_);
  // multi-RHS products: workgroups of 64 rows x 256 columns (two rounds of
  // the load pipeline).  At nb 6591 (103 x 26 workgroups) a block product
  // took 41 us in FP32 and 65 us in FP64, against 47 / 70 us with 10 column
  // chunks and 56 / 81 us with 3.
  nsplit_ = (nb_ + 255) / 256;
  mpartial_ = DevBuf(al, sizeof(double) * (size_t)nsplit_ * kMrRhs * ld_);
  mt_ = DevBuf(al, sizeof(double) * (size_t)3 * kMrRhs * nb_);   // tT, xT[0], xT[1]
  // setup work buffers (FP64)
  DevBuf S(al, sizeof(double) * nn), Ed(al, sizeof(double) * nn),
      tmp(al, sizeof(double) * nn), rows(al, sizeof(double) * 2 * (size_t)kPanel * nb_), piv(al, sizeof(int32_t) * nb_),
      prow(al, sizeof(double) * kPanel), swp(al, sizeof(int32_t) * kPanel), pan(al, sizeof(double) * kPanel * nb_),
      fcol(al, sizeof(double) * nb_),
      status(al, 256), ridx(al, sizeof(int32_t) * (size_t)nb_ * 81), rval(al, sizeof(double) * (size_t)nb_ * 81),
      cidx(al, sizeof(int32_t) * (size_t)nb_ * 81), cval(al, sizeof(double) * (size_t)nb_ * 81);
  const int nwg_max = (nb_ + 63) / 64;
  DevBuf candv(al, sizeof(double) * 2 * nwg_max), candi(al, sizeof(int32_t) * 2 * nwg_max),
      candrow(al, sizeof(double) * 2 * (size_t)nwg_max * kPanel), crow(al, sizeof(double) * 2 * kPanel),
      bar(al, 256);
  // STKKT_COARSE_SPIN_LIMIT lowers the barrier's poll bound (a test forces the
  // time-out path with it)
  const char *spin_env = std::getenv("STKKT_COARSE_SPIN_LIMIT");
  const unsigned spin = spin_env ? (unsigned)std::max(0, std::atoi(spin_env)) : kGjSpinLimit;
  const GjSync gs{candv.as<double>(), candi.as<int32_t>(), candrow.as<double>(), crow.as<double>(),
                  bar.as<unsigned>(), reinterpret_cast<int *>(bar.as<unsigned char>() + 128), spin};
  STKKT_HIP(hipMemsetAsync(status.ptr, 0, sizeof(int), s));
  std::vector<int32_t> hidx((size_t)nb_ * 81), hcidx;
  std::vector<double> hval((size_t)nb_ * 81), hcval;
  const int G = blocks_for(d.N, 128, 1024);
  const dim3 g2(blocks_for(nb_, 256, 64), nb_);
  const LookAhead la;
  for (int k = 0; k < nlev_; ++k) {
    // lower coupling of level k (to level k-1), kept for the application
    int32_t *Lk_idx = Lidx_.as<int32_t>() + (size_t)k * nb_ * 81;
    double *Lk_val = Lval_.as<double>() + (size_t)k * nb_ * 81;
    if (k > 0) hipLaunchKernelGGL(coupling_rows_kernel, dim3(G), dim3(128), 0, s, d, k, -1, Lk_idx, Lk_val);
    // S_k = D_k - L_k E_{k-1}
    fill_zero(S.as<double>(), (long long)nn, s);
    hipLaunchKernelGGL(coupling_rows_kernel, dim3(G), dim3(128), 0, s, d, k, 0, ridx.as<int32_t>(),
                       rval.as<double>());
    hipLaunchKernelGGL(dense_from_rows_kernel, dim3(blocks_for(nb_, 256, 64)), dim3(256), 0, s, nb_,
                       ridx.as<int32_t>(), rval.as<double>(), S.as<double>());
    if (k > 0)
      hipLaunchKernelGGL(schur_update_kernel, g2, dim3(256), 0, s, nb_, Lk_idx, Lk_val, Ed.as<double>(),
                         S.as<double>());
    STKKT_HIP(hipGetLastError());
    // S_k^{-1} (column-major S is the row-major transpose: invert it as is)
    gje_invert(nb_, S.as<double>(), tmp.as<double>(), rows.as<double>(), pan.as<double>(), fcol.as<double>(),
               piv.as<int32_t>(), swp.as<int32_t>(), prow.as<double>(), gs, status.as<int>(), la, s);
    // E_k = S_k^{-1} U_k
    if (k + 1 < nlev_) {
      hipLaunchKernelGGL(coupling_rows_kernel, dim3(G), dim3(128), 0, s, d, k, +1, ridx.as<int32_t>(),
                         rval.as<double>());
      STKKT_HIP(hipMemcpyAsync(hidx.data(), ridx.ptr, sizeof(int32_t) * hidx.size(), hipMemcpyDeviceToHost, s));
      STKKT_HIP(hipMemcpyAsync(hval.data(), rval.ptr, sizeof(double) * hval.size(), hipMemcpyDeviceToHost, s));
      STKKT_HIP(hipStreamSynchronize(s));
      transpose_rows(nb_, hidx, hval, hcidx, hcval);
      STKKT_HIP(hipMemcpyAsync(cidx.ptr, hcidx.data(), sizeof(int32_t) * hcidx.size(), hipMemcpyHostToDevice, s));
      STKKT_HIP(hipMemcpyAsync(cval.ptr, hcval.data(), sizeof(double) * hcval.size(), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(e_from_cols_kernel, g2, dim3(256), 0, s, nb_, cidx.as<int32_t>(), cval.as<double>(),
                         S.as<double>(), Ed.as<double>());
      STKKT_HIP(hipGetLastError());
    }
    // store S_k^{-1} and E_k in the application precision, columns padded to ld_
    const dim3 gp(blocks_for(ld_, 256, 64), nb_);
    if (prec_ == STKKT_F32) {
      hipLaunchKernelGGL(store_padded_kernel<float>, gp, dim3(256), 0, s, nb_, ld_, S.as<double>(),
                         Sinv_.as<float>() + (size_t)k * nld);
      if (k + 1 < nlev_)
        hipLaunchKernelGGL(store_padded_kernel<float>, gp, dim3(256), 0, s, nb_, ld_, Ed.as<double>(),
                           E_.as<float>() + (size_t)k * nld);
    } else {
      hipLaunchKernelGGL(store_padded_kernel<double>, gp, dim3(256), 0, s, nb_, ld_, S.as<double>(),
                         Sinv_.as<double>() + (size_t)k * nld);
      if (k + 1 < nlev_)
        hipLaunchKernelGGL(store_padded_kernel<double>, gp, dim3(256), 0, s, nb_, ld_, Ed.as<double>(),
                           E_.as<double>() + (size_t)k * nld);
    }
    STKKT_HIP(hipGetLastError());
  }
  int st = 0;
  STKKT_HIP(hipMemcpyAsync(&st, status.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
  STKKT_HIP(hipStreamSynchronize(s));   // the setup buffers are released on return
  if (st == 2) throw Error(STKKT_EHIP, "coarse LU: panel elimination barrier timed out");
  if (st) throw Error(STKKT_EBREAKDOWN, "coarse LU: singular Schur complement block");
}

template <typename T>
static void gemv(int nb, int ld, const T *A, const double *x, const double *base, double sign, double *partial,
                 double *out, hipStream_t s) {
  const int nch = (nb + kGvCols - 1) / kGvCols;
  hipLaunchKernelGGL(gemv_partial_kernel<T>, dim3((nb + kGvRows - 1) / kGvRows, nch), dim3(kGvRows), 0, s, nb, ld, A,
                     x, partial);
  hipLaunchKernelGGL(gemv_reduce_kernel, dim3(blocks_for(nb, 64, 4096)), dim3(64), 0, s, nb, nch, partial, base,
                     sign, out);
}

template <typename T> void CoarseLU::solve_t(const double *r, double *x, hipStream_t s) const {
  const size_t nn = (size_t)ld_ * nb_;
  const T *Si = static_cast<const T *>(Sinv_.ptr);
  const T *E = static_cast<const T *>(E_.ptr);
  double *t = t_.as<double>(), *part = partial_.as<double>();
  // forward: y_k = S_k^{-1} (r_k - L_k y_{k-1}), y kept in x
  for (int k = 0; k < nlev_; ++k) {
    const double *rk = r + (size_t)k * nb_;
    const double *yprev = k > 0 ? x + (size_t)(k - 1) * nb_ : nullptr;
    hipLaunchKernelGGL(lower_rhs_kernel, dim3(blocks_for(nb_, 4, 1 << 16)), dim3(256), 0, s, nb_,
                       Lidx_.as<int32_t>() + (size_t)k * nb_ * 81, Lval_.as<double>() + (size_t)k * nb_ * 81, rk,
                       0LL, yprev, 0LL, t, 1, 0);
    gemv<T>(nb_, ld_, Si + (size_t)k * nn, t, nullptr, 1.0, part, x + (size_t)k * nb_, s);
  }
  // backward: x_k = y_k - E_k x_{k+1}
  for (int k = nlev_ - 2; k >= 0; --k)
    gemv<T>(nb_, ld_, E + (size_t)k * nn, x + (size_t)(k + 1) * nb_, x + (size_t)k * nb_, -1.0, part,
            x + (size_t)k * nb_, s);
  STKKT_HIP(hipGetLastError());
}

void CoarseLU::solve(const double *r, double *x, hipStream_t s) const {
  if (prec_ == STKKT_F32) solve_t<float>(r, x, s);
  else solve_t<double>(r, x, s);
}

// out_c = base_c + sign A x_c for q <= 16 right-hand sides given transposed
// (xT, see above); out_c at stride ldo, and transposed into outT
template <typename T>
static void gemm(int nb, int ld, int nsplit, const T *A, int q, const double *xT, const double *base, double sign,
                 double *partial, double *out, long long ldo, double *outT, hipStream_t s) {
  const int steps = (nb + 15) / 16;
  const int csplit = (steps + nsplit - 1) / nsplit * 16;
  const int nch = (nb + csplit - 1) / csplit;
  hipLaunchKernelGGL(gemm_partial_kernel<T>, dim3(ld / kMrRows, nch), dim3(kMrThreads), 0, s, nb, ld, csplit, A, q,
                     xT, partial);
  hipLaunchKernelGGL(gemm_reduce_kernel, dim3(blocks_for(nb, 64, 4096), q), dim3(64), 0, s, nb, ld, q, nch, partial,
                     base, ldo, sign, out, ldo, outT);
}

template <typename T>
void CoarseLU::solve_multi_t(int q, const double *r, long long ldr, double *x, long long ldx, hipStream_t s) const {
  const size_t nn = (size_t)ld_ * nb_;
  const T *Si = static_cast<const T *>(Sinv_.ptr);
  const T *E = static_cast<const T *>(E_.ptr);
  double *tT = mt_.as<double>(), *part = mpartial_.as<double>();
  double *xT[2] = {tT + (size_t)kMrRhs * nb_, tT + (size_t)2 * kMrRhs * nb_};
  for (int c0 = 0; c0 < q; c0 += kMrRhs) {
    const int qq = std::min(kMrRhs, q - c0);
    const double *rg = r + c0 * ldr;
    double *xg = x + c0 * ldx;
    // forward: y_k = S_k^{-1} (r_k - L_k y_{k-1}), y kept in x (the last one also in xT[0])
    for (int k = 0; k < nlev_; ++k) {
      const double *yprev = k > 0 ? xg + (size_t)(k - 1) * nb_ : nullptr;
      hipLaunchKernelGGL(lower_rhs_kernel, dim3(blocks_for(nb_, 4, 1 << 16), qq), dim3(256), 0, s, nb_,
                         Lidx_.as<int32_t>() + (size_t)k * nb_ * 81, Lval_.as<double>() + (size_t)k * nb_ * 81,
                         rg + (size_t)k * nb_, ldr, yprev, ldx, tT, kMrRhs, 1);
      gemm<T>(nb_, ld_, nsplit_, Si + (size_t)k * nn, qq, tT, nullptr, 1.0, part, xg + (size_t)k * nb_, ldx, xT[0],
              s);
    }
    // backward: x_k = y_k - E_k x_{k+1}, x_{k+1} read transposed
    int cur = 0;
    for (int k = nlev_ - 2; k >= 0; --k) {
      gemm<T>(nb_, ld_, nsplit_, E + (size_t)k * nn, qq, xT[cur], xg + (size_t)k * nb_, -1.0, part,
              xg + (size_t)k * nb_, ldx, xT[1 - cur], s);
      cur = 1 - cur;
    }
  }
  STKKT_HIP(hipGetLastError());
}

void CoarseLU::solve_multi(int q, const double *r, long long ldr, double *x, long long ldx, hipStream_t s) const {
  if (q <= 0) return;
  if (prec_ == STKKT_F32) solve_multi_t<float>(q, r, ldr, x, ldx, s);
  else solve_multi_t<double>(q, r, ldr, x, ldx, s);
}

size_t CoarseLU::bytes_per_solve() const {
  const size_t esz = prec_ == STKKT_F32 ? sizeof(float) : sizeof(double);
  return esz * (size_t)nb_ * nb_ * (2 * nlev_ - 1);
}

}  // namespace stkkt
