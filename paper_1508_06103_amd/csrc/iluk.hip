// Space-time RAS with ILU(k), k >= 1: symbolic factorisation (host), the
// numeric factorisation and the two triangular sweeps (device).  Layout and
// ordering are described in iluk.hpp.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdlib>
#include <exception>
#include <queue>
#include <thread>

#include "block33.hpp"
#include "iluk.hpp"
#include "ras.hpp"
#include "stencil.hpp"

namespace stkkt {

namespace {

constexpr int kApplyThreads = 512;
constexpr int kWaves = kApplyThreads / 64;
constexpr int kPhaseChunks = 4;   // 64-row chunks per phase of the sweeps
constexpr size_t kFactorLds = 160 * 1024;   // LDS of one gfx950 workgroup

__host__ __device__ inline void unpack4(uint64_t c, int &x, int &y, int &z, int &t) {
  x = (int)(c & 0xffff);
  y = (int)((c >> 16) & 0xffff);
  z = (int)((c >> 32) & 0xffff);
  t = (int)(c >> 48);
}

// ---------------------------------------------------------------------------
// symbolic level-k factorisation of a box (rows in natural order)
// ---------------------------------------------------------------------------
struct SymRow {
  std::vector<int32_t> col;   // sorted natural columns
  std::vector<int8_t> lev;
};

std::vector<SymRow> symbolic(const int dims[4], int level) {
  const int lx = dims[0], ly = dims[1], lz = dims[2], lt = dims[3];
  const int n = lx * ly * lz * lt;
  std::vector<SymRow> rows(n);
  std::vector<int> lev(n, INT_MAX), stamp(n, -1);
  std::vector<int32_t> touched;
  for (int i = 0; i < n; ++i) {
    const int x = i % lx, y = (i / lx) % ly, z = (i / (lx * ly)) % lz, t = i / (lx * ly * lz);
    touched.clear();
    std::priority_queue<int, std::vector<int>, std::greater<int>> heap;
    for (int dt = -1; dt <= 1; ++dt)
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int a = x + dx, b = y + dy, c = z + dz, d = t + dt;
            if (a < 0 || a >= lx || b < 0 || b >= ly || c < 0 || c >= lz || d < 0 || d >= lt) continue;
            const int j = a + lx * (b + ly * (c + lz * d));
            lev[j] = 0;
            touched.push_back(j);
            if (j < i) heap.push(j);
          }
    while (!heap.empty()) {
      const int k = heap.top();
      heap.pop();
      if (stamp[k] == i) continue;
      stamp[k] = i;
      const int lik = lev[k];
      const SymRow &rk = rows[k];
      for (size_t p = 0; p < rk.col.size(); ++p) {
        const int j = rk.col[p];
        if (j <= k) continue;
        const int cand = lik + rk.lev[p] + 1;
        if (cand > level) continue;
        if (lev[j] == INT_MAX) {
          lev[j] = cand;
          touched.push_back(j);
          if (j < i) heap.push(j);
        } else if (cand < lev[j]) {
          lev[j] = cand;
        }
      }
    }
    std::sort(touched.begin(), touched.end());
    SymRow &ri = rows[i];
    ri.col.reserve(touched.size());
    for (int j : touched) {
      ri.col.push_back(j);
      ri.lev.push_back((int8_t)lev[j]);
      lev[j] = INT_MAX;
    }
  }
  return rows;
}

IlukShapeHost make_iluk_shape(const int dims[4], int level) {
  IlukShapeHost sh;
  for (int d = 0; d < 4; ++d) sh.dims[d] = dims[d];
  const int lx = dims[0], ly = dims[1], lz = dims[2];
  const std::vector<SymRow> rows = symbolic(dims, level);
  const int n = (int)rows.size();
  sh.nrows = n;
  // dependency levels and the level order
  std::vector<int> dl(n, 0);
  int nlev = 0;
  for (int i = 0; i < n; ++i) {
    int m = -1;
    for (int j : rows[i].col) {
      if (j >= i) break;
      m = std::max(m, dl[j]);
    }
    dl[i] = m + 1;
    nlev = std::max(nlev, dl[i] + 1);
  }
  sh.nlev = nlev;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return dl[a] < dl[b]; });
  std::vector<int32_t> pos(n);
  for (int p = 0; p < n; ++p) pos[order[p]] = p;
  sh.coords.resize(n);
  sh.rho.resize(n);
  sh.nL.resize(n);
  sh.nU.resize(n);
  sh.pchunk.resize(n);
  for (int p = 0; p < n; ++p) {
    const int i = order[p];
    const int x = i % lx, y = (i / lx) % ly, z = (i / (lx * ly)) % lz, t = i / (lx * ly * lz);
    sh.coords[p] = (uint64_t)x | ((uint64_t)y << 16) | ((uint64_t)z << 32) | ((uint64_t)t << 48);
    sh.rho[p] = i;
    int nl = 0, nu = 0;
    for (int j : rows[i].col) {
      if (j < i) ++nl;
      else if (j > i) ++nu;
    }
    if (nl > INT16_MAX || nu > INT16_MAX) throw Error(STKKT_EINVAL, "ras_setup: ILU(k) row too long");
    sh.nL[p] = (int16_t)nl;
    sh.nU[p] = (int16_t)nu;
    sh.nblocks += nl + nu + 1;
  }
  // chunks: every level cut into groups of 64 consecutive positions
  sh.lvl_chunk.assign(nlev + 1, 0);
  int64_t foff = 0, coff = 0;
  int p = 0;
  for (int L = 0; L < nlev; ++L) {
    sh.lvl_chunk[L] = (int32_t)sh.chunks.size();
    int end = p;
    while (end < n && dl[order[end]] == L) ++end;
    for (int c0 = p; c0 < end; c0 += 64) {
      IlukChunk ch{};
      ch.pos0 = c0;
      ch.rows = std::min(64, end - c0);
      for (int q = 0; q < ch.rows; ++q) {
        ch.lmax = std::max<int>(ch.lmax, sh.nL[c0 + q]);
        ch.umax = std::max<int>(ch.umax, sh.nU[c0 + q]);
        sh.pchunk[c0 + q] = (int32_t)sh.chunks.size();
      }
      ch.foff = foff;
      ch.coff = coff;
      foff += (int64_t)(ch.lmax + 1 + ch.umax) * 9 * ch.rows;
      coff += (int64_t)(ch.lmax + ch.umax) * ch.rows;
      sh.chunks.push_back(ch);
    }
    p = end;
  }
  sh.lvl_chunk[nlev] = (int32_t)sh.chunks.size();
  if (foff > INT32_MAX * 16LL) throw Error(STKKT_EINVAL, "ras_setup: ILU(k) subdomain too large");
  sh.felems = foff;
  sh.cols.assign((size_t)coff, n);
  for (const IlukChunk &ch : sh.chunks)
    for (int q = 0; q < ch.rows; ++q) {
      const int i = order[ch.pos0 + q];
      int e = 0, u = 0;
      for (int j : rows[i].col) {
        if (j < i) sh.cols[ch.coff + (int64_t)e++ * ch.rows + q] = pos[j];
        else if (j > i) sh.cols[ch.coff + (int64_t)(ch.lmax + u++) * ch.rows + q] = pos[j];
      }
    }
  sh.indptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    sh.indptr[i + 1] = sh.indptr[i] + (int32_t)rows[i].col.size();
    sh.indices.insert(sh.indices.end(), rows[i].col.begin(), rows[i].col.end());
  }
  return sh;
}

// ---------------------------------------------------------------------------
// numeric factorisation: one workgroup per subdomain, one wavefront per row
// (wavefront w of the workgroup takes the rows w, w + waves, ... of a level),
// IKJ order inside a row:
//   for the columns k < i of row i, ascending: L_ik = W_ik inv(U_kk),
//     W_ij -= L_ik U_kj for every j > k of row k that is in row i
//     (the lanes take the entries of row k; each finds its column in row i by
//     binary search),
//   then inv(U_ii).
// The row being factored lives in LDS (its sorted natural columns and its
// blocks); rows of earlier levels are read from W, the FP64 ELL layout.
// ---------------------------------------------------------------------------
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Blocks of a chunk: entry e of the chunk's row q, element v, at
// foff + (e 9 + v) rows + q (L entries, then the diagonal, then U entries).
__device__ inline int64_t lpos(const IlukChunk &ch, int e, int lane) { return ch.foff + (int64_t)e * 9 * ch.rows + lane; }
__device__ inline int64_t dpos(const IlukChunk &ch, int lane) { return ch.foff + (int64_t)ch.lmax * 9 * ch.rows + lane; }
__device__ inline int64_t upos(const IlukChunk &ch, int e, int lane) {
  return ch.foff + (int64_t)(ch.lmax + 1 + e) * 9 * ch.rows + lane;
}

__device__ inline void block_of(const OpDev &op, const SubInfo &sd, uint64_t ci, uint64_t cj, double *blk) {
  int xi, yi, zi, ti, xj, yj, zj, tj;
  unpack4(ci, xi, yi, zi, ti);
  unpack4(cj, xj, yj, zj, tj);
  const int dx = xj - xi, dy = yj - yi, dz = zj - zi, dt = tj - ti;
  if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1 && abs(dt) <= 1) {
    kkt_block(op, sd.org[0] + xi, sd.org[1] + yi, sd.org[2] + zi, sd.org[3] + ti, dx, dy, dz, dt, blk);
  } else {
    for (int e = 0; e < 9; ++e) blk[e] = 0.0;   // fill entry: zero in F_h
  }
}

__global__ void __launch_bounds__(256) iluk_factor_kernel(OpDev op, const SubInfo *__restrict__ subs, int sub0,
                                                          const IlukShapeDev *__restrict__ shapes,
                                                          const IlukChunk *__restrict__ chunks,
                                                          const int32_t *__restrict__ lvl_chunk,
                                                          const uint64_t *__restrict__ coords,
                                                          const int32_t *__restrict__ rho,
                                                          const int32_t *__restrict__ pchunk,
                                                          const int16_t *__restrict__ nL,
                                                          const int16_t *__restrict__ nU,
                                                          const int32_t *__restrict__ cols, int maxlen, double *W,
                                                          int *status) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int waves = (int)(blockDim.x >> 6);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = (int)__lane_id();
  double *rowb = reinterpret_cast<double *>(smem) + (size_t)wave * maxlen * 9;
  int32_t *rcol = reinterpret_cast<int32_t *>(smem + sizeof(double) * (size_t)waves * maxlen * 9) + (size_t)wave * maxlen;
  const SubInfo sd = subs[sub0 + blockIdx.x];
  const IlukShapeDev sh = shapes[sd.shape];
  double *Wb = W + sd.wbase;
  const IlukChunk *chs = chunks + sh.chunk_off;
  const uint64_t *crd = coords + sh.pos_off;
  const int32_t *rh = rho + sh.pos_off, *pc = pchunk + sh.pos_off, *cl = cols + sh.col_off;
  const int16_t *nl = nL + sh.pos_off, *nu = nU + sh.pos_off;
  for (int L = 0; L < sh.nlev; ++L) {
    const int c0 = lvl_chunk[sh.lvl_off + L], c1 = lvl_chunk[sh.lvl_off + L + 1];
    const int p0 = chs[c0].pos0, p1 = chs[c1 - 1].pos0 + chs[c1 - 1].rows;
    for (int pi = p0 + wave; pi < p1; pi += waves) {
      const IlukChunk ch = chs[pc[pi]];
      const int q = pi - ch.pos0, rs = ch.rows;
      const int ni = nl[pi], mi = nu[pi], len = ni + 1 + mi;
      const uint64_t ci = crd[pi];
      // natural columns (L entries, the diagonal, U entries: ascending) and A's blocks
      for (int t = lane; t < len; t += 64) {
        const int pj = t < ni ? cl[ch.coff + (int64_t)t * rs + q]
                              : t == ni ? pi : cl[ch.coff + (int64_t)(ch.lmax + t - ni - 1) * rs + q];
        rcol[t] = rh[pj];
        double blk[9];
        block_of(op, sd, ci, crd[pj], blk);
        for (int v = 0; v < 9; ++v) rowb[9 * t + v] = blk[v];
      }
      wave_sync();
      for (int e = 0; e < ni; ++e) {
        const int pk = cl[ch.coff + (int64_t)e * rs + q];
        const IlukChunk chk = chs[pc[pk]];
        const int qk = pk - chk.pos0, rk = chk.rows, mk = nu[pk];
        double a[9], d[9], l[9];
        const double *dk = Wb + dpos(chk, qk);
        for (int v = 0; v < 9; ++v) {
          a[v] = rowb[9 * e + v];
          d[v] = dk[(int64_t)v * rk];
        }
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) l[3 * r + c] = a[3 * r] * d[c] + a[3 * r + 1] * d[3 + c] + a[3 * r + 2] * d[6 + c];
        wave_sync();
        if (lane == 0)
          for (int v = 0; v < 9; ++v) rowb[9 * e + v] = l[v];
        for (int f = lane; f < mk; f += 64) {
          const int pj = cl[chk.coff + (int64_t)(chk.lmax + f) * rk + qk];
          const int rj = rh[pj];
          int lo = e + 1, hi = len;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (rcol[mid] < rj) lo = mid + 1;
            else hi = mid;
          }
          if (lo < len && rcol[lo] == rj) {
            const double *u = Wb + upos(chk, f, qk);
            double ub[9];
            for (int v = 0; v < 9; ++v) ub[v] = u[(int64_t)v * rk];
            double *w = rowb + 9 * lo;
            for (int r = 0; r < 3; ++r)
              for (int c = 0; c < 3; ++c) {
                const double sm = l[3 * r] * ub[c] + l[3 * r + 1] * ub[3 + c] + l[3 * r + 2] * ub[6 + c];
                w[3 * r + c] -= sm;
              }
          }
        }
        wave_sync();
      }
      if (lane == 0) {
        double dd[9], inv[9];
        for (int v = 0; v < 9; ++v) dd[v] = rowb[9 * ni + v];
        bool ok;
        inv33_pivot(dd, inv, ok);
        if (!ok) {
          atomicMax(status, 1);
          for (int v = 0; v < 9; ++v) inv[v] = 0.0;
        }
        for (int v = 0; v < 9; ++v) rowb[9 * ni + v] = inv[v];
      }
      wave_sync();
      for (int t = lane; t < len; t += 64) {
        const int64_t at = t < ni ? lpos(ch, t, q) : t == ni ? dpos(ch, q) : upos(ch, t - ni - 1, q);
        for (int v = 0; v < 9; ++v) Wb[at + (int64_t)v * rs] = rowb[9 * t + v];
      }
      wave_sync();
    }
    __syncthreads();   // the next level reads these rows from W
  }
}

__global__ void to_float_kernel(const double *__restrict__ a, float *__restrict__ b, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

// ---------------------------------------------------------------------------
// apply: one workgroup of 8 wavefronts per subdomain.  A level is swept in
// phases of up to 4 chunks; wavefront w takes the entries e = w, w + 8, ... of
// every chunk of the phase (lane = row), partial sums meet in LDS, and after a
// barrier one thread per row finishes it: y = r - sum (forward, y into the
// local vector) or z = inv(U_ii)(y - sum) (backward, z over y in the local
// vector, owned rows to the output).
// ---------------------------------------------------------------------------
template <typename T, bool kFwd>
__device__ inline void iluk_sweep(const OpDev &op, const SubInfo &sd, const IlukShapeDev &sh,
                                  const IlukChunk *__restrict__ chs, const int32_t *__restrict__ lvc,
                                  const uint64_t *__restrict__ crd, const int16_t *__restrict__ cnt,
                                  const int32_t *__restrict__ cl, const T *__restrict__ Fb, T *__restrict__ Yb,
                                  const double *__restrict__ r, double *__restrict__ z,
                                  T (*part)[kPhaseChunks * 64][3]) {
  const int lane = (int)__lane_id();
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tq = (int)threadIdx.x;
  for (int li = 0; li < sh.nlev; ++li) {
    const int L = kFwd ? li : sh.nlev - 1 - li;
    const int c0 = lvc[L], c1 = lvc[L + 1];
    for (int cp = c0; cp < c1; cp += kPhaseChunks) {
      const int np = min(kPhaseChunks, c1 - cp);
      for (int cc = 0; cc < np; ++cc) {
        const IlukChunk ch = load_uniform(chs + cp + cc);
        // a chunk of rp <= 32 rows (rp a power of two >= its rows) is swept by
        // 64 / rp lane groups that take alternate entries
        const int rp = ch.rows > 32 ? 64 : ch.rows > 16 ? 32 : ch.rows > 8 ? 16 : 8;
        const int grp = lane / rp, ngrp = 64 / rp, row = lane % rp;
        const bool valid = row < ch.rows;
        const int n = valid ? (int)cnt[ch.pos0 + row] : 0;
        const int base = kFwd ? 0 : ch.lmax;                       // column block of the entries
        const int rs = ch.rows;
        const int64_t fo = ch.foff + (kFwd ? 0 : (int64_t)(ch.lmax + 1) * 9 * rs);
        const int emax = kFwd ? ch.lmax : ch.umax;
        const int estep = kWaves * ngrp;
        T a0 = 0, a1 = 0, a2 = 0;
        // four entries per step, all their loads issued before the products
        for (int e0 = wave + kWaves * grp; e0 < emax; e0 += 4 * estep) {
          int col[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * estep;
            col[u] = e < n ? cl[ch.coff + (int64_t)(base + e) * rs + row] : -1;
          }
          T f[4][9], yv[4][3];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * estep;
            const bool has = col[u] >= 0;
            const T *fp = Fb + fo + (int64_t)(has ? e : 0) * 9 * rs + row;
            const T *yp = Yb + 3 * (int64_t)(has ? col[u] : 0);
#pragma unroll
            for (int v = 0; v < 9; ++v) f[u][v] = has ? fp[(int64_t)v * rs] : (T)0;
#pragma unroll
            for (int k = 0; k < 3; ++k) yv[u][k] = has ? yp[k] : (T)0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            a0 += f[u][0] * yv[u][0] + f[u][1] * yv[u][1] + f[u][2] * yv[u][2];
            a1 += f[u][3] * yv[u][0] + f[u][4] * yv[u][1] + f[u][5] * yv[u][2];
            a2 += f[u][6] * yv[u][0] + f[u][7] * yv[u][1] + f[u][8] * yv[u][2];
          }
        }
        part[wave][cc * 64 + lane][0] = a0;
        part[wave][cc * 64 + lane][1] = a1;
        part[wave][cc * 64 + lane][2] = a2;
      }
      __syncthreads();
      if (tq < np * 64) {
        const IlukChunk ch = chs[cp + (tq >> 6)];
        const int q = tq & 63;
        if (q < ch.rows) {
          const int pi = ch.pos0 + q;
          const int rp = ch.rows > 32 ? 64 : ch.rows > 16 ? 32 : ch.rows > 8 ? 16 : 8;
          const int base = tq & ~63;
          T s[3];
          for (int k = 0; k < 3; ++k) {
            T acc = 0;
            for (int w = 0; w < kWaves; ++w)
              for (int g = 0; g < 64; g += rp) acc += part[w][base + g + q][k];
            s[k] = acc;
          }
          int x, y, zc, t;
          unpack4(crd[pi], x, y, zc, t);
          const long long node = (sd.org[0] + x) +
                                 (long long)op.nn[0] * ((sd.org[1] + y) + (long long)op.nn[1] * (sd.org[2] + zc));
          const long long gi = 3 * ((long long)(sd.org[3] + t) * op.N + node);
          T *yr = Yb + 3 * (int64_t)pi;
          if (kFwd) {
            for (int k = 0; k < 3; ++k) yr[k] = (T)r[gi + k] - s[k];
          } else {
            const int rs = ch.rows;
            const T *d = Fb + ch.foff + (int64_t)ch.lmax * 9 * rs + q;
            T v[3], o[3];
            for (int k = 0; k < 3; ++k) v[k] = yr[k] - s[k];
            for (int k = 0; k < 3; ++k)
              o[k] = d[(3 * k) * rs] * v[0] + d[(3 * k + 1) * rs] * v[1] + d[(3 * k + 2) * rs] * v[2];
            for (int k = 0; k < 3; ++k) yr[k] = o[k];
            const bool owned = x >= sd.olo[0] && x < sd.ohi[0] && y >= sd.olo[1] && y < sd.ohi[1] &&
                               zc >= sd.olo[2] && zc < sd.ohi[2] && t >= sd.olo[3] && t < sd.ohi[3];
            if (owned)
              for (int k = 0; k < 3; ++k) z[gi + k] = (double)o[k];
          }
        }
      }
      __syncthreads();
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kApplyThreads) iluk_apply_kernel(
    OpDev op, const SubInfo *__restrict__ subs, const int32_t *__restrict__ order,
    const IlukShapeDev *__restrict__ shapes, const IlukChunk *__restrict__ chunks,
    const int32_t *__restrict__ lvl_chunk, const uint64_t *__restrict__ coords, const int16_t *__restrict__ nL,
    const int16_t *__restrict__ nU, const int32_t *__restrict__ cols, const T *__restrict__ F, T *__restrict__ Y,
    const double *__restrict__ r, double *__restrict__ z) {
  __shared__ T part[kWaves][kPhaseChunks * 64][3];
  const SubInfo sd = load_uniform(subs + as_const(order)[blockIdx.x]);
  const IlukShapeDev sh = load_uniform(shapes + sd.shape);
  const IlukChunk *chs = chunks + sh.chunk_off;
  const int32_t *lvc = lvl_chunk + sh.lvl_off;
  const uint64_t *crd = coords + sh.pos_off;
  const int32_t *cl = cols + sh.col_off;
  const T *Fb = F + sd.fbase;
  T *Yb = Y + sd.sbase;
  iluk_sweep<T, true>(op, sd, sh, chs, lvc, crd, nL + sh.pos_off, cl, Fb, Yb, r, z, part);
  iluk_sweep<T, false>(op, sd, sh, chs, lvc, crd, nU + sh.pos_off, cl, Fb, Yb, r, z, part);
}

template <class V> void upload_vec(const Allocator *al, DevBuf &buf, const std::vector<V> &host, hipStream_t s) {
  buf = DevBuf(al, std::max<size_t>(sizeof(V) * host.size(), 256));
  if (!host.empty())
    STKKT_HIP(hipMemcpyAsync(buf.ptr, host.data(), sizeof(V) * host.size(), hipMemcpyHostToDevice, s));
}

}  // namespace

void iluk_create(ras *R, const kkt_op *op, hipStream_t s) {
  auto K = std::make_shared<IlukData>();
  K->level = R->params.ilu_level;
  // the symbolic factorisations of the distinct box shapes are independent: host threads
  const int nsh = (int)R->shapes.size();
  K->shapes.resize(nsh);
  std::vector<std::exception_ptr> err(nsh);
  std::atomic<int> next{0};
  const int nthr = std::max(1, std::min(nsh, (int)std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int w = 0; w < nthr; ++w)
    pool.emplace_back([&] {
      for (int i = next++; i < nsh; i = next++) {
        try {
          K->shapes[i] = make_iluk_shape(R->shapes[i].dims, K->level);
        } catch (...) {
          err[i] = std::current_exception();
        }
      }
    });
  for (auto &t : pool) t.join();
  for (auto &e : err)
    if (e) std::rethrow_exception(e);
  // subdomain offsets in the ELL layout
  int64_t fb = 0, sb = 0;
  for (SubInfo &si : R->subs) {
    const IlukShapeHost &sh = K->shapes[si.shape];
    si.fbase = fb;
    si.sbase = sb;
    fb += sh.felems;
    sb += 3LL * (sh.nrows + 1);
    K->total_blocks += sh.nblocks;
  }
  K->factor_elems = fb;
  K->scratch_elems = sb;
  R->total_blocks = K->total_blocks;
  R->factor_elems = fb;
  R->scratch_elems = sb;
  // concatenated shape tables
  std::vector<IlukShapeDev> sdev;
  std::vector<IlukChunk> chunks;
  std::vector<int32_t> lvl, rho, pch, cols;
  std::vector<uint64_t> crd;
  std::vector<int16_t> nl, nu;
  for (const IlukShapeHost &sh : K->shapes) {
    IlukShapeDev d{};
    for (int k = 0; k < 4; ++k) d.dims[k] = sh.dims[k];
    d.nrows = sh.nrows;
    d.nlev = sh.nlev;
    d.nchunk = (int32_t)sh.chunks.size();
    d.chunk_off = (int64_t)chunks.size();
    d.lvl_off = (int64_t)lvl.size();
    d.pos_off = (int64_t)crd.size();
    d.col_off = (int64_t)cols.size();
    sdev.push_back(d);
    chunks.insert(chunks.end(), sh.chunks.begin(), sh.chunks.end());
    lvl.insert(lvl.end(), sh.lvl_chunk.begin(), sh.lvl_chunk.end());
    crd.insert(crd.end(), sh.coords.begin(), sh.coords.end());
    rho.insert(rho.end(), sh.rho.begin(), sh.rho.end());
    pch.insert(pch.end(), sh.pchunk.begin(), sh.pchunk.end());
    nl.insert(nl.end(), sh.nL.begin(), sh.nL.end());
    nu.insert(nu.end(), sh.nU.begin(), sh.nU.end());
    cols.insert(cols.end(), sh.cols.begin(), sh.cols.end());
  }
  const Allocator *al = &R->al;
  upload_vec(al, K->d_shapes, sdev, s);
  upload_vec(al, K->d_chunks, chunks, s);
  upload_vec(al, K->d_lvl, lvl, s);
  upload_vec(al, K->d_coords, crd, s);
  upload_vec(al, K->d_rho, rho, s);
  upload_vec(al, K->d_pchunk, pch, s);
  upload_vec(al, K->d_nL, nl, s);
  upload_vec(al, K->d_nU, nu, s);
  upload_vec(al, K->d_cols, cols, s);
  upload_vec(al, R->d_subs, R->subs, s);
  // launch order: largest factor first
  std::vector<int32_t> order(R->nsub);
  for (int i = 0; i < R->nsub; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return K->shapes[R->subs[a].shape].felems > K->shapes[R->subs[b].shape].felems;
  });
  upload_vec(al, R->d_order, order, s);
  const bool f32 = R->params.precision == STKKT_F32;
  const size_t esz = f32 ? sizeof(float) : sizeof(double);
  DevBuf d_status(al, 256);
  STKKT_HIP(hipMemsetAsync(d_status.ptr, 0, sizeof(int), s));
  K->factors = DevBuf(al, esz * ((size_t)fb + 1));
  // LDS of the factorisation: per wavefront, the longest row's blocks and columns
  int maxlen = 1;
  for (const IlukShapeHost &sh : K->shapes)
    for (int p = 0; p < sh.nrows; ++p) maxlen = std::max(maxlen, sh.nL[p] + sh.nU[p] + 1);
  const size_t per_wave = (size_t)maxlen * (9 * sizeof(double) + sizeof(int32_t));
  const int fwaves = (int)std::min<size_t>(4, kFactorLds / per_wave);
  STKKT_REQUIRE(fwaves >= 1, "ras_setup: ILU(k) rows too long for the factorisation's LDS");
  STKKT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&iluk_factor_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFactorLds));
  auto factor = [&](int first, int count, double *W) {
    hipLaunchKernelGGL(iluk_factor_kernel, dim3(count), dim3(64 * fwaves), per_wave * fwaves, s, op->d,
                       R->d_subs.as<SubInfo>(), first, K->d_shapes.as<IlukShapeDev>(), K->d_chunks.as<IlukChunk>(),
                       K->d_lvl.as<int32_t>(), K->d_coords.as<uint64_t>(), K->d_rho.as<int32_t>(),
                       K->d_pchunk.as<int32_t>(), K->d_nL.as<int16_t>(), K->d_nU.as<int16_t>(),
                       K->d_cols.as<int32_t>(), maxlen, W, d_status.as<int>());
    STKKT_HIP(hipGetLastError());
  };
  if (!f32) {
    // FP64: factor in place
    for (SubInfo &si : R->subs) si.wbase = si.fbase;
    STKKT_HIP(hipMemcpyAsync(R->d_subs.ptr, R->subs.data(), sizeof(SubInfo) * R->subs.size(),
                             hipMemcpyHostToDevice, s));
    factor(0, R->nsub, K->factors.as<double>());
  } else {
    // FP32: subdomains factored in FP64 in batches that fit a workspace budget, then narrowed
    size_t budget = (size_t)64 << 30;
    if (const char *e = getenv("STKKT_SETUP_WORK_GB")) budget = (size_t)(atof(e) * (double)(1ull << 30));
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) budget = std::min(budget, free_b / 2);
    int first = 0;
    while (first < R->nsub) {
      size_t used = 0;
      int last = first;
      while (last < R->nsub) {
        const size_t need = sizeof(double) * (size_t)K->shapes[R->subs[last].shape].felems;
        if (last > first && used + need > budget) break;
        R->subs[last].wbase = (int64_t)(used / sizeof(double));
        used += need;
        ++last;
      }
      STKKT_HIP(hipMemcpyAsync(R->d_subs.ptr, R->subs.data(), sizeof(SubInfo) * R->subs.size(),
                               hipMemcpyHostToDevice, s));
      DevBuf work(al, used + sizeof(double));
      factor(first, last - first, work.as<double>());
      // the batch's subdomains are contiguous in both layouts
      const int64_t n0 = R->subs[first].fbase;
      const int64_t n1 = last < R->nsub ? R->subs[last].fbase : fb;
      hipLaunchKernelGGL(to_float_kernel, dim3(blocks_for(n1 - n0, 256, 16384)), dim3(256), 0, s, work.as<double>(),
                         K->factors.as<float>() + n0, (long long)(n1 - n0));
      STKKT_HIP(hipGetLastError());
      STKKT_HIP(hipStreamSynchronize(s));   // the workspace is released at the end of this scope
      first = last;
    }
  }
  K->scratch = DevBuf(al, esz * ((size_t)sb + 4));
  STKKT_HIP(hipMemsetAsync(K->scratch.ptr, 0, esz * ((size_t)sb + 4), s));
  int status = 0;
  STKKT_HIP(hipMemcpyAsync(&status, d_status.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
  STKKT_HIP(hipStreamSynchronize(s));
  if (status != 0) throw Error(STKKT_EBREAKDOWN, "ras_setup: singular 3x3 pivot block in ILU(k)");
  R->iluk = K;
}

size_t iluk_local_bytes(const ras *R) {
  const size_t esz = R->params.precision == STKKT_F32 ? sizeof(float) : sizeof(double);
  return esz * ((size_t)R->iluk->scratch_elems + 4);
}

void iluk_apply(const ras *R, const double *r, double *z, void *local, hipStream_t s) {
  const IlukData &K = *R->iluk;
  if (R->params.precision == STKKT_F32) {
    float *Y = local ? static_cast<float *>(local) : K.scratch.as<float>();
    hipLaunchKernelGGL(iluk_apply_kernel<float>, dim3(R->nsub), dim3(kApplyThreads), 0, s, R->d,
                       R->d_subs.as<SubInfo>(), R->d_order.as<int32_t>(), K.d_shapes.as<IlukShapeDev>(),
                       K.d_chunks.as<IlukChunk>(), K.d_lvl.as<int32_t>(), K.d_coords.as<uint64_t>(),
                       K.d_nL.as<int16_t>(), K.d_nU.as<int16_t>(), K.d_cols.as<int32_t>(), K.factors.as<float>(),
                       Y, r, z);
  } else {
    double *Y = local ? static_cast<double *>(local) : K.scratch.as<double>();
    hipLaunchKernelGGL(iluk_apply_kernel<double>, dim3(R->nsub), dim3(kApplyThreads), 0, s, R->d,
                       R->d_subs.as<SubInfo>(), R->d_order.as<int32_t>(), K.d_shapes.as<IlukShapeDev>(),
                       K.d_chunks.as<IlukChunk>(), K.d_lvl.as<int32_t>(), K.d_coords.as<uint64_t>(),
                       K.d_nL.as<int16_t>(), K.d_nU.as<int16_t>(), K.d_cols.as<int32_t>(), K.factors.as<double>(),
                       Y, r, z);
  }
  STKKT_HIP(hipGetLastError());
}

int64_t iluk_subdomain_blocks(const ras *R, int sub) {
  return R->iluk->shapes[R->subs[sub].shape].nblocks;
}

void iluk_export_csr(const ras *R, int sub, int32_t *indptr, int32_t *indices, double *blocks) {
  const IlukData &K = *R->iluk;
  const SubInfo &sd = R->subs[sub];
  const IlukShapeHost &sh = K.shapes[sd.shape];
  std::vector<double> buf((size_t)sh.felems);
  if (R->params.precision == STKKT_F32) {
    std::vector<float> tmp((size_t)sh.felems);
    STKKT_HIP(hipMemcpy(tmp.data(), K.factors.as<float>() + sd.fbase, sizeof(float) * tmp.size(),
                        hipMemcpyDeviceToHost));
    for (size_t i = 0; i < tmp.size(); ++i) buf[i] = tmp[i];
  } else {
    STKKT_HIP(hipMemcpy(buf.data(), K.factors.as<double>() + sd.fbase, sizeof(double) * buf.size(),
                        hipMemcpyDeviceToHost));
  }
  const int n = sh.nrows;
  std::copy(sh.indptr.begin(), sh.indptr.end(), indptr);
  std::copy(sh.indices.begin(), sh.indices.end(), indices);
  std::vector<int32_t> pos(n);
  for (int p = 0; p < n; ++p) pos[sh.rho[p]] = p;
  for (int i = 0; i < n; ++i) {
    const int p = pos[i];
    const IlukChunk &ch = sh.chunks[sh.pchunk[p]];
    const int q = p - ch.pos0;
    int e = 0, u = 0;
    for (int k = sh.indptr[i]; k < sh.indptr[i + 1]; ++k) {
      const int j = sh.indices[k];
      int64_t at;
      const int rs = ch.rows;
      if (j < i) at = ch.foff + (int64_t)e++ * 9 * rs + q;
      else if (j == i) at = ch.foff + (int64_t)ch.lmax * 9 * rs + q;
      else at = ch.foff + (int64_t)(ch.lmax + 1 + u++) * 9 * rs + q;
      for (int v = 0; v < 9; ++v) blocks[9 * (int64_t)k + v] = buf[at + (int64_t)v * rs];
    }
  }
}

}  // namespace stkkt
