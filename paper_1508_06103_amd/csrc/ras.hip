// One-level space-time restricted additive Schwarz with 3x3 point-block
// ILU(0) subdomain solves (Section 3.2 of the paper: overlapping space-time
// decomposition, subdomain matrices taken from F_h on the extended boxes,
// restricted prolongation of the owned part; Section 4: ILU(0)).
//
// Factor storage ("chunk-major SoA"): the rows of a subdomain are grouped by
// wavefront level L = x + 2y + 4z + 8t (every lower neighbour of the 81-point
// stencil has a smaller level) and, inside a level, in 64-row chunks.  For
// every (level, chunk, stencil slot s) with s = (dx+1) + 3(dy+1) + 9(dz+1) +
// 27(dt+1) -- s < 40 the L blocks, s = 40 inv(U_rr), s > 40 the U blocks --
// the blocks of the chunk's rows that have neighbour s inside the box are
// stored entry-major: value(e, k) at off9 + e * cnt + k, k being the rank of
// the row among those rows.  A wavefront of 64 rows reads each entry of a slot
// with one coalesced load, the five slots it owns for a chunk form one
// contiguous stretch, and no padding is stored for neighbours outside the box.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <memory>
#include <tuple>

#include "block33.hpp"
#include "iluk.hpp"
#include "ras.hpp"
#include "stencil.hpp"

namespace stkkt {

namespace {

constexpr int kApplyThreads = 512;
constexpr size_t kRingLdsLimit = 160 * 1024;   // LDS of one gfx950 workgroup

__host__ __device__ inline void slot_off(int s, int &dx, int &dy, int &dz, int &dt) {
  dx = s % 3 - 1;
  dy = (s / 3) % 3 - 1;
  dz = (s / 9) % 3 - 1;
  dt = s / 27 - 1;
}

__host__ __device__ inline bool inside(int x, int y, int z, int t, const int32_t *dims) {
  return x >= 0 && x < dims[0] && y >= 0 && y < dims[1] && z >= 0 && z < dims[2] && t >= 0 && t < dims[3];
}

__host__ __device__ inline void unpack(uint64_t c, int &x, int &y, int &z, int &t) {
  x = (int)(c & 0xffff);
  y = (int)((c >> 16) & 0xffff);
  z = (int)((c >> 32) & 0xffff);
  t = (int)(c >> 48);
}

// Place of entry e (row-major 3x3) of block k in a group of cnt blocks: the
// entries 0-3 of all blocks as consecutive quads, then entries 4-7 as quads,
// then entry 8.  Groups start on a multiple of kGroupAlign elements, so a
// lane reads its block with two 16-byte loads plus one (FP32) or four plus
// one (FP64).
constexpr int kGroupAlign = 4;
__host__ __device__ inline int64_t blk_pos(int e, int64_t k, int64_t cnt) {
  return e < 4 ? 4 * k + e : e < 8 ? 4 * cnt + 4 * k + (e - 4) : 8 * cnt + k;
}

// Crout-ordered elimination: the entry of row i at slot st is
//   A_it - sum_k L_ik U_kt  over lower neighbours k of i with t an upper
// neighbour of k (slot pair (sk, su) with off(sk) + off(su) = off(st), sk < 40
// < su, sk < st), in ascending k; then L_it = (...) inv(U_tt) for st < 40.
// This is the IKJ ILU(0) of the paper's subdomain solver reordered by entry.
void build_pairs(std::vector<int16_t> &start, std::vector<uint8_t> &pairs) {
  start.assign(82, 0);
  pairs.clear();
  for (int st = 0; st < 81; ++st) {
    start[st] = (int16_t)(pairs.size() / 2);
    int tx, ty, tz, tt;
    slot_off(st, tx, ty, tz, tt);
    for (int sk = 0; sk < 40 && sk < st; ++sk) {
      int kx, ky, kz, kt;
      slot_off(sk, kx, ky, kz, kt);
      const int ux = tx - kx, uy = ty - ky, uz = tz - kz, ut = tt - kt;
      if (ux < -1 || ux > 1 || uy < -1 || uy > 1 || uz < -1 || uz > 1 || ut < -1 || ut > 1) continue;
      const int su = (ux + 1) + 3 * (uy + 1) + 9 * (uz + 1) + 27 * (ut + 1);
      if (su <= 40) continue;
      pairs.push_back((uint8_t)sk);
      pairs.push_back((uint8_t)su);
    }
  }
  start[81] = (int16_t)(pairs.size() / 2);
}

ShapeHost make_shape(const int dims[4]) {
  ShapeHost sh;
  for (int d = 0; d < 4; ++d) sh.dims[d] = dims[d];
  const int lx = dims[0], ly = dims[1], lz = dims[2], lt = dims[3];
  sh.vol = lx * ly * lz * lt;
  sh.nlev = (lx - 1) + 2 * (ly - 1) + 4 * (lz - 1) + 8 * (lt - 1) + 1;
  std::vector<std::vector<uint64_t>> lev(sh.nlev);
  for (int t = 0; t < lt; ++t)
    for (int z = 0; z < lz; ++z)
      for (int y = 0; y < ly; ++y)
        for (int x = 0; x < lx; ++x)
          lev[x + 2 * y + 4 * z + 8 * t].push_back((uint64_t)x | ((uint64_t)y << 16) | ((uint64_t)z << 32) |
                                                   ((uint64_t)t << 48));
  sh.lvl_start.resize(sh.nlev + 1);
  sh.lvl_start[0] = 0;
  for (int L = 0; L < sh.nlev; ++L) {
    sh.lvl_start[L + 1] = sh.lvl_start[L] + (int32_t)lev[L].size();
    sh.rmax = std::max<int>(sh.rmax, (int)lev[L].size());
    for (auto c : lev[L]) sh.coords.push_back(c);
  }
  sh.nchunk = (sh.rmax + 63) / 64;
  const int32_t d32[4] = {lx, ly, lz, lt};
  // chunk-major factor layout: for level L, 64-row chunk c of the level, slot s,
  // the group of the blocks of the chunk's rows that have neighbour s (block k
  // = rank of its row among them), entry e of block k at ctab.off + blk_pos(e, k, ctab.cnt)
  if ((size_t)sh.nlev * sh.nchunk * 81 * 2 > (size_t)INT32_MAX) throw Error(STKKT_EINVAL, "ras_setup: subdomain too large");
  sh.ctab.assign((size_t)sh.nlev * sh.nchunk * 81 * 2, 0);
  int64_t off = 0;
  for (int L = 0; L < sh.nlev; ++L) {
    const int r0 = sh.lvl_start[L], R = sh.lvl_start[L + 1] - r0;
    for (int c = 0; c * 64 < R; ++c)
      for (int s = 0; s < 81; ++s) {
        int dx, dy, dz, dt;
        slot_off(s, dx, dy, dz, dt);
        int cnt = 0;
        for (int q = c * 64; q < std::min(R, c * 64 + 64); ++q) {
          int x, y, z, t;
          unpack(sh.coords[r0 + q], x, y, z, t);
          if (inside(x + dx, y + dy, z + dz, t + dt, d32)) ++cnt;
        }
        const int64_t len = (9 * (int64_t)cnt + kGroupAlign - 1) / kGroupAlign * kGroupAlign;
        if (off + len > INT32_MAX) throw Error(STKKT_EINVAL, "ras_setup: subdomain too large");
        const size_t i = (((size_t)L * sh.nchunk + c) * 81 + s) * 2;
        sh.ctab[i] = (int32_t)off;
        sh.ctab[i + 1] = cnt;
        off += len;
        sh.nblocks += cnt;
      }
  }
  sh.felems = off;
  // tzpref[L][t][z]: rows of level L in earlier (t, z) groups (rows of a level
  // are ordered by (t, z, y), x being implied by the level)
  sh.tzpref.assign((size_t)sh.nlev * lt * lz, 0);
  for (int L = 0; L < sh.nlev; ++L) {
    int cnt = 0;
    for (int t = 0; t < lt; ++t)
      for (int z = 0; z < lz; ++z) {
        sh.tzpref[((size_t)L * lt + t) * lz + z] = cnt;
        for (int y = 0; y < ly; ++y) {
          const int x = L - 8 * t - 4 * z - 2 * y;
          if (x >= 0 && x < lx) ++cnt;
        }
      }
    if (cnt != sh.lvl_start[L + 1] - sh.lvl_start[L]) throw Error(STKKT_EINVAL, "ras_setup: level table mismatch");
  }
  return sh;
}

// --------------------------------------------------------------------------
// setup: subdomain matrix from the operator formula, then ILU(0), one
// workgroup per subdomain, rows of a level in parallel (one thread per row).
// W holds the subdomain's rows padded to 81 blocks: W[rho][s][e].
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) factor_kernel(OpDev op, const SubInfo *__restrict__ subs,
                                                     const ShapeInfo *__restrict__ shapes,
                                                     const int32_t *__restrict__ lvl_start,
                                                     const uint64_t *__restrict__ coords,
                                                     const int16_t *__restrict__ pstart,
                                                     const uint8_t *__restrict__ pairs, int sub0, double *W,
                                                     int *status) {
  const SubInfo sd = subs[sub0 + blockIdx.x];
  const ShapeInfo sh = shapes[sd.shape];
  const int lx = sh.dims[0], ly = sh.dims[1], lz = sh.dims[2];
  double *Wb = W + sd.wbase;
  for (int L = 0; L < sh.nlev; ++L) {
    const int r0 = lvl_start[sh.lvl_off + L], r1 = lvl_start[sh.lvl_off + L + 1];
    for (int q = r0 + (int)threadIdx.x; q < r1; q += blockDim.x) {
      int x, y, z, t;
      unpack(coords[sh.coord_off + q], x, y, z, t);
      const long long rho = x + (long long)lx * (y + (long long)ly * (z + (long long)lz * t));
      double *Wr = Wb + rho * 729;
      const int gx = sd.org[0] + x, gy = sd.org[1] + y, gz = sd.org[2] + z, gn = sd.org[3] + t;
      for (int s = 0; s < 81; ++s) {
        int dx, dy, dz, dt;
        slot_off(s, dx, dy, dz, dt);
        double blk[9];
        if (inside(x + dx, y + dy, z + dz, t + dt, sh.dims)) {
          kkt_block(op, gx, gy, gz, gn, dx, dy, dz, dt, blk);
        } else {
          for (int e = 0; e < 9; ++e) blk[e] = 0.0;
        }
        for (int e = 0; e < 9; ++e) Wr[9 * s + e] = blk[e];
      }
      for (int st = 0; st < 81; ++st) {
        int tx, ty, tz, tt;
        slot_off(st, tx, ty, tz, tt);
        if (!inside(x + tx, y + ty, z + tz, t + tt, sh.dims)) continue;
        double acc[9];
        for (int e = 0; e < 9; ++e) acc[e] = Wr[9 * st + e];
        for (int p = pstart[st]; p < pstart[st + 1]; ++p) {
          const int sk = pairs[2 * p], su = pairs[2 * p + 1];
          int kx, ky, kz, kt;
          slot_off(sk, kx, ky, kz, kt);
          if (!inside(x + kx, y + ky, z + kz, t + kt, sh.dims)) continue;
          const long long rk = rho + kx + (long long)lx * (ky + (long long)ly * (kz + (long long)lz * kt));
          const double *Lik = Wr + 9 * sk;
          const double *Ukt = Wb + rk * 729 + 9 * su;
          double l[9], u[9];
          for (int e = 0; e < 9; ++e) {
            l[e] = Lik[e];
            u[e] = Ukt[e];
          }
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
              acc[3 * a + b] -= l[3 * a] * u[b] + l[3 * a + 1] * u[3 + b] + l[3 * a + 2] * u[6 + b];
        }
        if (st < 40) {
          const long long rt = rho + tx + (long long)lx * (ty + (long long)ly * (tz + (long long)lz * tt));
          const double *D = Wb + rt * 729 + 9 * 40;
          double d[9], o[9];
          for (int e = 0; e < 9; ++e) d[e] = D[e];
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
              o[3 * a + b] = acc[3 * a] * d[b] + acc[3 * a + 1] * d[3 + b] + acc[3 * a + 2] * d[6 + b];
          for (int e = 0; e < 9; ++e) acc[e] = o[e];
        } else if (st == 40) {
          double o[9];
          bool ok;
          inv33_pivot(acc, o, ok);
          if (!ok) {
            atomicMax(status, 1);
            for (int e = 0; e < 9; ++e) o[e] = 0.0;
          }
          for (int e = 0; e < 9; ++e) acc[e] = o[e];
        }
        for (int e = 0; e < 9; ++e) Wr[9 * st + e] = acc[e];
      }
    }
    __syncthreads();
  }
}

__device__ inline unsigned lanes_below(unsigned long long mask) {
  const unsigned lane = __lane_id();
  return (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
}

template <typename T>
__global__ void __launch_bounds__(512) compact_kernel(const SubInfo *__restrict__ subs,
                                                      const ShapeInfo *__restrict__ shapes,
                                                      const int32_t *__restrict__ lvl_start,
                                                      const uint64_t *__restrict__ coords,
                                                      const int32_t *__restrict__ ctab, int sub0,
                                                      const double *__restrict__ W, T *__restrict__ F) {
  const SubInfo sd = subs[sub0 + blockIdx.x];
  const ShapeInfo sh = shapes[sd.shape];
  const int lx = sh.dims[0], ly = sh.dims[1], lz = sh.dims[2];
  const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6), nwaves = (int)(blockDim.x >> 6);
  const double *Wb = W + sd.wbase;
  for (int L = 0; L < sh.nlev; ++L) {
    const int r0 = lvl_start[sh.lvl_off + L], r1 = lvl_start[sh.lvl_off + L + 1];
    const int R = r1 - r0, nch = (R + 63) / 64;
    for (int item = wave; item < nch * 9; item += nwaves) {
      const int c = item / 9, g = item % 9;
      const int q = c * 64 + lane;
      const bool valid = q < R;
      int x = 0, y = 0, z = 0, t = 0;
      if (valid) unpack(coords[sh.coord_off + r0 + q], x, y, z, t);
      const long long rho = x + (long long)lx * (y + (long long)ly * (z + (long long)lz * t));
      for (int j = 0; j < 9; ++j) {
        const int s = 9 * g + j;
        int dx, dy, dz, dt;
        slot_off(s, dx, dy, dz, dt);
        const bool has = valid && inside(x + dx, y + dy, z + dz, t + dt, sh.dims);
        const unsigned long long mask = __ballot(has);
        if (has) {
          const int32_t *ct = ctab + sh.ct_off + (((int64_t)L * sh.nchunk + c) * 81 + s) * 2;
          const int64_t cnt = ct[1], k = lanes_below(mask);
          T *dst = F + sd.fbase + ct[0];
          const double *src = Wb + rho * 729 + 9 * s;
          for (int e = 0; e < 9; ++e) dst[blk_pos(e, k, cnt)] = (T)src[e];
        }
      }
    }
  }
}

// --------------------------------------------------------------------------
// apply: z = sum_i (R^0_i)^T U_i^{-1} L_i^{-1} R^delta_i r
//
// One workgroup (8 wavefronts) per subdomain runs the forward sweep over the
// levels, then the backward sweep.  A level is cut into phases of up to
// kRows rows.  Wavefront w owns 5 of the 40 off-diagonal stencil slots of the
// sweep and walks the 64-row chunks of a phase in "units" of three slots
// (chunk, slots 0-2) and (chunk, slots 3-4): the loads of the next unit
// (factor blocks and neighbour values) are issued before the current unit is
// multiplied, so a wavefront always has a unit of loads in flight.  Partial
// sums go to LDS; after a barrier each thread finishes one row (y = r - sum,
// or z = inv(D)(y - sum)) and a second barrier publishes the new values.
// Everything a phase needs besides the factor stream is requested at the
// start of the phase, ahead of the factor loads: the coordinates of the next
// phase (kept in LDS, so address computation never waits on a vector load)
// and the inputs of the final step (r, or inv(D) and y).
//
// Local vectors use a strided (level, t, z, y) layout
//     row index = L * (lt lz ly) + (t lz + z) ly + y      (x = L - 2y - 4z - 8t)
// so the neighbour of any row through slot s is at a constant offset
// (dx + 2dy + 4dz + 8dt)(lt lz ly) + (dt lz + dz) ly + dy, and the 64 rows of
// a chunk touch nearly contiguous neighbour rows.
// --------------------------------------------------------------------------
constexpr int kRows = 256;
constexpr int kWaves = kApplyThreads / 64;
constexpr int kSlotsPerWave = 40 / kWaves;   // 5
constexpr int kUnit = 3;                     // slots per pipeline unit

template <typename T>
struct SweepArgs {
  SubInfo sd;
  ShapeInfo sh;
  OpDev op;
  cptr<int32_t> lvls;       // shape-relative level starts
  const uint64_t *crd;      // shape coords (read per lane)
  cptr<int32_t> ct;         // shape chunk table: (off9, cnt) per (level, chunk, slot)
  const T *F;
  T *Y;
  int64_t fzero, yzero;
  int64_t SL;               // lt * lz * ly
  const double *r;
  double *z;
};

// (element offset inside the subdomain, count) of the blocks of (level L, chunk cl, slot s).
// All arguments are wavefront-uniform; the index is made so explicitly, so that
// the entry comes through the scalar cache and never queues behind the factor
// loads in flight (a vector load here would have to drain them before the
// addresses that depend on it could be formed).
template <typename T>
__device__ inline void chunk_slot(const SweepArgs<T> &a, int L, int cl, int s, int64_t &off9, int64_t &cnt) {
  const int i = __builtin_amdgcn_readfirstlane(((L * a.sh.nchunk + cl) * 81 + s) * 2);
  off9 = a.ct[i];
  cnt = a.ct[i + 1];
}

// Block k of a group of cnt blocks starting at g (blk_pos layout; g is
// 16-byte aligned): two 16-byte loads and one 4-byte load.
__device__ inline void load_block(const float *g, int64_t k, int64_t cnt, float (&f)[9]) {
  const float4 a = *reinterpret_cast<const float4 *>(g + 4 * k);
  const float4 b = *reinterpret_cast<const float4 *>(g + 4 * cnt + 4 * k);
  f[0] = a.x, f[1] = a.y, f[2] = a.z, f[3] = a.w;
  f[4] = b.x, f[5] = b.y, f[6] = b.z, f[7] = b.w;
  f[8] = g[8 * cnt + k];
}
// FP64: four 16-byte loads and one 8-byte load.
__device__ inline void load_block(const double *g, int64_t k, int64_t cnt, double (&f)[9]) {
  const double2 a = *reinterpret_cast<const double2 *>(g + 4 * k);
  const double2 b = *reinterpret_cast<const double2 *>(g + 4 * k + 2);
  const double2 c = *reinterpret_cast<const double2 *>(g + 4 * cnt + 4 * k);
  const double2 d = *reinterpret_cast<const double2 *>(g + 4 * cnt + 4 * k + 2);
  f[0] = a.x, f[1] = a.y, f[2] = b.x, f[3] = b.y;
  f[4] = c.x, f[5] = c.y, f[6] = d.x, f[7] = d.y;
  f[8] = g[8 * cnt + k];
}

template <typename T>
__device__ inline int64_t yrow_of(const SweepArgs<T> &a, int x, int y, int zc, int t) {
  const int L = x + 2 * y + 4 * zc + 8 * t;
  return (int64_t)L * a.SL + ((int64_t)t * a.sh.dims[2] + zc) * a.sh.dims[1] + y;
}

template <typename T>
__device__ inline int64_t global_row(const SweepArgs<T> &a, int x, int y, int zc, int t) {
  const long long node =
      (a.sd.org[0] + x) + (long long)a.op.nn[0] * ((a.sd.org[1] + y) + (long long)a.op.nn[1] * (a.sd.org[2] + zc));
  return 3 * ((long long)(a.sd.org[3] + t) * a.op.N + node);
}

// Issue the loads of one unit: slots 3h .. 3h+2 of this wavefront's five for
// the lane's row (coordinates cw) in chunk cl of level L.
template <typename T, bool kFwd>
__device__ inline void load_unit(const SweepArgs<T> &a, int L, int cl, bool valid, uint64_t cw, int wave, int h,
                                 T (&f)[kUnit][9], T (&yv)[kUnit][3]) {
  int x, y, zc, t;
  unpack(cw, x, y, zc, t);
  const int64_t own = yrow_of(a, x, y, zc, t);
#pragma unroll
  for (int u = 0; u < kUnit; ++u) {
    const int j = kUnit * h + u;
    const bool real = j < kSlotsPerWave;
    const int s = (kFwd ? 0 : 41) + kSlotsPerWave * wave + (real ? j : 0);
    int dx, dy, dz, dt;
    slot_off(s, dx, dy, dz, dt);
    const bool has = real && valid && inside(x + dx, y + dy, zc + dz, t + dt, a.sh.dims);
    const unsigned long long mask = __ballot(has);
    int64_t off9, cnt;
    chunk_slot(a, L, cl, s, off9, cnt);
    const int64_t dY = (int64_t)(dx + 2 * dy + 4 * dz + 8 * dt) * a.SL + ((int64_t)dt * a.sh.dims[2] + dz) * a.sh.dims[1] + dy;
    // rows without the neighbour read the zero block (k = cnt = 0)
    const int64_t gi = has ? a.sd.fbase + off9 : a.fzero;
    const int64_t k = has ? (int64_t)lanes_below(mask) : 0, kc = has ? cnt : 0;
    const int64_t yi = has ? a.sd.sbase + 3 * (own + dY) : a.yzero;
    load_block(a.F + gi, k, kc, f[u]);
    const T *q = a.Y + yi;
    yv[u][0] = q[0];
    yv[u][1] = q[1];
    yv[u][2] = q[2];
  }
}

template <typename T>
__device__ inline void mac_unit(const T (&f)[kUnit][9], const T (&yv)[kUnit][3], T &a0, T &a1, T &a2) {
#pragma unroll
  for (int u = 0; u < kUnit; ++u) {
    a0 += f[u][0] * yv[u][0] + f[u][1] * yv[u][1] + f[u][2] * yv[u][2];
    a1 += f[u][3] * yv[u][0] + f[u][4] * yv[u][1] + f[u][5] * yv[u][2];
    a2 += f[u][6] * yv[u][0] + f[u][7] * yv[u][1] + f[u][8] * yv[u][2];
  }
}

// Next non-empty level after level counter li of the sweep (-1 if none).
__device__ inline int next_level(cptr<int32_t> lvls, int nlev, int li, bool fwd) {
  for (int k = li + 1; k < nlev; ++k) {
    const int L = fwd ? k : nlev - 1 - k;
    if (lvls[L + 1] > lvls[L]) return k;
  }
  return -1;
}

template <typename T, bool kFwd>
__device__ inline void sweep(const SweepArgs<T> &a, T (*part)[kRows][3], uint64_t *crdL) {
  const int lane = (int)__lane_id();
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tq = (int)threadIdx.x;
  const int nlev = a.sh.nlev;
  int li = next_level(a.lvls, nlev, -1, kFwd);
  if (li < 0) return;
  // coordinates of the first phase
  {
    const int L = kFwd ? li : nlev - 1 - li;
    const int r0 = a.lvls[L], segR = min(kRows, a.lvls[L + 1] - r0);
    if (tq < segR) crdL[tq] = a.crd[a.sh.coord_off + r0 + tq];
    __syncthreads();
  }
  int seg = 0;
  while (li >= 0) {
    const int L = kFwd ? li : nlev - 1 - li;
    const int r0 = a.lvls[L];
    const int R = a.lvls[L + 1] - r0;
    const int segR = min(kRows, R - seg * kRows);
    const int nch = (segR + 63) >> 6;
    // the phase after this one
    int nli = li, nseg = seg + 1;
    if (nseg * kRows >= R) {
      nli = next_level(a.lvls, nlev, li, kFwd);
      nseg = 0;
    }
    int nsegR = 0, nr0 = 0;
    if (nli >= 0) {
      const int nL = kFwd ? nli : nlev - 1 - nli;
      nr0 = a.lvls[nL];
      nsegR = min(kRows, a.lvls[nL + 1] - nr0 - nseg * kRows);
    }
    // requests issued ahead of the factor stream
    uint64_t cnext = 0;
    if (tq < nsegR) cnext = a.crd[a.sh.coord_off + nr0 + nseg * kRows + tq];
    uint64_t fc = 0;
    T pre[12];
    int64_t gi = 0, yown = 0;
    if (tq < segR) {
      fc = crdL[tq];
      int x, y, zc, t;
      unpack(fc, x, y, zc, t);
      gi = global_row(a, x, y, zc, t);
      yown = a.sd.sbase + 3 * yrow_of(a, x, y, zc, t);
      if (kFwd) {
        pre[0] = (T)a.r[gi];
        pre[1] = (T)a.r[gi + 1];
        pre[2] = (T)a.r[gi + 2];
      } else {
        const int qrow = seg * kRows + tq;   // slot 40: every row of the chunk, rank = row & 63
        int64_t off9, cnt;
        chunk_slot(a, L, __builtin_amdgcn_readfirstlane(qrow >> 6), 40, off9, cnt);
        T dg[9];
        load_block(a.F + a.sd.fbase + off9, qrow & 63, cnt, dg);
#pragma unroll
        for (int e = 0; e < 9; ++e) pre[e] = dg[e];
        pre[9] = a.Y[yown];
        pre[10] = a.Y[yown + 1];
        pre[11] = a.Y[yown + 2];
      }
    }
    // factor stream: units (chunk c, slots 0-2) and (chunk c, slots 3-4)
    const int cl0 = (seg * kRows) >> 6;
    T fA[kUnit][9], yA[kUnit][3], fB[kUnit][9], yB[kUnit][3];
    load_unit<T, kFwd>(a, L, cl0, lane < segR, crdL[lane], wave, 0, fA, yA);
    for (int c = 0; c < nch; ++c) {
      const bool valid = c * 64 + lane < segR;
      const uint64_t cw = crdL[c * 64 + lane];
      load_unit<T, kFwd>(a, L, cl0 + c, valid, cw, wave, 1, fB, yB);
      T a0 = 0, a1 = 0, a2 = 0;
      mac_unit(fA, yA, a0, a1, a2);
      if (c + 1 < nch) {
        const bool valid1 = (c + 1) * 64 + lane < segR;
        load_unit<T, kFwd>(a, L, cl0 + c + 1, valid1, crdL[(c + 1) * 64 + lane], wave, 0, fA, yA);
      }
      mac_unit(fB, yB, a0, a1, a2);
      if (valid) {
        part[wave][c * 64 + lane][0] = a0;
        part[wave][c * 64 + lane][1] = a1;
        part[wave][c * 64 + lane][2] = a2;
      }
    }
    __syncthreads();
    if (tq < segR) {
      T s3[3];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        T acc = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) acc += part[w][tq][cc];
        s3[cc] = acc;
      }
      T *yr = a.Y + yown;
      if (kFwd) {
        for (int cc = 0; cc < 3; ++cc) yr[cc] = pre[cc] - s3[cc];
      } else {
        T v[3], o[3];
        for (int cc = 0; cc < 3; ++cc) v[cc] = pre[9 + cc] - s3[cc];
        for (int cc = 0; cc < 3; ++cc) o[cc] = pre[3 * cc] * v[0] + pre[3 * cc + 1] * v[1] + pre[3 * cc + 2] * v[2];
        for (int cc = 0; cc < 3; ++cc) yr[cc] = o[cc];
        int x, y, zc, t;
        unpack(fc, x, y, zc, t);
        const SubInfo &sd = a.sd;
        const bool owned = x >= sd.olo[0] && x < sd.ohi[0] && y >= sd.olo[1] && y < sd.ohi[1] && zc >= sd.olo[2] &&
                           zc < sd.ohi[2] && t >= sd.olo[3] && t < sd.ohi[3];
        if (owned)
          for (int cc = 0; cc < 3; ++cc) a.z[gi + cc] = (double)o[cc];
      }
    }
    if (tq < nsegR) crdL[tq] = cnext;
    __syncthreads();
    li = nli;
    seg = nseg;
  }
}

template <typename T>
__global__ void __launch_bounds__(kApplyThreads, 2) apply_kernel(OpDev op, const SubInfo *__restrict__ subs,
                                                                 const int32_t *__restrict__ order,
                                                                 const ShapeInfo *__restrict__ shapes,
                                                                 const int32_t *__restrict__ lvl_start,
                                                                 const uint64_t *__restrict__ coords,
                                                                 const int32_t *__restrict__ ctab,
                                                                 const T *__restrict__ F, T *__restrict__ Y,
                                                                 int64_t fzero, int64_t yzero,
                                                                 const double *__restrict__ r,
                                                                 double *__restrict__ z) {
  __shared__ T part[kWaves][kRows][3];
  __shared__ uint64_t crdL[kRows];
  SweepArgs<T> a;
  const int sub = as_const(order)[blockIdx.x];
  a.sd = load_uniform(subs + sub);
  a.sh = load_uniform(shapes + a.sd.shape);
  a.op = op;
  a.lvls = as_const(lvl_start) + a.sh.lvl_off;
  a.crd = coords;
  a.ct = as_const(ctab) + a.sh.ct_off;
  a.F = F;
  a.Y = Y;
  a.fzero = fzero;
  a.yzero = yzero;
  a.SL = (int64_t)a.sh.dims[3] * a.sh.dims[2] * a.sh.dims[1];
  a.r = r;
  a.z = z;
  sweep<T, true>(a, part, crdL);
  __syncthreads();
  sweep<T, false>(a, part, crdL);
}

// --------------------------------------------------------------------------
// apply, LDS-ring form (used when the ring fits in LDS).
//
// Same work split as above, but the values of the last 16 levels live in an
// LDS ring (16 is one more than the largest level distance between a row and
// its stencil neighbours, x + 2y + 4z + 8t changes by at most 15).  A row's
// place inside its level is (rows of the level in earlier (t, z) groups) +
// (y - first y of its group); the per-level (t, z) prefix rows sit in a
// second LDS ring.  Level barriers therefore only synchronise LDS, so the
// factor loads of the next chunk -- also across phase and level boundaries --
// stay in flight through them: a wavefront streams its factor blocks
// continuously, one 64-row chunk ahead of the multiply.  The forward result y
// is also written to global memory (the backward sweep reads it once per row),
// and z is written to the output on owned rows.
// --------------------------------------------------------------------------
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A phase: segment seg (KR rows) of level L, the level's rows starting
// at r0 (R of them); L < 0 once the sweep has no further phase.  Only these
// four values are kept (the kernel is short of scalar registers); the rest
// is derived.
template <int KR>
struct Phase {
  int L, seg, r0, R;
  __device__ bool done() const { return L < 0; }
  __device__ int segR() const { return min(KR, R - seg * KR); }
  __device__ int nch() const { return (segR() + 63) >> 6; }
};

// li: index of the level in sweep order
template <int KR>
__device__ inline void phase_at(Phase<KR> &p, cptr<int32_t> lvls, int nlev, int li, int seg, bool fwd) {
  if (li < 0) {
    p.L = -1, p.seg = 0, p.r0 = 0, p.R = 0;
    return;
  }
  p.L = fwd ? li : nlev - 1 - li;
  p.r0 = lvls[p.L];
  p.R = lvls[p.L + 1] - p.r0;
  p.seg = seg;
}

template <int KR>
__device__ inline void phase_next(Phase<KR> &n, const Phase<KR> &p, cptr<int32_t> lvls, int nlev, bool fwd) {
  if (p.done()) {
    n = p;
    return;
  }
  const int li = fwd ? p.L : nlev - 1 - p.L;
  if ((p.seg + 1) * KR < p.R) phase_at(n, lvls, nlev, li, p.seg + 1, fwd);
  else phase_at(n, lvls, nlev, next_level(lvls, nlev, li, fwd), 0, fwd);
}

struct Ring {
  int rmax;   // rows per ring level
  int ltlz;   // (t, z) groups per level
};

// Boundary code of a row of the subdomain box: bit k set if the row lies on
// the low face of dimension k, bit 4+k on the high face.  A stencil slot whose
// offset leaves the box through one of those faces has no neighbour there.
template <typename T>
__device__ inline int face_code(const SweepArgs<T> &a, int x, int y, int zc, int t) {
  return (x == 0 ? 1 : 0) | (y == 0 ? 2 : 0) | (zc == 0 ? 4 : 0) | (t == 0 ? 8 : 0) |
         (x == a.sh.dims[0] - 1 ? 16 : 0) | (y == a.sh.dims[1] - 1 ? 32 : 0) | (zc == a.sh.dims[2] - 1 ? 64 : 0) |
         (t == a.sh.dims[3] - 1 ? 128 : 0);
}

// The faces (same bit layout) through which slot offset (dx, dy, dz, dt) leaves.
__device__ inline int slot_faces(int dx, int dy, int dz, int dt) {
  return (dx < 0 ? 1 : 0) | (dy < 0 ? 2 : 0) | (dz < 0 ? 4 : 0) | (dt < 0 ? 8 : 0) | (dx > 0 ? 16 : 0) |
         (dy > 0 ? 32 : 0) | (dz > 0 ? 64 : 0) | (dt > 0 ? 128 : 0);
}

// Factor loads of all five slots of this wavefront for chunk c of phase p.
// The chunk-table entries of the five slots are adjacent and are requested
// together, so a single scalar round trip precedes the 45 vector loads.
// The chunk is given by its level L, its chunk index cl inside the level and
// its number of rows (done: past the last phase, nothing is loaded).
template <typename T, bool kFwd>
__device__ inline void load_chunk_f(const SweepArgs<T> &a, bool done, int L, int cl, int rows, uint64_t cw,
                                    int wave, T (&f)[kSlotsPerWave][9]) {
  const int lane = (int)__lane_id();
  int x, y, zc, t;
  unpack(cw, x, y, zc, t);
  const bool valid = !done && lane < rows;
  const int code = face_code(a, x, y, zc, t);
  const int s0 = (kFwd ? 0 : 41) + kSlotsPerWave * wave;
  int32_t tab[2 * kSlotsPerWave];
  if (!done) {
    const int i0 = __builtin_amdgcn_readfirstlane(((L * a.sh.nchunk + cl) * 81 + s0) * 2);
#pragma unroll
    for (int k = 0; k < 2 * kSlotsPerWave; ++k) tab[k] = a.ct[i0 + k];
  } else {
#pragma unroll
    for (int k = 0; k < 2 * kSlotsPerWave; ++k) tab[k] = 0;
  }
#pragma unroll
  for (int j = 0; j < kSlotsPerWave; ++j) {
    int dx, dy, dz, dt;
    slot_off(s0 + j, dx, dy, dz, dt);
    const bool has = valid && (code & slot_faces(dx, dy, dz, dt)) == 0;
    const unsigned long long mask = __ballot(has);
    // rows without the neighbour read the zero block (k = cnt = 0)
    const int64_t gi = has ? a.sd.fbase + tab[2 * j] : a.fzero;
    const int64_t k = has ? (int64_t)lanes_below(mask) : 0, kc = has ? tab[2 * j + 1] : 0;
    load_block(a.F + gi, k, kc, f[j]);
  }
}

template <typename T, bool kFwd, int KR>
__device__ inline void load_chunk_f(const SweepArgs<T> &a, const Phase<KR> &p, int c, uint64_t cw, int wave,
                                    T (&f)[kSlotsPerWave][9]) {
  load_chunk_f<T, kFwd>(a, p.done(), p.L, p.seg * (KR / 64) + c, p.segR() - 64 * c, cw, wave, f);
}

// Multiply chunk c of phase p: neighbour values from the LDS ring.  All rows
// of a phase lie on level p.L, so a slot's neighbours all lie on level
// p.L + dx + 2dy + 4dz + 8dt, and its ring slot is the same for the whole
// wavefront.  The lookups carry no branches: rows without the neighbour read
// ring entry 0 and discard the value, so the LDS requests of the five slots
// can be in flight together.
template <typename T, bool kFwd, int KR>
__device__ inline void mac_chunk_ring(const SweepArgs<T> &a, const Phase<KR> &p, int c, uint64_t cw, int wave,
                                      const T (&f)[kSlotsPerWave][9], const T *yring, const int32_t *tzr,
                                      const Ring &rg, T &a0, T &a1, T &a2) {
  const int lane = (int)__lane_id();
  int x, y, zc, t;
  unpack(cw, x, y, zc, t);
  const bool valid = c * 64 + lane < p.segR();
  const int code = face_code(a, x, y, zc, t);
  const int lx = a.sh.dims[0], lz = a.sh.dims[2];
  const int xy = x + 2 * y, tz = t * lz + zc;
  const int s0 = (kFwd ? 0 : 41) + kSlotsPerWave * wave;
  // all prefix-row lookups first, so that they are in flight together
  int hb = 0, qv[kSlotsPerWave];
#pragma unroll
  for (int j = 0; j < kSlotsPerWave; ++j) {
    int dx, dy, dz, dt;
    slot_off(s0 + j, dx, dy, dz, dt);
    const bool has = valid && (code & slot_faces(dx, dy, dz, dt)) == 0;
    hb |= has ? 1 << j : 0;
    const int slot = (p.L + dx + 2 * dy + 4 * dz + 8 * dt) & 15;
    qv[j] = tzr[has ? slot * rg.ltlz + tz + dt * lz + dz : 0];
  }
#pragma unroll
  for (int j = 0; j < kSlotsPerWave; ++j) {
    int dx, dy, dz, dt;
    slot_off(s0 + j, dx, dy, dz, dt);
    const bool has = (hb >> j) & 1;
    const int slot = (p.L + dx + 2 * dy + 4 * dz + 8 * dt) & 15;
    const int rem = xy + dx + 2 * dy;   // nx + 2 ny of the neighbour
    const int ymin = max(0, (rem - lx + 2) >> 1);
    const int vi = has ? (slot * rg.rmax + qv[j] + (y + dy - ymin)) * 3 : 0;
    const T w0 = yring[vi], w1 = yring[vi + 1], w2 = yring[vi + 2];
    const T v0 = has ? w0 : (T)0, v1 = has ? w1 : (T)0, v2 = has ? w2 : (T)0;
    a0 += f[j][0] * v0 + f[j][1] * v1 + f[j][2] * v2;
    a1 += f[j][3] * v0 + f[j][4] * v1 + f[j][5] * v2;
    a2 += f[j][6] * v0 + f[j][7] * v1 + f[j][8] * v2;
  }
}

// Inputs of the final step of row tq of phase p (coordinates crd), requested
// at the start of the phase: r (forward; kept in FP64 until it is used, so
// that no conversion waits on the load while factor loads are in flight), or
// inv(U_rr) and y (backward).  The chunk-table entry of the diagonal slot is
// wavefront-uniform (a wavefront holds 64 consecutive rows) and is read
// through the scalar cache.
template <typename T, bool kFwd, int KR>
__device__ inline void load_pre(const SweepArgs<T> &a, const Phase<KR> &p, const uint64_t *crd, T (&pre)[12],
                                double (&rin)[3]) {
  const int tq = (int)threadIdx.x;
  if (tq >= p.segR()) return;
  int x, y, zc, t;
  unpack(crd[tq], x, y, zc, t);
  if (kFwd) {
    const int64_t gi = global_row(a, x, y, zc, t);
    rin[0] = a.r[gi];
    rin[1] = a.r[gi + 1];
    rin[2] = a.r[gi + 2];
  } else {
    const int qrow = p.seg * KR + tq;
    int64_t off9, cnt;
    chunk_slot(a, p.L, qrow >> 6, 40, off9, cnt);
    // the row's place in its chunk is made opaque here, so that the compiler
    // forms this address inside the sweep loop instead of keeping a per-lane
    // pointer alive across it (which does not fit the FP64 register budget)
    int lrow = qrow & 63;
    asm volatile("" : "+v"(lrow));
    T dg[9];
    load_block(a.F + a.sd.fbase + off9, lrow, cnt, dg);
#pragma unroll
    for (int e = 0; e < 9; ++e) pre[e] = dg[e];
    const int64_t yo = a.sd.sbase + 3 * yrow_of(a, x, y, zc, t);
    pre[9] = a.Y[yo];
    pre[10] = a.Y[yo + 1];
    pre[11] = a.Y[yo + 2];
  }
}

// Final step of a phase, one thread per row: sum the wavefronts' partial
// products, then y = r - sum (forward, y also kept in global memory for the
// backward sweep) or z = inv(U_rr)(y - sum) (backward, owned rows written to
// the output); the result goes into the LDS ring.
template <typename T, bool kFwd, int KR>
__device__ inline void ring_finish(const SweepArgs<T> &a, const Phase<KR> &pc, const uint64_t *crd, T (*part)[KR][3],
                                   const T (&pre)[12], const double (&rin)[3], T *yring, const Ring &rg) {
  const int tq = (int)threadIdx.x;
  if (tq < pc.segR()) {
    const uint64_t fc = crd[tq];
    T s3[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T acc = 0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) acc += part[w][tq][k];
      s3[k] = acc;
    }
    T o[3];
    int x, y, zc, t;
    unpack(fc, x, y, zc, t);
    if (kFwd) {
      for (int k = 0; k < 3; ++k) o[k] = (T)rin[k] - s3[k];
      T *yg = a.Y + a.sd.sbase + 3 * yrow_of(a, x, y, zc, t);
      for (int k = 0; k < 3; ++k) yg[k] = o[k];
    } else {
      T v[3];
      for (int k = 0; k < 3; ++k) v[k] = pre[9 + k] - s3[k];
      for (int k = 0; k < 3; ++k) o[k] = pre[3 * k] * v[0] + pre[3 * k + 1] * v[1] + pre[3 * k + 2] * v[2];
      const SubInfo &sd = a.sd;
      const bool owned = x >= sd.olo[0] && x < sd.ohi[0] && y >= sd.olo[1] && y < sd.ohi[1] && zc >= sd.olo[2] &&
                         zc < sd.ohi[2] && t >= sd.olo[3] && t < sd.ohi[3];
      if (owned) {
        const int64_t gi = global_row(a, x, y, zc, t);
        for (int k = 0; k < 3; ++k) a.z[gi + k] = (double)o[k];
      }
    }
    T *yr = yring + ((int64_t)(pc.L & 15) * rg.rmax + pc.seg * KR + tq) * 3;
    for (int k = 0; k < 3; ++k) yr[k] = o[k];
  }
}

// One chunk step: issue the factor loads of the next chunk, multiply the
// current one, and close the phase if this was its last chunk.
template <typename T, bool kFwd, int KR>
__device__ inline void ring_step(const SweepArgs<T> &a, cptr<int32_t> tzp, int nlev, int wave, Phase<KR> &pc, int &cc,
                                 int &par, Phase<KR> &pn, Phase<KR> &pnn, const T (&fcur)[kSlotsPerWave][9],
                                 T (&fnext)[kSlotsPerWave][9], T (*part)[KR][3], uint64_t *crd2, T *yring,
                                 int32_t *tzr, const Ring &rg, uint64_t &c2, int &tzrow, T (&pre)[12],
                                 double (&rin)[3]) {
  const int lane = (int)__lane_id();
  const int tq = (int)threadIdx.x;
  // requests of the phase, issued when its first chunk is multiplied: coordinates
  // two phases ahead, the (t, z) prefix row of a new level, final-step inputs
  if (cc == 0) {
    if (!pnn.done() && tq < pnn.segR()) c2 = a.crd[a.sh.coord_off + pnn.r0 + pnn.seg * KR + tq];
    if (pc.seg == 0 && tq < rg.ltlz) tzrow = tzp[pc.L * rg.ltlz + tq];
    load_pre<T, kFwd>(a, pc, crd2 + par * KR, pre, rin);
  }
  // next chunk: same phase, or the first chunk of the next phase
  const bool last = cc == pc.nch() - 1;
  {
    // chosen with selects, field by field, so that the phases stay in registers
    const bool tdone = last ? pn.done() : pc.done();
    const int tL = last ? pn.L : pc.L, tseg = last ? pn.seg : pc.seg, tsegR = last ? pn.segR() : pc.segR();
    const int ct = last ? 0 : cc + 1;
    const int pt_par = last ? par ^ 1 : par;
    const uint64_t cw = crd2[pt_par * KR + ct * 64 + lane];
    load_chunk_f<T, kFwd>(a, tdone, tL, tseg * (KR / 64) + ct, tsegR - 64 * ct, cw, wave, fnext);
  }
  // multiply the current chunk
  {
    const uint64_t cw = crd2[par * KR + cc * 64 + lane];
    T a0 = 0, a1 = 0, a2 = 0;
    mac_chunk_ring<T, kFwd>(a, pc, cc, cw, wave, fcur, yring, tzr, rg, a0, a1, a2);
    if (cc * 64 + lane < pc.segR()) {
      part[wave][cc * 64 + lane][0] = a0;
      part[wave][cc * 64 + lane][1] = a1;
      part[wave][cc * 64 + lane][2] = a2;
    }
  }
  if (!last) {
    ++cc;
    return;
  }
  // close the phase
  lds_barrier();
  ring_finish<T, kFwd>(a, pc, crd2 + par * KR, part, pre, rin, yring, rg);
  if (pc.seg == 0 && tq < rg.ltlz) tzr[(pc.L & 15) * rg.ltlz + tq] = tzrow;
  if (!pnn.done() && tq < pnn.segR()) crd2[par * KR + tq] = c2;   // phase after next reuses this buffer
  lds_barrier();
  // advance
  pc = pn;
  pn = pnn;
  phase_next(pnn, pn, a.lvls, nlev, kFwd);
  par ^= 1;
  cc = 0;
}

template <typename T, bool kFwd, int KR>
__device__ inline void sweep_ring(const SweepArgs<T> &a, cptr<int32_t> tzp, T (*part)[KR][3], uint64_t *crd2,
                                  T *yring, int32_t *tzr, const Ring &rg) {
  const int lane = (int)__lane_id();
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tq = (int)threadIdx.x;
  const int nlev = a.sh.nlev;
  Phase<KR> pc, pn, pnn;
  phase_at(pc, a.lvls, nlev, next_level(a.lvls, nlev, -1, kFwd), 0, kFwd);
  if (pc.done()) return;
  phase_next(pn, pc, a.lvls, nlev, kFwd);
  phase_next(pnn, pn, a.lvls, nlev, kFwd);
  // coordinates of the first two phases
  if (tq < pc.segR()) crd2[tq] = a.crd[a.sh.coord_off + pc.r0 + pc.seg * KR + tq];
  if (!pn.done() && tq < pn.segR()) crd2[KR + tq] = a.crd[a.sh.coord_off + pn.r0 + pn.seg * KR + tq];
  __syncthreads();
  int par = 0, cc = 0;
  uint64_t c2 = 0;
  int tzrow = 0;
  T pre[12];
  double rin[3];
  T fA[kSlotsPerWave][9], fB[kSlotsPerWave][9];
  load_chunk_f<T, kFwd>(a, pc, 0, crd2[lane], wave, fA);
  for (;;) {
    ring_step<T, kFwd>(a, tzp, nlev, wave, pc, cc, par, pn, pnn, fA, fB, part, crd2, yring, tzr, rg, c2, tzrow, pre,
                       rin);
    if (pc.done()) break;
    ring_step<T, kFwd>(a, tzp, nlev, wave, pc, cc, par, pn, pnn, fB, fA, part, crd2, yring, tzr, rg, c2, tzrow, pre,
                       rin);
    if (pc.done()) break;
  }
}

// Depth-2 form of the pipeline (FP32 factors, whose registers allow three
// chunk buffers): the factor loads of the chunk two steps ahead are issued
// before the current chunk is multiplied.  That chunk may lie up to two phases
// ahead, so the coordinates of the current phase and the next two live in
// three LDS buffers (par, par+1, par+2 mod 3); the phase three ahead is read
// into registers at the start of a phase and stored into the buffer the
// closing phase frees.
template <typename T, bool kFwd, int KR>
__device__ inline void ring_step2(const SweepArgs<T> &a, cptr<int32_t> tzp, int nlev, int wave, Phase<KR> &pc, int &cc,
                                  int &par, Phase<KR> &pn, Phase<KR> &pnn, Phase<KR> &p3, const T (&fcur)[kSlotsPerWave][9],
                                  T (&fload)[kSlotsPerWave][9], T (*part)[KR][3], uint64_t *crd3, T *yring,
                                  int32_t *tzr, const Ring &rg, uint64_t &c3, int &tzrow, T (&pre)[12],
                                  double (&rin)[3]) {
  const int lane = (int)__lane_id();
  const int tq = (int)threadIdx.x;
  if (cc == 0) {
    if (!p3.done() && tq < p3.segR()) c3 = a.crd[a.sh.coord_off + p3.r0 + p3.seg * KR + tq];
    if (pc.seg == 0 && tq < rg.ltlz) tzrow = tzp[pc.L * rg.ltlz + tq];
    load_pre<T, kFwd>(a, pc, crd3 + par * KR, pre, rin);
  }
  // the chunk two steps ahead: (pc, cc+2), (pn, 0), (pn, 1) or (pnn, 0)
  {
    const int p1 = par == 2 ? 0 : par + 1, p2 = par == 0 ? 2 : par - 1;
    // chosen with selects, field by field, so that the phases stay in registers
    const int which = cc + 2 < pc.nch() ? 0 : (cc + 2 == pc.nch() || (!pn.done() && pn.nch() >= 2)) ? 1 : 2;
    const bool tdone = which == 0 ? pc.done() : which == 1 ? pn.done() : pnn.done();
    const int tL = which == 0 ? pc.L : which == 1 ? pn.L : pnn.L;
    const int tseg = which == 0 ? pc.seg : which == 1 ? pn.seg : pnn.seg;
    const int tsegR = which == 0 ? pc.segR() : which == 1 ? pn.segR() : pnn.segR();
    const int ct = which == 0 ? cc + 2 : which == 1 ? (cc + 2 == pc.nch() ? 0 : 1) : 0;
    const int tpar = which == 0 ? par : which == 1 ? p1 : p2;
    const uint64_t cw = crd3[tpar * KR + ct * 64 + lane];
    load_chunk_f<T, kFwd>(a, tdone, tL, tseg * (KR / 64) + ct, tsegR - 64 * ct, cw, wave, fload);
  }
  // multiply the current chunk
  {
    const uint64_t cw = crd3[par * KR + cc * 64 + lane];
    T a0 = 0, a1 = 0, a2 = 0;
    mac_chunk_ring<T, kFwd>(a, pc, cc, cw, wave, fcur, yring, tzr, rg, a0, a1, a2);
    if (cc * 64 + lane < pc.segR()) {
      part[wave][cc * 64 + lane][0] = a0;
      part[wave][cc * 64 + lane][1] = a1;
      part[wave][cc * 64 + lane][2] = a2;
    }
  }
  if (cc != pc.nch() - 1) {
    ++cc;
    return;
  }
  // close the phase
  lds_barrier();
  ring_finish<T, kFwd>(a, pc, crd3 + par * KR, part, pre, rin, yring, rg);
  if (pc.seg == 0 && tq < rg.ltlz) tzr[(pc.L & 15) * rg.ltlz + tq] = tzrow;
  if (!p3.done() && tq < p3.segR()) crd3[par * KR + tq] = c3;   // the phase three ahead reuses this buffer
  lds_barrier();
  pc = pn;
  pn = pnn;
  pnn = p3;
  phase_next(p3, pnn, a.lvls, nlev, kFwd);
  par = par == 2 ? 0 : par + 1;
  cc = 0;
}

template <typename T, bool kFwd, int KR>
__device__ inline void sweep_ring2(const SweepArgs<T> &a, cptr<int32_t> tzp, T (*part)[KR][3], uint64_t *crd3,
                                   T *yring, int32_t *tzr, const Ring &rg) {
  const int lane = (int)__lane_id();
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int tq = (int)threadIdx.x;
  const int nlev = a.sh.nlev;
  Phase<KR> pc, pn, pnn, p3;
  phase_at(pc, a.lvls, nlev, next_level(a.lvls, nlev, -1, kFwd), 0, kFwd);
  if (pc.done()) return;
  phase_next(pn, pc, a.lvls, nlev, kFwd);
  phase_next(pnn, pn, a.lvls, nlev, kFwd);
  phase_next(p3, pnn, a.lvls, nlev, kFwd);
  // coordinates of the first three phases
  if (tq < pc.segR()) crd3[tq] = a.crd[a.sh.coord_off + pc.r0 + pc.seg * KR + tq];
  if (!pn.done() && tq < pn.segR()) crd3[KR + tq] = a.crd[a.sh.coord_off + pn.r0 + pn.seg * KR + tq];
  if (!pnn.done() && tq < pnn.segR()) crd3[2 * KR + tq] = a.crd[a.sh.coord_off + pnn.r0 + pnn.seg * KR + tq];
  __syncthreads();
  int par = 0, cc = 0;
  uint64_t c3 = 0;
  int tzrow = 0;
  T pre[12];
  double rin[3];
  T fA[kSlotsPerWave][9], fB[kSlotsPerWave][9], fC[kSlotsPerWave][9];
  load_chunk_f<T, kFwd>(a, pc, 0, crd3[lane], wave, fA);
  if (pc.nch() >= 2) load_chunk_f<T, kFwd>(a, pc, 1, crd3[64 + lane], wave, fB);
  else load_chunk_f<T, kFwd>(a, pn, 0, crd3[KR + lane], wave, fB);
  for (;;) {
    ring_step2<T, kFwd>(a, tzp, nlev, wave, pc, cc, par, pn, pnn, p3, fA, fC, part, crd3, yring, tzr, rg, c3, tzrow,
                        pre, rin);
    if (pc.done()) break;
    ring_step2<T, kFwd>(a, tzp, nlev, wave, pc, cc, par, pn, pnn, p3, fB, fA, part, crd3, yring, tzr, rg, c3, tzrow,
                        pre, rin);
    if (pc.done()) break;
    ring_step2<T, kFwd>(a, tzp, nlev, wave, pc, cc, par, pn, pnn, p3, fC, fB, part, crd3, yring, tzr, rg, c3, tzrow,
                        pre, rin);
    if (pc.done()) break;
  }
}

// Chunk-coordinate buffers of the apply kernel: two for the depth-1 pipeline
// (FP64), three for the depth-2 one (FP32).
template <typename T> constexpr int kCrdBufs = sizeof(T) == 4 ? 3 : 2;

// Both sweeps of subdomain `sub` with the values of the last 16 levels in LDS.
template <typename T, int KR>
__device__ inline void apply_ring_sub(const OpDev &op, const SubInfo *__restrict__ subs, int sub,
                                      const ShapeInfo *__restrict__ shapes, const int32_t *__restrict__ lvl_start,
                                      const uint64_t *__restrict__ coords, const int32_t *__restrict__ ctab,
                                      const int32_t *__restrict__ tzpref, const T *__restrict__ F,
                                      T *__restrict__ Y, int64_t fzero, int64_t yzero, const Ring &rg,
                                      const double *__restrict__ r, double *__restrict__ z) {
  extern __shared__ __align__(16) unsigned char smem[];
  T(*part)[KR][3] = reinterpret_cast<T(*)[KR][3]>(smem);
  uint64_t *crd2 = reinterpret_cast<uint64_t *>(smem + sizeof(T) * kWaves * KR * 3);
  T *yring = reinterpret_cast<T *>(smem + sizeof(T) * kWaves * KR * 3 + sizeof(uint64_t) * kCrdBufs<T> * KR);
  int32_t *tzr = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(yring) +
                                             sizeof(T) * (size_t)16 * rg.rmax * 3);
  SweepArgs<T> a;
  a.sd = load_uniform(subs + sub);
  a.sh = load_uniform(shapes + a.sd.shape);
  a.op = op;
  a.lvls = as_const(lvl_start) + a.sh.lvl_off;
  a.crd = coords;
  a.ct = as_const(ctab) + a.sh.ct_off;
  a.F = F;
  a.Y = Y;
  a.fzero = fzero;
  a.yzero = yzero;
  a.SL = (int64_t)a.sh.dims[3] * a.sh.dims[2] * a.sh.dims[1];
  a.r = r;
  a.z = z;
  const cptr<int32_t> tzp = as_const(tzpref) + a.sh.tz_off;
  Ring rl = rg;
  rl.ltlz = a.sh.dims[3] * a.sh.dims[2];
  if (kCrdBufs<T> == 3) {
    sweep_ring2<T, true>(a, tzp, part, crd2, yring, tzr, rl);
    __syncthreads();   // forward results in global memory are read by the backward sweep
    sweep_ring2<T, false>(a, tzp, part, crd2, yring, tzr, rl);
  } else {
    sweep_ring<T, true>(a, tzp, part, crd2, yring, tzr, rl);
    __syncthreads();
    sweep_ring<T, false>(a, tzp, part, crd2, yring, tzr, rl);
  }
}

template <typename T, int KR>
__global__ void __launch_bounds__(kApplyThreads, 2) apply_ring_kernel(
    OpDev op, const SubInfo *__restrict__ subs, const int32_t *__restrict__ order,
    const ShapeInfo *__restrict__ shapes, const int32_t *__restrict__ lvl_start,
    const uint64_t *__restrict__ coords, const int32_t *__restrict__ ctab, const int32_t *__restrict__ tzpref, const T *__restrict__ F, T *__restrict__ Y, int64_t fzero, int64_t yzero,
    Ring rg, const double *__restrict__ r, double *__restrict__ z) {
  const int sub = as_const(order)[blockIdx.x];
  apply_ring_sub<T, KR>(op, subs, sub, shapes, lvl_start, coords, ctab, tzpref, F, Y, fzero, yzero, rg, r, z);
}

// One preconditioner of a batched application; its vectors start at element
// voff of the batch's concatenated r and z.
template <typename T>
struct RasBatchDesc {
  OpDev op;
  const SubInfo *subs;
  const ShapeInfo *shapes;
  const int32_t *lvl;
  const uint64_t *coords;
  const int32_t *ctab;
  const int32_t *tz;
  const T *F;
  T *Y;
  int64_t fzero, yzero, voff;
  Ring rg;
};

// Work list entry (preconditioner, subdomain), ordered largest box first
// over the whole batch.
template <typename T, int KR>
__global__ void __launch_bounds__(kApplyThreads, 2) apply_ring_batch_kernel(const RasBatchDesc<T> *__restrict__ descs,
                                                                            const int2 *__restrict__ work,
                                                                            const int *__restrict__ act,
                                                                            const double *__restrict__ r,
                                                                            const double *__restrict__ r2,
                                                                            double *__restrict__ z) {
  const int2 wk = load_uniform(work + blockIdx.x);
  const int a = as_const(act)[wk.x];
  if (!a) return;
  const RasBatchDesc<T> d = load_uniform(descs + wk.x);
  // The pointers are read as pointers from the constant address space: the
  // compiler then takes them to address global memory and emits global loads.
  // (Pointers rebuilt from copied words would be generic, and generic loads
  // also count against the LDS counter, so every LDS wait of the sweep would
  // drain the factor loads in flight.)
  const cptr<RasBatchDesc<T>> dp = as_const(descs + wk.x);
  apply_ring_sub<T, KR>(d.op, dp->subs, wk.y, dp->shapes, dp->lvl, dp->coords, dp->ctab, dp->tz, dp->F, dp->Y, d.fzero,
                    d.yzero, d.rg, (a == 2 ? r2 : r) + d.voff, z + d.voff);
}

}  // namespace

// LDS of the ring kernel with KR rows per phase: partial sums, phase
// coordinates, the 16-level value ring and the (t, z) prefix rows of its levels.
template <typename T, int KR>
static size_t ring_lds_bytes(const ras *R) {
  return sizeof(T) * kWaves * KR * 3 + sizeof(uint64_t) * kCrdBufs<T> * KR +
         sizeof(T) * (size_t)16 * R->ring_rmax * 3 +
         sizeof(int32_t) * (size_t)16 * R->ring_ltlz;
}

template <typename T, int KR>
static void launch_ring(const ras *R, const double *r, double *z, T *Y, size_t lds, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    STKKT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&apply_ring_kernel<T, KR>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRingLdsLimit));
    attr_set = true;
  }
  Ring rg{R->ring_rmax, R->ring_ltlz};
  hipLaunchKernelGGL((apply_ring_kernel<T, KR>), dim3(R->nsub), dim3(kApplyThreads), lds, s, R->d,
                     R->d_subs.as<SubInfo>(), R->d_order.as<int32_t>(), R->d_shapes.as<ShapeInfo>(),
                     R->d_lvl.as<int32_t>(), R->d_coords.as<uint64_t>(), R->d_ctab.as<int32_t>(),
                     R->d_tz.as<int32_t>(), R->factors.as<T>(), Y, R->factor_elems, R->scratch_elems, rg, r, z);
}

// Rows per phase of the ring kernel for this preconditioner: 256 when the ring
// fits with them, else 128 (e.g. 13^4 boxes in FP64), else 64 (14^4 boxes in
// FP64), else 0 (no ring: the kernel with the local vector in global memory).
template <typename T>
static int ring_rows(const ras *R) {
  if (R->ring_ltlz > kApplyThreads) return 0;
  if (ring_lds_bytes<T, 256>(R) <= kRingLdsLimit) return 256;
  if (ring_lds_bytes<T, 128>(R) <= kRingLdsLimit) return 128;
  if (ring_lds_bytes<T, 64>(R) <= kRingLdsLimit) return 64;
  return 0;
}

template <typename T>
static void launch_apply(const ras *R, const double *r, double *z, T *Y, hipStream_t s) {
  const int kr = ring_rows<T>(R);
  if (kr == 256) {
    launch_ring<T, 256>(R, r, z, Y, ring_lds_bytes<T, 256>(R), s);
  } else if (kr == 128) {
    launch_ring<T, 128>(R, r, z, Y, ring_lds_bytes<T, 128>(R), s);
  } else if (kr == 64) {
    launch_ring<T, 64>(R, r, z, Y, ring_lds_bytes<T, 64>(R), s);
  } else {
    hipLaunchKernelGGL((apply_kernel<T>), dim3(R->nsub), dim3(kApplyThreads), 0, s, R->d, R->d_subs.as<SubInfo>(),
                       R->d_order.as<int32_t>(), R->d_shapes.as<ShapeInfo>(), R->d_lvl.as<int32_t>(),
                       R->d_coords.as<uint64_t>(), R->d_ctab.as<int32_t>(), R->factors.as<T>(), Y,
                       R->factor_elems, R->scratch_elems, r, z);
  }
}

size_t ras_local_bytes(const ras *R) {
  if (R->iluk) return iluk_local_bytes(R);
  const size_t esz = R->params.precision == STKKT_F32 ? sizeof(float) : sizeof(double);
  return esz * ((size_t)R->scratch_elems + 4);
}

bool ras_uses_ring(const ras *R) {
  if (R->iluk) return false;
  return (R->params.precision == STKKT_F32 ? ring_rows<float>(R) : ring_rows<double>(R)) == 256;
}

int ras_apply_rows_per_phase(const ras *R) {
  if (R->iluk) return 0;
  return R->params.precision == STKKT_F32 ? ring_rows<float>(R) : ring_rows<double>(R);
}

void ras_apply_device(const ras *R, const double *r, double *z, hipStream_t s, void *local) {
  if (R->iluk) {
    iluk_apply(R, r, z, local, s);
    return;
  }
  if (R->params.precision == STKKT_F32)
    launch_apply<float>(R, r, z, local ? static_cast<float *>(local) : R->scratch.as<float>(), s);
  else
    launch_apply<double>(R, r, z, local ? static_cast<double *>(local) : R->scratch.as<double>(), s);
  STKKT_HIP(hipGetLastError());
}

template <typename T>
static void ras_batch_prepare_t(const ras *const *R, const long long *voff, void *const *local, int count,
                                const std::vector<char> &solo, const Allocator *al, RasBatch &out, hipStream_t s) {
  std::vector<RasBatchDesc<T>> d(count);
  std::vector<std::pair<int64_t, int2>> items;
  size_t lds = 0;
  for (int i = 0; i < count; ++i) {
    const ras *q = R[i];
    d[i] = RasBatchDesc<T>{};
    if (!q || solo[i]) continue;   // empty slot, or launched on its own
    d[i].op = q->d;
    d[i].subs = q->d_subs.as<SubInfo>();
    d[i].shapes = q->d_shapes.as<ShapeInfo>();
    d[i].lvl = q->d_lvl.as<int32_t>();
    d[i].coords = q->d_coords.as<uint64_t>();
    d[i].ctab = q->d_ctab.as<int32_t>();
    d[i].tz = q->d_tz.as<int32_t>();
    d[i].F = q->factors.as<T>();
    d[i].Y = local && local[i] ? static_cast<T *>(local[i]) : q->scratch.as<T>();
    d[i].fzero = q->factor_elems;
    d[i].yzero = q->scratch_elems;
    d[i].voff = voff[i];
    d[i].rg = Ring{q->ring_rmax, q->ring_ltlz};
    lds = std::max(lds, out.kr == 256   ? ring_lds_bytes<T, 256>(q)
                        : out.kr == 128 ? ring_lds_bytes<T, 128>(q)
                                        : ring_lds_bytes<T, 64>(q));
    for (int k = 0; k < q->nsub; ++k)
      items.push_back({q->shapes[q->subs[k].shape].nblocks, make_int2(i, k)});
  }
  std::stable_sort(items.begin(), items.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
  std::vector<int2> work(items.size());
  for (size_t k = 0; k < items.size(); ++k) work[k] = items[k].second;
  out.desc = DevBuf(al, sizeof(RasBatchDesc<T>) * (size_t)count);
  out.work = DevBuf(al, sizeof(int2) * std::max<size_t>(work.size(), 1));
  STKKT_HIP(hipMemcpyAsync(out.desc.ptr, d.data(), sizeof(RasBatchDesc<T>) * (size_t)count, hipMemcpyHostToDevice, s));
  STKKT_HIP(hipMemcpyAsync(out.work.ptr, work.data(), sizeof(int2) * work.size(), hipMemcpyHostToDevice, s));
  STKKT_HIP(hipStreamSynchronize(s));   // host staging is released on return
  out.blocks = (int)work.size();
  out.lds = lds;
}

// One launch covers every member whose LDS ring fits, with the largest rows
// per phase (256, 128 or 64) that all of them allow (the per-row sums, and
// so the results, are the same for every phase size).  Members without a ring (or with ILU(k) factors)
// are launched on their own after it; members of different precisions make
// every member its own launch.
void ras_batch_prepare(const ras *const *R, const long long *voff, void *const *local, int count,
                       const Allocator *al, RasBatch &out, hipStream_t s) {
  out = RasBatch{};
  out.count = count;
  out.precision = -1;
  bool uniform = true;
  for (int i = 0; i < count; ++i) {
    out.members.push_back(R[i]);
    out.voff.push_back(voff[i]);
    out.local.push_back(local ? local[i] : nullptr);
    if (!R[i]) continue;
    if (out.precision < 0) out.precision = R[i]->params.precision;
    uniform = uniform && R[i]->params.precision == out.precision;
  }
  if (out.precision < 0) out.precision = STKKT_F64;
  if (!uniform) return;   // per-preconditioner launches
  std::vector<char> solo(count, 0);
  int kr = 256;
  bool any = false;
  for (int i = 0; i < count; ++i) {
    if (!R[i]) continue;
    const int rows = ras_apply_rows_per_phase(R[i]);   // 256, 128, 64, or 0 (no ring, ILU(k))
    if (rows == 0) {
      solo[i] = 1;
      out.solo.push_back(i);
    } else {
      any = true;
      kr = std::min(kr, rows);
    }
  }
  if (!any) {   // every member on its own
    out.solo.clear();
    return;
  }
  out.ring = true;
  out.kr = kr;
  if (out.precision == STKKT_F32) ras_batch_prepare_t<float>(R, voff, local, count, solo, al, out, s);
  else ras_batch_prepare_t<double>(R, voff, local, count, solo, al, out, s);
}

template <typename T>
static void ras_batch_launch(const RasBatch &b, const double *r, const double *r2, double *z, const int *act,
                             hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    STKKT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&apply_ring_batch_kernel<T, 256>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRingLdsLimit));
    STKKT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&apply_ring_batch_kernel<T, 128>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRingLdsLimit));
    STKKT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&apply_ring_batch_kernel<T, 64>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRingLdsLimit));
    attr_set = true;
  }
  if (b.kr == 256)
    hipLaunchKernelGGL((apply_ring_batch_kernel<T, 256>), dim3(b.blocks), dim3(kApplyThreads), b.lds, s,
                       b.desc.as<RasBatchDesc<T>>(), b.work.as<int2>(), act, r, r2 ? r2 : r, z);
  else if (b.kr == 128)
    hipLaunchKernelGGL((apply_ring_batch_kernel<T, 128>), dim3(b.blocks), dim3(kApplyThreads), b.lds, s,
                       b.desc.as<RasBatchDesc<T>>(), b.work.as<int2>(), act, r, r2 ? r2 : r, z);
  else
    hipLaunchKernelGGL((apply_ring_batch_kernel<T, 64>), dim3(b.blocks), dim3(kApplyThreads), b.lds, s,
                       b.desc.as<RasBatchDesc<T>>(), b.work.as<int2>(), act, r, r2 ? r2 : r, z);
}

void ras_batch_run(const RasBatch &b, const double *r, double *z, const int *act, const int *act_host,
                   hipStream_t s, const double *r2) {
  if (!b.ring) {
    for (int i = 0; i < b.count; ++i)
      if (act_host[i] && b.members[i])
        ras_apply_device(b.members[i], (act_host[i] == 2 && r2 ? r2 : r) + b.voff[i], z + b.voff[i], s,
                         b.local[i]);
    return;
  }
  if (b.blocks > 0) {
    if (b.precision == STKKT_F32) ras_batch_launch<float>(b, r, r2, z, act, s);
    else ras_batch_launch<double>(b, r, r2, z, act, s);
    STKKT_HIP(hipGetLastError());
  }
  for (const int i : b.solo)
    if (act_host[i])
      ras_apply_device(b.members[i], (act_host[i] == 2 && r2 ? r2 : r) + b.voff[i], z + b.voff[i], s, b.local[i]);
}

static std::vector<int> split(int L, int p) {
  std::vector<int> s(p + 1);
  const int q = L / p, r = L % p;
  for (int k = 0; k <= p; ++k) s[k] = k * q + std::min(k, r);
  return s;
}

template <class V> static void upload(const Allocator *al, DevBuf &buf, const std::vector<V> &host, hipStream_t s) {
  buf = DevBuf(al, std::max<size_t>(sizeof(V) * host.size(), 256));
  if (!host.empty())
    STKKT_HIP(hipMemcpyAsync(buf.ptr, host.data(), sizeof(V) * host.size(), hipMemcpyHostToDevice, s));
}

ras *ras_create(const kkt_op *op, const ras_params_t *rp, hipStream_t s) {
  STKKT_REQUIRE(rp != nullptr, "ras_setup: params is NULL");
  STKKT_REQUIRE(rp->ilu_level >= 0 && rp->ilu_level <= 3, "ras_setup: ilu_level must be 0, 1, 2 or 3");
  STKKT_REQUIRE(rp->precision == STKKT_F64 || rp->precision == STKKT_F32, "ras_setup: bad precision");
  STKKT_REQUIRE(rp->overlap >= 0, "ras_setup: negative overlap");
  const int L[4] = {op->d.nn[0], op->d.nn[1], op->d.nn[2], op->d.M + 1};
  for (int d = 0; d < 4; ++d)
    STKKT_REQUIRE(rp->p[d] >= 1 && rp->p[d] <= L[d], "ras_setup: parts must be in [1, nodes] per dimension");
  auto R = std::make_unique<ras>();
  R->op = op;
  R->al = op->al;
  R->d = op->d;
  R->params = *rp;
  std::vector<int> cut[4];
  for (int d = 0; d < 4; ++d) cut[d] = split(L[d], rp->p[d]);
  const int nsub = rp->p[0] * rp->p[1] * rp->p[2] * rp->p[3];
  R->nsub = nsub;
  std::map<std::tuple<int, int, int, int>, int> shape_id;
  int64_t fb = 0, sb = 0;
  for (int kt = 0; kt < rp->p[3]; ++kt)
    for (int kz = 0; kz < rp->p[2]; ++kz)
      for (int ky = 0; ky < rp->p[1]; ++ky)
        for (int kx = 0; kx < rp->p[0]; ++kx) {
          const int k[4] = {kx, ky, kz, kt};
          int lo[4], hi[4], blo[4], bhi[4], dims[4];
          for (int d = 0; d < 4; ++d) {
            lo[d] = cut[d][k[d]];
            hi[d] = cut[d][k[d] + 1];
            blo[d] = std::max(0, lo[d] - rp->overlap);
            bhi[d] = std::min(L[d], hi[d] + rp->overlap);
            dims[d] = bhi[d] - blo[d];
            STKKT_REQUIRE(dims[d] < 65536, "ras_setup: box too large");
          }
          auto key = std::make_tuple(dims[0], dims[1], dims[2], dims[3]);
          auto it = shape_id.find(key);
          int sid;
          if (it == shape_id.end()) {
            sid = (int)R->shapes.size();
            shape_id[key] = sid;
            R->shapes.push_back(make_shape(dims));
          } else {
            sid = it->second;
          }
          SubInfo si{};
          si.shape = sid;
          for (int d = 0; d < 4; ++d) {
            si.org[d] = blo[d];
            si.olo[d] = lo[d] - blo[d];
            si.ohi[d] = hi[d] - blo[d];
          }
          const ShapeHost &sh = R->shapes[sid];
          si.fbase = fb;
          si.sbase = sb;
          fb += sh.felems;
          R->total_blocks += sh.nblocks;
          sb += 3LL * sh.nlev * sh.dims[3] * sh.dims[2] * sh.dims[1];
          R->subs.push_back(si);
          for (int d = 0; d < 4; ++d) {
            R->boxes.push_back(lo[d]);
          }
          for (int d = 0; d < 4; ++d) R->boxes.push_back(hi[d]);
          for (int d = 0; d < 4; ++d) R->boxes.push_back(blo[d]);
          for (int d = 0; d < 4; ++d) R->boxes.push_back(bhi[d]);
        }
  R->factor_elems = fb;
  R->scratch_elems = sb;
  if (rp->ilu_level > 0) {   // ILU(k): its own pattern, layout and kernels
    R->total_blocks = 0;
    iluk_create(R.get(), op, s);
    return R.release();
  }
  // launch order: largest boxes first, so that the last workgroups to start are the short ones
  std::vector<int32_t> order(nsub);
  for (int i = 0; i < nsub; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return R->shapes[R->subs[a].shape].nblocks > R->shapes[R->subs[b].shape].nblocks;
  });
  // shape tables
  std::vector<ShapeInfo> shinfo;
  std::vector<int32_t> lvl;
  std::vector<uint64_t> crd;
  std::vector<int32_t> ctb;
  std::vector<int32_t> tzp;
  for (auto &sh : R->shapes) {
    ShapeInfo si{};
    for (int d = 0; d < 4; ++d) si.dims[d] = sh.dims[d];
    si.nlev = sh.nlev;
    si.nchunk = sh.nchunk;
    si.rmax = sh.rmax;
    si.vol = sh.vol;
    si.lvl_off = (int64_t)lvl.size();
    si.coord_off = (int64_t)crd.size();
    si.ct_off = (int64_t)ctb.size();
    si.tz_off = (int64_t)tzp.size();
    R->ring_rmax = std::max(R->ring_rmax, sh.rmax);
    R->ring_ltlz = std::max(R->ring_ltlz, sh.dims[3] * sh.dims[2]);
    lvl.insert(lvl.end(), sh.lvl_start.begin(), sh.lvl_start.end());
    crd.insert(crd.end(), sh.coords.begin(), sh.coords.end());
    ctb.insert(ctb.end(), sh.ctab.begin(), sh.ctab.end());
    tzp.insert(tzp.end(), sh.tzpref.begin(), sh.tzpref.end());
    shinfo.push_back(si);
  }
  const Allocator *al = &R->al;
  upload(al, R->d_shapes, shinfo, s);
  upload(al, R->d_lvl, lvl, s);
  upload(al, R->d_coords, crd, s);
  upload(al, R->d_ctab, ctb, s);
  upload(al, R->d_tz, tzp, s);
  upload(al, R->d_order, order, s);
  std::vector<int16_t> pstart;
  std::vector<uint8_t> pairs;
  build_pairs(pstart, pairs);
  DevBuf d_pstart, d_pairs;
  upload(al, d_pstart, pstart, s);
  upload(al, d_pairs, pairs, s);
  const size_t esz = rp->precision == STKKT_F32 ? sizeof(float) : sizeof(double);
  // trailing all-zero sentinels read for neighbours outside a box
  R->factors = DevBuf(al, esz * ((size_t)fb + 16));
  R->scratch = DevBuf(al, esz * ((size_t)sb + 4));
  STKKT_HIP(hipMemsetAsync(static_cast<char *>(R->factors.ptr) + esz * (size_t)fb, 0, esz * 16, s));
  STKKT_HIP(hipMemsetAsync(static_cast<char *>(R->scratch.ptr) + esz * (size_t)sb, 0, esz * 4, s));
  // working buffer: subdomains factored in batches that fit the budget
  size_t budget = (size_t)64 << 30;
  if (const char *e = getenv("STKKT_SETUP_WORK_GB")) budget = (size_t)(atof(e) * (double)(1ull << 30));
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) budget = std::min(budget, free_b / 2);
  DevBuf d_status(al, 256);
  STKKT_HIP(hipMemsetAsync(d_status.ptr, 0, sizeof(int), s));
  int first = 0;
  while (first < nsub) {
    size_t used = 0;
    int last = first;
    while (last < nsub) {
      const size_t need = (size_t)R->shapes[R->subs[last].shape].vol * 729 * sizeof(double);
      if (last > first && used + need > budget) break;
      R->subs[last].wbase = (int64_t)(used / sizeof(double));
      used += need;
      ++last;
    }
    if (first == 0) upload(al, R->d_subs, R->subs, s);
    else STKKT_HIP(hipMemcpyAsync(R->d_subs.ptr, R->subs.data(), sizeof(SubInfo) * R->subs.size(),
                                  hipMemcpyHostToDevice, s));
    DevBuf work(al, used);
    STKKT_REQUIRE(work.ptr != nullptr, "ras_setup: out of memory for the factorisation workspace");
    hipLaunchKernelGGL(factor_kernel, dim3(last - first), dim3(256), 0, s, op->d, R->d_subs.as<SubInfo>(),
                       R->d_shapes.as<ShapeInfo>(), R->d_lvl.as<int32_t>(), R->d_coords.as<uint64_t>(),
                       d_pstart.as<int16_t>(), d_pairs.as<uint8_t>(), first, work.as<double>(),
                       d_status.as<int>());
    STKKT_HIP(hipGetLastError());
    if (rp->precision == STKKT_F32) {
      hipLaunchKernelGGL(compact_kernel<float>, dim3(last - first), dim3(512), 0, s, R->d_subs.as<SubInfo>(),
                         R->d_shapes.as<ShapeInfo>(), R->d_lvl.as<int32_t>(), R->d_coords.as<uint64_t>(),
                         R->d_ctab.as<int32_t>(), first, work.as<double>(),
                         R->factors.as<float>());
    } else {
      hipLaunchKernelGGL(compact_kernel<double>, dim3(last - first), dim3(512), 0, s, R->d_subs.as<SubInfo>(),
                         R->d_shapes.as<ShapeInfo>(), R->d_lvl.as<int32_t>(), R->d_coords.as<uint64_t>(),
                         R->d_ctab.as<int32_t>(), first, work.as<double>(),
                         R->factors.as<double>());
    }
    STKKT_HIP(hipGetLastError());
    STKKT_HIP(hipStreamSynchronize(s));   // the workspace is released at the end of this scope
    first = last;
  }
  int status = 0;
  STKKT_HIP(hipMemcpy(&status, d_status.ptr, sizeof(int), hipMemcpyDeviceToHost));
  if (status != 0) throw Error(STKKT_EBREAKDOWN, "ras_setup: singular 3x3 pivot block in ILU(0)");
  return R.release();
}

void ras_export(const ras *R, int sub, double *out) {
  STKKT_REQUIRE(sub >= 0 && sub < R->nsub, "ras_export_factors: bad subdomain");
  STKKT_REQUIRE(!R->iluk, "ras_export_factors: ILU(k) factors have no 81-slot layout; use ras_export_factors_csr");
  const SubInfo &sd = R->subs[sub];
  const ShapeHost &sh = R->shapes[sd.shape];
  const int64_t nb = sh.felems;
  const bool f32 = R->params.precision == STKKT_F32;
  std::vector<double> buf((size_t)nb);
  if (f32) {
    std::vector<float> tmp((size_t)nb);
    STKKT_HIP(hipMemcpy(tmp.data(), R->factors.as<float>() + sd.fbase, sizeof(float) * tmp.size(),
                        hipMemcpyDeviceToHost));
    for (size_t i = 0; i < tmp.size(); ++i) buf[i] = tmp[i];
  } else {
    STKKT_HIP(hipMemcpy(buf.data(), R->factors.as<double>() + sd.fbase, sizeof(double) * buf.size(),
                        hipMemcpyDeviceToHost));
  }
  const int lx = sh.dims[0], ly = sh.dims[1], lz = sh.dims[2];
  const int32_t d32[4] = {sh.dims[0], sh.dims[1], sh.dims[2], sh.dims[3]};
  std::fill(out, out + (size_t)sh.vol * 729, 0.0);
  for (int L = 0; L < sh.nlev; ++L) {
    const int r0 = sh.lvl_start[L], R = sh.lvl_start[L + 1] - r0;
    for (int c = 0; c * 64 < R; ++c)
      for (int s = 0; s < 81; ++s) {
        int dx, dy, dz, dt;
        slot_off(s, dx, dy, dz, dt);
        const size_t i = (((size_t)L * sh.nchunk + c) * 81 + s) * 2;
        const int64_t off9 = sh.ctab[i], cnt = sh.ctab[i + 1];
        int64_t k = 0;
        for (int q = c * 64; q < std::min(R, c * 64 + 64); ++q) {
          int x, y, z, t;
          unpack(sh.coords[r0 + q], x, y, z, t);
          if (!inside(x + dx, y + dy, z + dz, t + dt, d32)) continue;
          const int64_t rho = x + (int64_t)lx * (y + (int64_t)ly * (z + (int64_t)lz * t));
          for (int e = 0; e < 9; ++e) out[rho * 729 + 9 * s + e] = buf[off9 + blk_pos(e, k, cnt)];
          ++k;
        }
        if (k != cnt) throw Error(STKKT_EINVAL, "ras_export_factors: inconsistent layout");
      }
  }
}

int64_t ras_sub_blocks(const ras *R, int sub) {
  STKKT_REQUIRE(sub >= 0 && sub < R->nsub, "ras_subdomain_blocks: bad subdomain");
  if (R->iluk) return iluk_subdomain_blocks(R, sub);
  return R->shapes[R->subs[sub].shape].nblocks;
}

void ras_export_csr(const ras *R, int sub, int32_t *indptr, int32_t *indices, double *blocks) {
  STKKT_REQUIRE(sub >= 0 && sub < R->nsub, "ras_export_factors_csr: bad subdomain");
  if (R->iluk) {
    iluk_export_csr(R, sub, indptr, indices, blocks);
    return;
  }
  const ShapeHost &sh = R->shapes[R->subs[sub].shape];
  std::vector<double> pad((size_t)sh.vol * 729);
  ras_export(R, sub, pad.data());
  const int lx = sh.dims[0], ly = sh.dims[1], lz = sh.dims[2];
  const int32_t d32[4] = {sh.dims[0], sh.dims[1], sh.dims[2], sh.dims[3]};
  int64_t k = 0;
  indptr[0] = 0;
  for (int rho = 0; rho < sh.vol; ++rho) {
    const int x = rho % lx, y = (rho / lx) % ly, z = (rho / (lx * ly)) % lz, t = rho / (lx * ly * lz);
    for (int s = 0; s < 81; ++s) {   // ascending slot = ascending column
      int dx, dy, dz, dt;
      slot_off(s, dx, dy, dz, dt);
      if (!inside(x + dx, y + dy, z + dz, t + dt, d32)) continue;
      indices[k] = (x + dx) + lx * ((y + dy) + ly * ((z + dz) + lz * (t + dt)));
      for (int e = 0; e < 9; ++e) blocks[9 * k + e] = pad[(size_t)rho * 729 + 9 * s + e];
      ++k;
    }
    indptr[rho + 1] = (int32_t)k;
  }
}

}  // namespace stkkt
