// One-level space-time restricted additive Schwarz with 3x3 point-block
// ILU(0) subdomain solves (Section 3.2 of the paper: overlapping space-time
// decomposition, subdomain matrices taken from F_h on the extended boxes,
// restricted prolongation of the owned part; Section 4: ILU(0)).
//
// Factor storage ("level-major, slot-major SoA"): for every subdomain, level
// L and stencil slot s (0..80, s = (dx+1) + 3(dy+1) + 9(dz+1) + 27(dt+1);
// s < 40 are the L blocks, s = 40 holds inv(U_rr), s > 40 the U blocks), the
// blocks of the rows of level L that have neighbour s inside the box are
// stored entry-major: value(e, k) at base(L, s) + e * count(L, s) + k, where
// k is the rank of the row among those rows.  A wavefront of 64 consecutive
// rows therefore reads every entry of a slot with one coalesced load, and no
// padding is stored for neighbours outside the box.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <memory>
#include <tuple>

#include "ras.hpp"
#include "stencil.hpp"

namespace stkkt {

namespace {

constexpr int kSeg = 256;       // rows per level segment in the apply kernel
constexpr int kApplyThreads = 512;

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
  sh.blkoff.assign((size_t)sh.nlev * 81 + 1, 0);
  sh.rankbase.assign((size_t)sh.nlev * sh.nchunk * 81, 0);
  int64_t off = 0;
  for (int L = 0; L < sh.nlev; ++L) {
    const int r0 = sh.lvl_start[L], r1 = sh.lvl_start[L + 1];
    for (int s = 0; s < 81; ++s) {
      int dx, dy, dz, dt;
      slot_off(s, dx, dy, dz, dt);
      sh.blkoff[(size_t)L * 81 + s] = off;
      int cnt = 0;
      for (int q = r0; q < r1; ++q) {
        if ((q - r0) % 64 == 0) sh.rankbase[((size_t)L * sh.nchunk + (q - r0) / 64) * 81 + s] = cnt;
        int x, y, z, t;
        unpack(sh.coords[q], x, y, z, t);
        if (inside(x + dx, y + dy, z + dz, t + dt, d32)) ++cnt;
      }
      off += cnt;
    }
  }
  sh.blkoff[(size_t)sh.nlev * 81] = off;
  return sh;
}

// --------------------------------------------------------------------------
// setup: subdomain matrix from the operator formula, then ILU(0), one
// workgroup per subdomain, rows of a level in parallel (one thread per row).
// W holds the subdomain's rows padded to 81 blocks: W[rho][s][e].
// --------------------------------------------------------------------------
__device__ inline void inv33_pivot(const double *a, double *out, bool &ok) {
  double m[3][6];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      m[r][c] = a[3 * r + c];
      m[r][3 + c] = (r == c) ? 1.0 : 0.0;
    }
  ok = true;
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (fabs(m[r][col]) > fabs(m[piv][col])) piv = r;
    if (!(fabs(m[piv][col]) > 0.0)) {
      ok = false;
      return;
    }
    if (piv != col)
      for (int c = 0; c < 6; ++c) {
        double t = m[col][c];
        m[col][c] = m[piv][c];
        m[piv][c] = t;
      }
    const double dinv = 1.0 / m[col][col];
    for (int c = 0; c < 6; ++c) m[col][c] *= dinv;
    for (int r = 0; r < 3; ++r) {
      if (r == col) continue;
      const double f = m[r][col];
      for (int c = 0; c < 6; ++c) m[r][c] -= f * m[col][c];
    }
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) out[3 * r + c] = m[r][3 + c];
}

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
                                                      const int64_t *__restrict__ blkoff,
                                                      const int32_t *__restrict__ rankbase, int sub0,
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
          const int rank = rankbase[sh.rank_off + ((int64_t)L * sh.nchunk + c) * 81 + s] + (int)lanes_below(mask);
          const int64_t b0 = blkoff[sh.blk_off + (int64_t)L * 81 + s];
          const int64_t cnt = blkoff[sh.blk_off + (int64_t)L * 81 + s + 1] - b0;
          T *dst = F + sd.fbase + 9 * b0 + rank;
          const double *src = Wb + rho * 729 + 9 * s;
          for (int e = 0; e < 9; ++e) dst[e * cnt] = (T)src[e];
        }
      }
    }
  }
}

// --------------------------------------------------------------------------
// apply: z = sum_i (R^0_i)^T U_i^{-1} L_i^{-1} R^delta_i r
// One workgroup (8 wavefronts) per subdomain runs the forward sweep over the
// levels, then the backward sweep.  For each level, work items are (chunk of
// 64 rows, group of 10 slots); partial products go to LDS and are summed in a
// fixed order, so results are reproducible run to run.
// --------------------------------------------------------------------------
template <typename T, bool kForward>
__device__ inline void sweep_level(const SubInfo &sd, const ShapeInfo &sh, int L, int r0, int R, OpDev op,
                                   const uint64_t *__restrict__ coords, const int64_t *__restrict__ blkoff,
                                   const int32_t *__restrict__ rankbase, const T *__restrict__ F, T *__restrict__ Y,
                                   const double *__restrict__ r, double *__restrict__ z, T (*part)[kSeg][3]) {
  const int lx = sh.dims[0], ly = sh.dims[1], lz = sh.dims[2];
  const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
  constexpr int nwaves = kApplyThreads / 64;
  const int sbase = kForward ? 0 : 41;
  for (int seg0 = 0; seg0 < R; seg0 += kSeg) {
    const int segR = min(kSeg, R - seg0);
    const int nch = (segR + 63) / 64;
    for (int item = wave; item < nch * 4; item += nwaves) {
      const int cl = item >> 2, g = item & 3;
      const int qq = cl * 64 + lane;
      const int q = seg0 + qq;
      const int c = q >> 6;
      const bool valid = qq < segR;
      int x = 0, y = 0, zc = 0, t = 0;
      if (valid) unpack(coords[sh.coord_off + r0 + q], x, y, zc, t);
      const long long rho = x + (long long)lx * (y + (long long)ly * (zc + (long long)lz * t));
      T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
      for (int j = 0; j < 10; ++j) {
        const int s = sbase + 10 * g + j;
        int dx, dy, dz, dt;
        slot_off(s, dx, dy, dz, dt);
        const bool has = valid && inside(x + dx, y + dy, zc + dz, t + dt, sh.dims);
        const unsigned long long mask = __ballot(has);
        if (has) {
          const int rank = rankbase[sh.rank_off + ((int64_t)L * sh.nchunk + c) * 81 + s] + (int)lanes_below(mask);
          const int64_t b0 = blkoff[sh.blk_off + (int64_t)L * 81 + s];
          const int64_t cnt = blkoff[sh.blk_off + (int64_t)L * 81 + s + 1] - b0;
          const T *f = F + sd.fbase + 9 * b0 + rank;
          const long long rk = rho + dx + (long long)lx * (dy + (long long)ly * (dz + (long long)lz * dt));
          const T *yk = Y + sd.sbase + 3 * rk;
          const T y0 = yk[0], y1 = yk[1], y2 = yk[2];
          a0 += f[0] * y0 + f[cnt] * y1 + f[2 * cnt] * y2;
          a1 += f[3 * cnt] * y0 + f[4 * cnt] * y1 + f[5 * cnt] * y2;
          a2 += f[6 * cnt] * y0 + f[7 * cnt] * y1 + f[8 * cnt] * y2;
        }
      }
      if (valid) {
        part[g][qq][0] = a0;
        part[g][qq][1] = a1;
        part[g][qq][2] = a2;
      }
    }
    __syncthreads();
    for (int qq = (int)threadIdx.x; qq < segR; qq += kApplyThreads) {
      const int q = seg0 + qq;
      int x, y, zc, t;
      unpack(coords[sh.coord_off + r0 + q], x, y, zc, t);
      const long long rho = x + (long long)lx * (y + (long long)ly * (zc + (long long)lz * t));
      T s3[3];
      for (int cc = 0; cc < 3; ++cc) s3[cc] = (part[0][qq][cc] + part[1][qq][cc]) + (part[2][qq][cc] + part[3][qq][cc]);
      const long long node = (sd.org[0] + x) + (long long)op.nn[0] * ((sd.org[1] + y) + (long long)op.nn[1] * (sd.org[2] + zc));
      const long long gi = 3 * ((long long)(sd.org[3] + t) * op.N + node);
      T *yr = Y + sd.sbase + 3 * rho;
      if (kForward) {
        for (int cc = 0; cc < 3; ++cc) yr[cc] = (T)r[gi + cc] - s3[cc];
      } else {
        const int64_t b0 = blkoff[sh.blk_off + (int64_t)L * 81 + 40];
        const T *d = F + sd.fbase + 9 * b0 + q;   // all R rows have slot 40: count = R, rank = q
        T v[3];
        for (int cc = 0; cc < 3; ++cc) v[cc] = yr[cc] - s3[cc];
        T o[3];
        for (int cc = 0; cc < 3; ++cc)
          o[cc] = d[(3 * cc) * (int64_t)R] * v[0] + d[(3 * cc + 1) * (int64_t)R] * v[1] + d[(3 * cc + 2) * (int64_t)R] * v[2];
        for (int cc = 0; cc < 3; ++cc) yr[cc] = o[cc];
        const bool owned = x >= sd.olo[0] && x < sd.ohi[0] && y >= sd.olo[1] && y < sd.ohi[1] && zc >= sd.olo[2] &&
                           zc < sd.ohi[2] && t >= sd.olo[3] && t < sd.ohi[3];
        if (owned)
          for (int cc = 0; cc < 3; ++cc) z[gi + cc] = (double)o[cc];
      }
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void __launch_bounds__(kApplyThreads) apply_kernel(OpDev op, const SubInfo *__restrict__ subs,
                                                              const ShapeInfo *__restrict__ shapes,
                                                              const int32_t *__restrict__ lvl_start,
                                                              const uint64_t *__restrict__ coords,
                                                              const int64_t *__restrict__ blkoff,
                                                              const int32_t *__restrict__ rankbase,
                                                              const T *__restrict__ F, T *__restrict__ Y,
                                                              const double *__restrict__ r, double *__restrict__ z) {
  __shared__ T part[4][kSeg][3];
  const SubInfo sd = subs[blockIdx.x];
  const ShapeInfo sh = shapes[sd.shape];
  for (int L = 0; L < sh.nlev; ++L) {
    const int r0 = lvl_start[sh.lvl_off + L], r1 = lvl_start[sh.lvl_off + L + 1];
    sweep_level<T, true>(sd, sh, L, r0, r1 - r0, op, coords, blkoff, rankbase, F, Y, r, z, part);
  }
  for (int L = sh.nlev - 1; L >= 0; --L) {
    const int r0 = lvl_start[sh.lvl_off + L], r1 = lvl_start[sh.lvl_off + L + 1];
    sweep_level<T, false>(sd, sh, L, r0, r1 - r0, op, coords, blkoff, rankbase, F, Y, r, z, part);
  }
}

}  // namespace

void ras_apply_device(const ras *R, const double *r, double *z, hipStream_t s) {
  if (R->params.precision == STKKT_F32) {
    hipLaunchKernelGGL(apply_kernel<float>, dim3(R->nsub), dim3(kApplyThreads), 0, s, R->d,
                       R->d_subs.as<SubInfo>(), R->d_shapes.as<ShapeInfo>(), R->d_lvl.as<int32_t>(),
                       R->d_coords.as<uint64_t>(), R->d_blkoff.as<int64_t>(), R->d_rank.as<int32_t>(),
                       R->factors.as<float>(), R->scratch.as<float>(), r, z);
  } else {
    hipLaunchKernelGGL(apply_kernel<double>, dim3(R->nsub), dim3(kApplyThreads), 0, s, R->d,
                       R->d_subs.as<SubInfo>(), R->d_shapes.as<ShapeInfo>(), R->d_lvl.as<int32_t>(),
                       R->d_coords.as<uint64_t>(), R->d_blkoff.as<int64_t>(), R->d_rank.as<int32_t>(),
                       R->factors.as<double>(), R->scratch.as<double>(), r, z);
  }
  STKKT_HIP(hipGetLastError());
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
  STKKT_REQUIRE(rp->ilu_level == 0, "ras_setup: only ILU(0) is supported");
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
          fb += 9 * sh.blkoff.back();
          sb += 3LL * sh.vol;
          R->subs.push_back(si);
          for (int d = 0; d < 4; ++d) {
            R->boxes.push_back(lo[d]);
          }
          for (int d = 0; d < 4; ++d) R->boxes.push_back(hi[d]);
          for (int d = 0; d < 4; ++d) R->boxes.push_back(blo[d]);
          for (int d = 0; d < 4; ++d) R->boxes.push_back(bhi[d]);
        }
  R->total_blocks = fb / 9;
  R->scratch_elems = sb;
  // shape tables
  std::vector<ShapeInfo> shinfo;
  std::vector<int32_t> lvl;
  std::vector<uint64_t> crd;
  std::vector<int64_t> blk;
  std::vector<int32_t> rnk;
  for (auto &sh : R->shapes) {
    ShapeInfo si{};
    for (int d = 0; d < 4; ++d) si.dims[d] = sh.dims[d];
    si.nlev = sh.nlev;
    si.nchunk = sh.nchunk;
    si.rmax = sh.rmax;
    si.vol = sh.vol;
    si.lvl_off = (int64_t)lvl.size();
    si.coord_off = (int64_t)crd.size();
    si.blk_off = (int64_t)blk.size();
    si.rank_off = (int64_t)rnk.size();
    lvl.insert(lvl.end(), sh.lvl_start.begin(), sh.lvl_start.end());
    crd.insert(crd.end(), sh.coords.begin(), sh.coords.end());
    blk.insert(blk.end(), sh.blkoff.begin(), sh.blkoff.end());
    rnk.insert(rnk.end(), sh.rankbase.begin(), sh.rankbase.end());
    shinfo.push_back(si);
  }
  const Allocator *al = &R->al;
  upload(al, R->d_shapes, shinfo, s);
  upload(al, R->d_lvl, lvl, s);
  upload(al, R->d_coords, crd, s);
  upload(al, R->d_blkoff, blk, s);
  upload(al, R->d_rank, rnk, s);
  std::vector<int16_t> pstart;
  std::vector<uint8_t> pairs;
  build_pairs(pstart, pairs);
  DevBuf d_pstart, d_pairs;
  upload(al, d_pstart, pstart, s);
  upload(al, d_pairs, pairs, s);
  const size_t esz = rp->precision == STKKT_F32 ? sizeof(float) : sizeof(double);
  R->factors = DevBuf(al, esz * (size_t)fb);
  STKKT_REQUIRE(R->factors.ptr != nullptr || fb == 0, "ras_setup: out of memory for factors");
  R->scratch = DevBuf(al, esz * (size_t)sb);
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
                         R->d_blkoff.as<int64_t>(), R->d_rank.as<int32_t>(), first, work.as<double>(),
                         R->factors.as<float>());
    } else {
      hipLaunchKernelGGL(compact_kernel<double>, dim3(last - first), dim3(512), 0, s, R->d_subs.as<SubInfo>(),
                         R->d_shapes.as<ShapeInfo>(), R->d_lvl.as<int32_t>(), R->d_coords.as<uint64_t>(),
                         R->d_blkoff.as<int64_t>(), R->d_rank.as<int32_t>(), first, work.as<double>(),
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
  const SubInfo &sd = R->subs[sub];
  const ShapeHost &sh = R->shapes[sd.shape];
  const int64_t nb = sh.blkoff.back();
  const bool f32 = R->params.precision == STKKT_F32;
  std::vector<double> buf(9 * (size_t)nb);
  if (f32) {
    std::vector<float> tmp(9 * (size_t)nb);
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
    for (int s = 0; s < 81; ++s) {
      int dx, dy, dz, dt;
      slot_off(s, dx, dy, dz, dt);
      const int64_t b0 = sh.blkoff[(size_t)L * 81 + s], cnt = sh.blkoff[(size_t)L * 81 + s + 1] - b0;
      int64_t k = 0;
      for (int q = sh.lvl_start[L]; q < sh.lvl_start[L + 1]; ++q) {
        int x, y, z, t;
        unpack(sh.coords[q], x, y, z, t);
        if (!inside(x + dx, y + dy, z + dz, t + dt, d32)) continue;
        const int64_t rho = x + (int64_t)lx * (y + (int64_t)ly * (z + (int64_t)lz * t));
        for (int e = 0; e < 9; ++e) out[rho * 729 + 9 * s + e] = buf[9 * b0 + e * cnt + k];
        ++k;
      }
      if (k != cnt) throw Error(STKKT_EINVAL, "ras_export_factors: inconsistent layout");
    }
  }
}

}  // namespace stkkt
