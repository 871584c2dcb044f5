// Two-level space-time preconditioner (Section 3.2, two-level paragraph):
// nested coarse space-time mesh, linear interpolation I_c^h and its transpose
// (or injection) as transfers, and the coarse KKT system rediscretised on the
// coarse mesh.  F_c^{-1} is applied either as in the paper's experiments
// (Section 4): a few steps of restarted GMRES from zero, right-preconditioned
// by the one-level space-time RAS of the coarse mesh; or exactly, by block
// elimination in time with explicitly inverted Schur complements (CoarseLU).
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "coarse.hpp"
#include "coarse_lu.hpp"
#include "ras.hpp"

struct coarse {
  stkkt::Allocator al;
  const kkt_op *fine_op = nullptr;   // identity only
  stkkt::OpDev fine{};
  int fac[4] = {1, 1, 1, 1};
  coarse_params_t params{};
  kkt_op *cop = nullptr;    // owned coarse operator
  ras *cras = nullptr;      // owned coarse preconditioner
  stkkt::DevBuf xc, yc;     // coarse vectors
  stkkt::DevBuf rt[2];      // intermediate vectors of the axis-by-axis restriction
  // coarse vectors of several right-hand sides (exact coarse solve), grown on demand
  mutable stkkt::DevBuf xcm, ycm;
  mutable int mcap = 0;
  std::unique_ptr<stkkt::GmresWork> work;   // inner GMRES workspace
  std::unique_ptr<stkkt::CoarseLU> lu;       // exact coarse solve (method LU)
  ~coarse() {
    lu.reset();
    work.reset();
    delete cras;
    delete cop;
  }
};

namespace stkkt {

namespace {

// 1-D linear interpolation weight of coarse node I at fine node i (factor f,
// rf = 1 / f): (f - |i - I f|) / f inside the support, else 0.
__device__ inline double hat(int i, int I, int f, double rf) {
  const int d = i - I * f;
  const int ad = d < 0 ? -d : d;
  return ad >= f ? 0.0 : (double)(f - ad) * rf;
}

// y_fine = I_c^h x_coarse: every fine node interpolates the (up to 16) coarse
// nodes of the coarse space-time cell that contains it (the interpolation is
// the tensor product of the 1-D hat functions).  A workgroup owns the fine
// lines (nodes (., i1, i2, n), components innermost) of one coarse (y, z)
// cell group at one time level: i1 in [g1 fy, g1 fy + fy), i2 in
// [g2 fz, g2 fz + fz) (the last group of an axis is its last node alone).
// Such lines need the coarse lines (lo1 + b1, lo2 + b2) of levels lo3 + b3,
// b = 0, 1 (lo = g, lo3 = n / ft), and the work is done in three passes over
// LDS:
//   V[b1][b2][t] = sum_b3 hat_t(n, lo3 + b3) xc[lo3 + b3, lo1 + b1, lo2 + b2][t]
//   U[line][t]   = sum_b2 hat_z(i2, lo2 + b2) sum_b1 hat_y(i1, lo1 + b1) V[b1][b2][t]
//   y[line][3 i0 + c] = hat_x(i0, lo0) U[line][3 lo0 + c] + hat_x(i0, lo0 + 1) U[line][3 lo0 + 3 + c]
// (t runs over the 3 x coarse-x entries of a coarse line).  The x weights and
// U positions of the 3 nn0 fine entries, and the y / z weights of the lines,
// are tabulated in LDS first.  The output pass runs over (line, entry) pairs
// with the entry innermost, so that lines of consecutive i1 (adjacent in
// memory) are written as one stream.  Lines go through U in batches of at
// most `lb` lines.
struct ProlongEntry {
  double w0, w1;   // hat_x(i0, lo0), hat_x(i0, lo0 + 1) (0 when i0 sits on a coarse node)
  int u0, pad;     // 3 lo0 + c
};
static_assert(sizeof(ProlongEntry) == 3 * sizeof(double), "ProlongEntry takes three doubles of LDS");

__global__ void __launch_bounds__(256) prolong_kernel(OpDev fo, OpDev co, int fx, int fy, int fz, int ft, int lb,
                                                      const double *__restrict__ xc, double *__restrict__ y) {
  extern __shared__ double pro_lds[];
  const int gy = (fo.nn[1] - 1) / fy + 1, gz = (fo.nn[2] - 1) / fz + 1;
  const int g1 = blockIdx.x % gy, g2 = (blockIdx.x / gy) % gz, n = blockIdx.x / (gy * gz);
  const int clen = 3 * co.nn[0], len = 3 * fo.nn[0];
  const int ly = min(fy, fo.nn[1] - g1 * fy), lz = min(fz, fo.nn[2] - g2 * fz);
  const int cy = ly > 1 ? 2 : 1, cz = lz > 1 ? 2 : 1;   // coarse y / z lines in use
  const int nl = ly * lz;
  const int lo3 = n / ft, ct = n % ft == 0 ? 1 : 2;
  const double rx = 1.0 / fx, ry = 1.0 / fy, rz = 1.0 / fz, rt = 1.0 / ft;
  const double wt0 = hat(n, lo3, ft, rt), wt1 = ct > 1 ? hat(n, lo3 + 1, ft, rt) : 0.0;
  ProlongEntry *ent = reinterpret_cast<ProlongEntry *>(pro_lds);   // [len]
  double *wl = pro_lds + 3 * len;   // [nl][4]: hat_y(i1, lo1 + b1), hat_z(i2, lo2 + b2)
  double *V = wl + 4 * nl;          // [4][clen]
  double *U = V + 4 * clen;         // [lb][clen]
  for (int t = threadIdx.x; t < len; t += blockDim.x) {
    const int i0 = t / 3, c = t - 3 * i0, lo0 = i0 / fx;
    ProlongEntry e;
    e.w0 = hat(i0, lo0, fx, rx);
    e.w1 = i0 % fx != 0 ? hat(i0, lo0 + 1, fx, rx) : 0.0;
    e.u0 = 3 * lo0 + c;
    e.pad = 0;
    ent[t] = e;
  }
  for (int l = threadIdx.x; l < nl; l += blockDim.x) {
    const int i1 = g1 * fy + l % ly, i2 = g2 * fz + l / ly;
    wl[4 * l] = hat(i1, g1, fy, ry);
    wl[4 * l + 1] = cy > 1 ? hat(i1, g1 + 1, fy, ry) : 0.0;
    wl[4 * l + 2] = hat(i2, g2, fz, rz);
    wl[4 * l + 3] = cz > 1 ? hat(i2, g2 + 1, fz, rz) : 0.0;
  }
  for (int k = threadIdx.x; k < cy * cz * clen; k += blockDim.x) {
    const int t = k % clen, b = k / clen, b1 = b % cy, b2 = b / cy;
    const long long cl = (long long)co.nn[0] * ((g1 + b1) + (long long)co.nn[1] * (g2 + b2));
    double v = wt0 * xc[3 * ((long long)lo3 * co.N + cl) + t];
    if (ct > 1) v += wt1 * xc[3 * ((long long)(lo3 + 1) * co.N + cl) + t];
    V[(b2 * 2 + b1) * clen + t] = v;
  }
  for (int l0 = 0; l0 < nl; l0 += lb) {
    const int nb = min(lb, nl - l0);
    __syncthreads();   // tables and V written (first batch), U free (later batches)
    for (int k = threadIdx.x; k < nb * clen; k += blockDim.x) {
      const int lq = k / clen, t = k - lq * clen;
      const double *w = wl + 4 * (l0 + lq);
      double u = w[2] * (w[0] * V[t] + (cy > 1 ? w[1] * V[clen + t] : 0.0));
      if (cz > 1) u += w[3] * (w[0] * V[2 * clen + t] + (cy > 1 ? w[1] * V[3 * clen + t] : 0.0));
      U[k] = u;
    }
    __syncthreads();
    // (line, entry) pairs of this thread, advanced without divisions
    const int dq = blockDim.x / len, dt = blockDim.x - dq * len;
    int lq = threadIdx.x / len, t = threadIdx.x - lq * len;
    for (; lq < nb;) {
      const int l = l0 + lq;
      const int i1 = g1 * fy + l % ly, i2 = g2 * fz + l / ly;
      const ProlongEntry e = ent[t];
      const double *u = U + lq * clen;
      double v = e.w0 * u[e.u0];
      if (e.w1 != 0.0) v += e.w1 * u[e.u0 + 3];
      y[(((long long)n * fo.nn[2] + i2) * fo.nn[1] + i1) * len + t] = v;
      lq += dq;
      t += dt;
      if (t >= len) {
        t -= len;
        ++lq;
      }
    }
  }
}

// x_coarse = injection of x_fine (the fine value at every coarse node)
__global__ void inject_kernel(OpDev fo, OpDev co, int fx, int fy, int fz, int ft, const double *__restrict__ x,
                              double *__restrict__ xc) {
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < co.V;
       g += (long long)gridDim.x * blockDim.x) {
    const int n = (int)(g / co.N);
    const long long j = g - (long long)n * co.N;
    const int I0 = (int)(j % co.nn[0]), I1 = (int)((j / co.nn[0]) % co.nn[1]),
              I2 = (int)(j / ((long long)co.nn[0] * co.nn[1]));
    const long long fg =
        3 * ((long long)(n * ft) * fo.N + I0 * fx + (long long)fo.nn[0] * (I1 * fy + (long long)fo.nn[1] * (I2 * fz)));
    xc[3 * g] = x[fg];
    xc[3 * g + 1] = x[fg + 1];
    xc[3 * g + 2] = x[fg + 2];
  }
}

// One axis of the transposed interpolation (the restriction is the tensor
// product of the 1-D ones, so it is applied axis by axis): `out` has the node
// counts `din` of `in` with axis d coarsened by f (D -> (D - 1) / f + 1),
// components innermost, and out[.., I, .., c] = sum over the fine nodes p of
// the support of coarse node I of hat(p, I, f) in[.., p, .., c], p ascending.
// One wavefront per output line (fixed node coordinates on axes 1..3; x and
// the component vary along the line, contiguous in memory; four lines per
// workgroup).
struct Dims4 {
  int n[4];
};

__global__ void __launch_bounds__(256) restrict_axis_kernel(Dims4 din, int d, int f, const double *__restrict__ in,
                                                            double *__restrict__ out) {
  int dout[4];
  for (int k = 0; k < 4; ++k) dout[k] = din.n[k];
  dout[d] = (din.n[d] - 1) / f + 1;
  const int lines = dout[1] * dout[2] * dout[3];
  const int lin = 3 * din.n[0], lout = 3 * dout[0];
  const double rf = 1.0 / f;
  const int lane = threadIdx.x & 63;
  for (int line = blockIdx.x * 4 + (threadIdx.x >> 6); line < lines; line += gridDim.x * 4) {
    double *orow = out + (long long)line * lout;
    if (d == 0) {   // (x lines too long for restrict_x_kernel's LDS)
      const double *irow = in + (long long)line * lin;   // axes 1..3 unchanged
      for (int t = lane; t < lout; t += 64) {
        const int I = t / 3, c = t - 3 * I;
        const int lo = max(0, I * f - f + 1), hi = min(din.n[0] - 1, I * f + f - 1);
        double acc = 0.0;
        for (int p = lo; p <= hi; ++p) acc += hat(p, I, f, rf) * irow[3 * p + c];
        orow[t] = acc;
      }
      continue;
    }
    // input line of node p on axis d: the output line's coordinates with axis d set to p
    const int o1 = line % dout[1], o2 = (line / dout[1]) % dout[2], o3 = line / (dout[1] * dout[2]);
    const int I = d == 1 ? o1 : d == 2 ? o2 : o3;
    const long long step = d == 1 ? 1 : d == 2 ? din.n[1] : (long long)din.n[1] * din.n[2];
    const long long line0 = o1 + (long long)din.n[1] * (o2 + (long long)din.n[2] * o3) - (long long)I * step;
    const int lo = max(0, I * f - f + 1), hi = min(din.n[d] - 1, I * f + f - 1);
    for (int t = lane; t < lout; t += 64) {
      double acc = 0.0;
      for (int p = lo; p <= hi; ++p) acc += hat(p, I, f, rf) * in[(line0 + p * step) * lin + t];
      orow[t] = acc;
    }
  }
}

// The x axis of the restriction (d = 0 above): lines are unchanged and
// contiguous, so a workgroup reads kRxLines consecutive input lines into LDS
// with one coalesced stream and forms all their outputs from there,
// out[line][3 I + c] = sum over p of hat(p, I, f) in[line][3 p + c].
constexpr int kRxLines = 16;

__global__ void __launch_bounds__(256) restrict_x_kernel(int nx, int lines, int f, const double *__restrict__ in,
                                                         double *__restrict__ out) {
  extern __shared__ double rx_lds[];
  const int lin = 3 * nx, cx = (nx - 1) / f + 1, lout = 3 * cx;
  const double rf = 1.0 / f;
  const int l0 = blockIdx.x * kRxLines, nl = min(kRxLines, lines - l0);
  const double *src = in + (long long)l0 * lin;
  for (int k = threadIdx.x; k < nl * lin; k += blockDim.x) rx_lds[k] = src[k];
  __syncthreads();
  double *dst = out + (long long)l0 * lout;
  for (int k = threadIdx.x; k < nl * lout; k += blockDim.x) {
    const int lq = k / lout, t = k - lq * lout;
    const int I = t / 3, c = t - 3 * I;
    const int lo = max(0, I * f - f + 1), hi = min(nx - 1, I * f + f - 1);
    const double *row = rx_lds + lq * lin + c;
    double acc = 0.0;
    for (int p = lo; p <= hi; ++p) acc += hat(p, I, f, rf) * row[3 * p];
    dst[k] = acc;
  }
}

}  // namespace

// Prolongation launch: one workgroup per (y group, z group, time level); U
// batches sized so that V and U take at most 32 KB of LDS (the x-entry and
// line tables come on top: 24 B per fine x entry, 32 B per line).
static void prolong(const coarse *C, const double *xc, double *y, hipStream_t s) {
  const OpDev &fo = C->fine, &co = C->cop->d;
  const int fy = C->fac[1], fz = C->fac[2];
  const int gy = (fo.nn[1] - 1) / fy + 1, gz = (fo.nn[2] - 1) / fz + 1;
  const long long blocks = (long long)gy * gz * (fo.M + 1);
  STKKT_REQUIRE(blocks < (1LL << 31), "coarse_apply: fine mesh too large for the prolongation grid");
  const int clen = 3 * co.nn[0], len = 3 * fo.nn[0];
  const int lb = std::max(1, std::min(fy * fz, (int)(4096 / clen) - 4));
  const size_t lds = sizeof(double) * ((size_t)3 * len + 4 * (size_t)fy * fz + (size_t)(4 + lb) * clen);
  constexpr size_t kLdsMax = 160 * 1024;
  STKKT_REQUIRE(lds <= kLdsMax, "coarse_apply: fine x line too long for the prolongation kernel");
  static bool attr_set = false;
  if (!attr_set) {
    STKKT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&prolong_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax));
    attr_set = true;
  }
  hipLaunchKernelGGL(prolong_kernel, dim3((unsigned)blocks), dim3(256), lds, s, fo, co, C->fac[0], fy, fz, C->fac[3],
                     lb, xc, y);
}

// xc = (I_c^h)^T x, axis by axis (x, y, z, t; axes with factor 1 are skipped)
static void restrict_transpose(const coarse *C, const double *x, double *xc, hipStream_t s) {
  const OpDev &fo = C->fine;
  Dims4 dm{{fo.nn[0], fo.nn[1], fo.nn[2], fo.M + 1}};
  int axes[4], na = 0;
  for (int d = 0; d < 4; ++d)
    if (C->fac[d] > 1) axes[na++] = d;
  if (na == 0) {
    STKKT_HIP(hipMemcpyAsync(xc, x, sizeof(double) * 3 * fo.V, hipMemcpyDeviceToDevice, s));
    return;
  }
  const double *src = x;
  for (int k = 0; k < na; ++k) {
    const int d = axes[k];
    double *dst = k == na - 1 ? xc : C->rt[k & 1].as<double>();
    Dims4 out = dm;
    out.n[d] = (dm.n[d] - 1) / C->fac[d] + 1;
    const int lines = out.n[1] * out.n[2] * out.n[3];
    const size_t xlds = sizeof(double) * kRxLines * 3 * (size_t)dm.n[0];
    if (d == 0 && xlds <= 64 * 1024)
      hipLaunchKernelGGL(restrict_x_kernel, dim3((lines + kRxLines - 1) / kRxLines), dim3(256), xlds, s, dm.n[0], lines,
                         C->fac[0], src, dst);
    else
      hipLaunchKernelGGL(restrict_axis_kernel, dim3(std::min((lines + 3) / 4, 1 << 20)), dim3(256), 0, s, dm, d,
                         C->fac[d], src, dst);
    dm = out;
    src = dst;
  }
  STKKT_HIP(hipGetLastError());
}

// xc = I_h^c x: the transposed interpolation or injection
static void restrict_to_coarse(const coarse *C, const double *x, double *xc, hipStream_t s) {
  if (C->params.restrict_kind == STKKT_RESTRICT_INJECTION) {
    const OpDev &fo = C->fine, &co = C->cop->d;
    hipLaunchKernelGGL(inject_kernel, dim3(blocks_for(co.V, 256, 8192)), dim3(256), 0, s, fo, co, C->fac[0],
                       C->fac[1], C->fac[2], C->fac[3], x, xc);
    STKKT_HIP(hipGetLastError());
  } else {
    restrict_transpose(C, x, xc, s);
  }
}

coarse *coarse_create(const kkt_op *fine, const coarse_params_t *cp, hipStream_t s) {
  STKKT_REQUIRE(cp->method == STKKT_COARSE_GMRES_RAS || cp->method == STKKT_COARSE_LU,
                "coarse_setup: unknown coarse solver");
  STKKT_REQUIRE(cp->precision == STKKT_F64 || cp->precision == STKKT_F32, "coarse_setup: bad precision");
  STKKT_REQUIRE(cp->restrict_kind == STKKT_RESTRICT_TRANSPOSE || cp->restrict_kind == STKKT_RESTRICT_INJECTION,
                "coarse_setup: bad restriction");
  if (cp->method == STKKT_COARSE_GMRES_RAS)
    STKKT_REQUIRE(cp->maxit >= 1 && cp->rtol > 0 && cp->rtol < 1, "coarse_setup: bad coarse solver settings");
  const OpDev &fd = fine->d;
  const int nf[4] = {fd.n[0], fd.n[1], fd.n[2], fd.M};
  for (int d = 0; d < 4; ++d)
    STKKT_REQUIRE(cp->factor[d] >= 1 && nf[d] % cp->factor[d] == 0,
                  "coarse_setup: coarsening factors must divide the element counts and nt");
  auto C = std::make_unique<coarse>();
  C->al = fine->al;
  C->fine = fd;
  C->fine_op = fine;
  C->params = *cp;
  for (int d = 0; d < 4; ++d) C->fac[d] = cp->factor[d];
  // coarse problem: same model, coarse mesh, averaged element coefficients
  kkt_problem_t p{};
  const int nc[3] = {fd.n[0] / cp->factor[0], fd.n[1] / cp->factor[1], fd.n[2] / cp->factor[2]};
  for (int d = 0; d < 3; ++d) {
    p.n[d] = nc[d];
    p.len[d] = fine->len[d];
    p.v[d] = fd.v[d];
  }
  p.nt = fd.M / cp->factor[3];
  p.T = fine->T;
  std::vector<double> ac((size_t)nc[0] * nc[1] * nc[2], 0.0);
  const int f0 = cp->factor[0], f1 = cp->factor[1], f2 = cp->factor[2];
  for (int ez = 0; ez < fd.n[2]; ++ez)
    for (int ey = 0; ey < fd.n[1]; ++ey)
      for (int ex = 0; ex < fd.n[0]; ++ex)
        ac[(ex / f0) + (size_t)nc[0] * ((ey / f1) + (size_t)nc[1] * (ez / f2))] +=
            fine->a_host[ex + (size_t)fd.n[0] * (ey + (size_t)fd.n[1] * ez)];
  for (double &v : ac) v /= (double)(f0 * f1 * f2);
  p.a_elem = ac.data();
  p.beta1 = fd.beta1;
  p.beta2 = fd.beta2;
  std::vector<int32_t> cs;
  for (int32_t j : fine->sensor_node) {
    const int i0 = j % fd.nn[0], i1 = (j / fd.nn[0]) % fd.nn[1], i2 = j / (fd.nn[0] * fd.nn[1]);
    STKKT_REQUIRE(i0 % f0 == 0 && i1 % f1 == 0 && i2 % f2 == 0,
                  "coarse_setup: every sensor must sit on a coarse node");
    cs.push_back((i0 / f0) + (nc[0] + 1) * ((i1 / f1) + (nc[1] + 1) * (i2 / f2)));
  }
  std::vector<double> zeros((size_t)(p.nt + 1) * cs.size(), 0.0);
  p.n_sensors = (int32_t)cs.size();
  p.sensor_node = cs.data();
  p.data = zeros.data();
  p.dirichlet_faces = fd.faces;
  p.variant = fd.variant;
  p.regularization = fd.reg;
  kkt_alloc_t al = fine->al.cb;
  C->cop = op_create(&p, al.alloc ? &al : nullptr, s);
  STKKT_REQUIRE(C->cop->d.nn[0] <= 512, "coarse_setup: more than 512 coarse nodes along x");
  const size_t nvc = 3 * (size_t)C->cop->d.V;
  C->xc = DevBuf(&C->al, sizeof(double) * nvc);
  C->yc = DevBuf(&C->al, sizeof(double) * nvc);
  {
    // the restriction's intermediates: sizes after the first and second coarsened axes
    long long dm[4] = {fd.nn[0], fd.nn[1], fd.nn[2], fd.M + 1}, sz[2] = {1, 1};
    int k = 0;
    for (int d = 0; d < 4 && k < 2; ++d)
      if (cp->factor[d] > 1) {
        dm[d] = (dm[d] - 1) / cp->factor[d] + 1;
        sz[k++] = 3 * dm[0] * dm[1] * dm[2] * dm[3];
      }
    C->rt[0] = DevBuf(&C->al, sizeof(double) * sz[0]);
    C->rt[1] = DevBuf(&C->al, sizeof(double) * sz[1]);
  }
  if (cp->method == STKKT_COARSE_LU) {
    C->lu = std::make_unique<CoarseLU>(&C->al, C->cop, cp->precision, s);
  } else {
    ras_params_t rp{};
    for (int d = 0; d < 4; ++d) rp.p[d] = cp->p[d];
    rp.overlap = cp->overlap;
    rp.precision = cp->precision;
    rp.ilu_level = 0;
    C->cras = ras_create(C->cop, &rp, s);
    C->work = std::make_unique<GmresWork>(&C->cop->al, (long long)nvc, cp->maxit, false, false);
  }
  return C.release();
}

void coarse_apply_device(const coarse *C, const double *x, double *y, hipStream_t s) {
  const OpDev &fo = C->fine, &co = C->cop->d;
  restrict_to_coarse(C, x, C->xc.as<double>(), s);
  if (C->lu) {
    const long long nvc = 3 * co.V;
    if (C->lu->one_vector_on_mfma()) C->lu->solve_multi(1, C->xc.as<double>(), nvc, C->yc.as<double>(), nvc, s);
    else C->lu->solve(C->xc.as<double>(), C->yc.as<double>(), s);
  } else {
    fill_zero(C->yc.as<double>(), 3 * co.V, s);
    solve_params_t sp{};
    sp.restart = C->params.maxit;
    sp.maxit = C->params.maxit;
    sp.rtol = C->params.rtol;
    sp.flexible = 0;
    sp.fixed_iters = 0;
    const int st = gmres_solve(C->cop, C->cras, nullptr, sp, C->xc.as<double>(), C->yc.as<double>(), s, nullptr,
                               C->work.get());
    if (st != STKKT_OK && st != STKKT_NOT_CONVERGED) throw Error(st, "coarse solve failed");
  }
  prolong(C, C->yc.as<double>(), y, s);
  STKKT_HIP(hipGetLastError());
}

void coarse_apply_multi_device(const coarse *C, int q, const double *const *x, double *const *y, hipStream_t s) {
  if (q <= 0) return;
  if (!C->lu) {
    for (int i = 0; i < q; ++i) coarse_apply_device(C, x[i], y[i], s);
    return;
  }
  const OpDev &fo = C->fine, &co = C->cop->d;
  const long long nvc = 3 * co.V;
  if (q > C->mcap) {
    STKKT_HIP(hipStreamSynchronize(s));   // launches already queued may still use the old vectors
    C->xcm = DevBuf(&C->al, sizeof(double) * (size_t)nvc * q);
    C->ycm = DevBuf(&C->al, sizeof(double) * (size_t)nvc * q);
    C->mcap = q;
  }
  double *xc = C->xcm.as<double>(), *yc = C->ycm.as<double>();
  for (int i = 0; i < q; ++i) restrict_to_coarse(C, x[i], xc + i * nvc, s);
  C->lu->solve_multi(q, xc, nvc, yc, nvc, s);
  for (int i = 0; i < q; ++i) prolong(C, yc + i * nvc, y[i], s);
  STKKT_HIP(hipGetLastError());
}

void coarse_apply_strided(const coarse *C, int q, const double *x, long long ldx, double *y, long long ldy,
                          hipStream_t s) {
  const long long n = 3 * C->fine.V;
  STKKT_REQUIRE(q >= 0, "coarse_apply_multi: q must be >= 0");
  if (q == 0) return;
  STKKT_REQUIRE(ldx >= n && ldy >= n, "coarse_apply_multi: strides shorter than the fine vector");
  const double *xe = x + (q - 1) * ldx + n;
  const double *ye = y + (q - 1) * ldy + n;
  STKKT_REQUIRE(ye <= x || xe <= y, "coarse_apply_multi: x and y must not overlap");
  std::vector<const double *> xs(q);
  std::vector<double *> ys(q);
  for (int i = 0; i < q; ++i) {
    xs[i] = x + i * ldx;
    ys[i] = y + i * ldy;
  }
  coarse_apply_multi_device(C, q, xs.data(), ys.data(), s);
}

void coarse_free(coarse *c) { delete c; }

bool coarse_built_for(const coarse *c, const kkt_op *op) { return c->fine_op == op; }

}  // namespace stkkt
