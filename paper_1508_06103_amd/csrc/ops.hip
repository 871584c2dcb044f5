// Operator assembly, right-hand side and the matrix-free space-time matvec.
#include <algorithm>
#include <climits>
#include <mutex>
#include <string>

#include "common.hpp"
#include "stencil.hpp"

namespace stkkt {

// --------------------------------------------------------------------------
// right-hand side: sensor data enter the G-slot rows only
//   DTO: b_G(n, j) = w_n d^n_j        OTD: b_G(n, j) = tau/2 (d^n_j + d^{n+1}_j), n < M
// --------------------------------------------------------------------------
__global__ void fill_zero_kernel(double *p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void rhs_scatter_kernel(OpDev op, const int32_t *sensor_node, int ns, const double *data, double *b) {
  const long long total = (long long)(op.M + 1) * ns;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < total;
       k += (long long)gridDim.x * blockDim.x) {
    const int n = (int)(k / ns), s = (int)(k % ns);
    const long long j = sensor_node[s];
    double val;
    if (op.variant == STKKT_DTO) {
      val = wtrap(op.tau, n, op.M) * data[k];
    } else {
      val = (n < op.M) ? 0.5 * op.tau * (data[k] + data[k + ns]) : 0.0;
    }
    b[3 * ((long long)n * op.N + j) + 1] = val;
  }
}

void fill_zero(double *p, long long n, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, p, n);
  STKKT_HIP(hipGetLastError());
}

void rhs_device(const kkt_op *op, const double *data_host, hipStream_t s, double *b) {
  const int ns = (int)op->sensor_node.size();
  const long long nb = 3LL * op->d.V;
  fill_zero(b, nb, s);
  DevBuf nodes(&op->al, sizeof(int32_t) * ns);
  DevBuf data(&op->al, sizeof(double) * (size_t)(op->d.M + 1) * ns);
  STKKT_HIP(hipMemcpyAsync(nodes.ptr, op->sensor_node.data(), nodes.bytes, hipMemcpyHostToDevice, s));
  STKKT_HIP(hipMemcpyAsync(data.ptr, data_host, data.bytes, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(rhs_scatter_kernel, dim3(blocks_for((long long)(op->d.M + 1) * ns, 256, 4096)), dim3(256), 0, s,
                     op->d, nodes.as<int32_t>(), ns, data.as<double>(), b);
  STKKT_HIP(hipGetLastError());
  // the staging buffers are freed when this returns: wait for the copies
  STKKT_HIP(hipStreamSynchronize(s));
}

// --------------------------------------------------------------------------
// right-hand side without allocation: the sensor ids and the data are staged
// in `scratch`, a device array of this file (one copy per GPU, alive until the
// process ends), instead of buffers from the allocator.  In host code the
// array's name is not a device address; the address comes from
// hipGetSymbolAddress, once per device, and only that pointer is used.
// --------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kRhsScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<unsigned char *> g_scratch_ptr;   // per device; null until looked up

unsigned char *scratch_ptr() {
  int dev = 0;
  STKKT_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    STKKT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(STKKT_EHIP, "kkt_rhs_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

size_t rhs_scratch_need(const kkt_op *op) {
  const size_t ns = op->sensor_node.size();
  const size_t ids = (sizeof(int32_t) * ns + 255) / 256 * 256;
  return ids + sizeof(double) * (size_t)(op->d.M + 1) * ns;
}

void rhs_device_noalloc(const kkt_op *op, const double *data_host, hipStream_t s, double *b) {
  const size_t need = rhs_scratch_need(op);
  if (need > kRhsScratchBytes)
    throw Error(STKKT_EINVAL, "kkt_rhs_noalloc: (nt+1) x n_sensors data need " + std::to_string(need) +
                                  " bytes of staging, more than the " + std::to_string(kRhsScratchBytes) +
                                  " the scratch array holds; use kkt_rhs");
  unsigned char *base = scratch_ptr();
  const int ns = (int)op->sensor_node.size();
  const size_t ids = (sizeof(int32_t) * ns + 255) / 256 * 256;
  int32_t *nodes = reinterpret_cast<int32_t *>(base);
  double *data = reinterpret_cast<double *>(base + ids);
  fill_zero(b, 3LL * op->d.V, s);
  STKKT_HIP(hipMemcpyAsync(nodes, op->sensor_node.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
  STKKT_HIP(hipMemcpyAsync(data, data_host, sizeof(double) * (size_t)(op->d.M + 1) * ns, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(rhs_scatter_kernel, dim3(blocks_for((long long)(op->d.M + 1) * ns, 256, 4096)), dim3(256), 0, s,
                     op->d, nodes, ns, data, b);
  STKKT_HIP(hipGetLastError());
  // the next call on this GPU reuses the scratch array: finish before returning
  STKKT_HIP(hipStreamSynchronize(s));
}

// --------------------------------------------------------------------------
// diffusion coefficient table: A[j, j+d] for the 27 spatial offsets
// (slot k = (dx+1) + 3(dy+1) + 9(dz+1)), zero where the neighbour is outside
// --------------------------------------------------------------------------
__global__ void stiff_table_kernel(OpDev op, double *tab) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < op.N;
       j += (long long)gridDim.x * blockDim.x) {
    const int jx = (int)(j % op.nn[0]);
    const int jy = (int)((j / op.nn[0]) % op.nn[1]);
    const int jz = (int)(j / ((long long)op.nn[0] * op.nn[1]));
    for (int k = 0; k < 27; ++k) {
      const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
      const bool in = jx + dx >= 0 && jx + dx < op.nn[0] && jy + dy >= 0 && jy + dy < op.nn[1] && jz + dz >= 0 &&
                      jz + dz < op.nn[2];
      tab[27 * j + k] = in ? stiff_var(op, jx, jy, jz, dx, dy, dz) : 0.0;
    }
  }
}

void stiff_table(const OpDev &d, double *tab, hipStream_t s) {
  hipLaunchKernelGGL(stiff_table_kernel, dim3(blocks_for(d.N, 128, 4096)), dim3(128), 0, s, d, tab);
  STKKT_HIP(hipGetLastError());
}

// --------------------------------------------------------------------------
// y = F_h x, matrix-free.  Rows follow the block formula of kkt_block_c()
// regrouped by spatial operator.  With P_i = 0 on Dirichlet nodes and 1
// elsewhere, and per node i the combined fields
//   U1 = P (c^n - c^{n-1}) - tau/2 (f^{n-1} + f^n)       S1 = P (c^n + c^{n-1})
//   U2 = P (m g^n - p g^{n+1})                          S2 = P (m g^n + p g^{n+1})
//   U3 = beta1 (St f)^n - { DTO: tau/2 S2 ; OTD: P (Tt g)^n }   T3 = beta2 (Tt f)^n
//   (H1-L2 regularisation: beta2 (Tt f)^n is added to U3 instead and T3 = 0)
// (m = [n >= 1] for DTO and 1 for OTD, p = [n < M]; (St f)^n, (Tt f)^n the
// time stiffness / mass rows of level n), the rows of an interior node j are
//   C (n >= 1):  sum_i B_ji U1_i + tau/2 (A + N)_ji S1_i
//   G:           sum_i B_ji U2_i + tau/2 (A + N^T)_ji S2_i
//                + DTO: [n = 0] g_j^0 + w_n S_j c_j^n ; OTD (n < M): tau/2 S_j (c_j^n + c_j^{n+1})
//   f:           sum_i B_ji U3_i + K_ji T3_i
// and Dirichlet C/G rows, the C row of level 0 and the OTD G row of level M
// are identity rows.
//
// One workgroup owns a TX x TY x TZ tile of spatial nodes over a chunk of
// consecutive time levels and marches through them: every thread keeps the
// raw (c, g, f) of up to KH halo nodes for three consecutive levels in
// registers, loads each level once, writes the six combined fields of its
// halo nodes to LDS, and evaluates the 27-point sums of its own node from
// LDS.  The fields of level n + 1 go to a second buffer while level n's
// sums read the first, so one barrier per level suffices.  The spatial 1-D factors of B, K and N are rebuilt from the node's
// position (end-node rules); the variable-coefficient diffusion A comes from
// the per-node table, read once per chunk into registers.
// --------------------------------------------------------------------------
namespace {

constexpr int kMvThreads = 256;

// Mesh and time constants of the matvec, formed on the host so that the
// kernel never evaluates a product of uniform values in vector registers.
struct MvConst {
  double h6[3], hinv[3];   // h/6 and 1/h per axis (off-centre mass, -stiffness)
  double v[3];
  double cyz[2][2][4];     // corner rows (dy, dz = +-1): myz, kyz, nyz, v0 myz
  double ht, inv_tau, tau6, tau3, beta1, beta2;
  int l2;   // H1-L2 regularisation: beta2 (Tt f) joins U3 (mass) instead of T3 (stiffness)
};

// One operator of a batched matvec: its vectors start at element voff of the
// batch's concatenated vectors.
struct MvBatchDesc {
  OpDev op;
  MvTile tl;
  MvConst mc;
  const double *atab;
  int64_t voff;
  int32_t w0, nw;
};

MvConst make_mv_const(const OpDev &d) {
  MvConst c{};
  for (int a = 0; a < 3; ++a) {
    c.h6[a] = d.h[a] / 6.0;
    c.hinv[a] = 1.0 / d.h[a];
    c.v[a] = d.v[a];
  }
  for (int sy = 0; sy < 2; ++sy)
    for (int sz = 0; sz < 2; ++sz) {
      const double dy = sy ? 1.0 : -1.0, dz = sz ? 1.0 : -1.0;
      const double my = c.h6[1], mz = c.h6[2], ky = -c.hinv[1], kz = -c.hinv[2];
      c.cyz[sy][sz][0] = my * mz;
      c.cyz[sy][sz][1] = ky * mz + my * kz;
      c.cyz[sy][sz][2] = d.v[1] * 0.5 * dy * mz + d.v[2] * my * 0.5 * dz;
      c.cyz[sy][sz][3] = d.v[0] * my * mz;
    }
  c.ht = 0.5 * d.tau;
  c.inv_tau = 1.0 / d.tau;
  c.tau6 = d.tau / 6.0;
  c.tau3 = d.tau / 3.0;
  c.beta1 = d.beta1;
  c.beta2 = d.beta2;
  c.l2 = d.reg == STKKT_REG_H1L2;
  return c;
}

struct Centre {
  double m, k, c;   // centre mass, stiffness and convection entries of the node on one axis
};

__device__ inline Centre axis_centre(const MvConst &mc, int a, int i, int nn) {
  const bool end = (i == 0) || (i == nn - 1);
  Centre r;
  r.m = end ? 2.0 * mc.h6[a] : 4.0 * mc.h6[a];
  r.k = end ? mc.hinv[a] : 2.0 * mc.hinv[a];
  r.c = (i == 0) ? -0.5 : ((i == nn - 1) ? 0.5 : 0.0);
  return r;
}

// Work item of this block such that consecutive work items run on the same
// XCD (the dispatcher deals blocks to the 8 XCDs round robin).
__device__ inline int xcd_work_index() {
  const int G = gridDim.x, b = blockIdx.x;
  const int q = G >> 3, r = G & 7, xcd = b & 7;
  return xcd * q + min(xcd, r) + (b >> 3);
}

// One (tile, time chunk) work item w of one operator.
template <int KH>
__device__ inline void matvec_tile_body(const OpDev &op, const MvTile &tl, const MvConst &mc,
                                        const double *__restrict__ Atab, const double *__restrict__ x,
                                        double *__restrict__ y, int w) {
  // per halo node: {U1, S1}, {U2, S2}, {U3, T3} side by side (48 B)
  extern __shared__ double2 mv_lds[];
  const int tile = w % tl.ntiles, chunk = w / tl.ntiles;
  const int M = op.M;
  const int n0 = chunk * tl.clen, n1 = min(n0 + tl.clen, M + 1);
  const int tix = tile % tl.nt[0], tiy = (tile / tl.nt[0]) % tl.nt[1], tiz = tile / (tl.nt[0] * tl.nt[1]);
  const int ox = tix * tl.t[0], oy = tiy * tl.t[1], oz = tiz * tl.t[2];
  const int hx = tl.t[0] + 2, hy = tl.t[1] + 2;
  const int nn0 = op.nn[0], nn1 = op.nn[1], nn2 = op.nn[2];
  const long long N = op.N;
  const double ht = mc.ht;
  const bool dto = op.variant == STKKT_DTO;

  // own node
  const int t = threadIdx.x;
  const int lx = t % tl.t[0], ly = (t / tl.t[0]) % tl.t[1], lz = t / (tl.t[0] * tl.t[1]);
  const int jx = ox + lx, jy = oy + ly, jz = oz + lz;
  const bool own = t < tl.t[0] * tl.t[1] * tl.t[2] && jx < nn0 && jy < nn1 && jz < nn2;
  const long long j = own ? jx + (long long)nn0 * (jy + (long long)nn1 * jz) : 0;
  double A[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) A[k] = own ? Atab[27 * j + k] : 0.0;
  Centre cx = axis_centre(mc, 0, jx, nn0), cy = axis_centre(mc, 1, jy, nn1), cz = axis_centre(mc, 2, jz, nn2);
  const bool Pj = own && !on_dirichlet(op, jx, jy, jz);
  const double sens = own ? op.sensor[j] : 0.0;
  const int hc = (lx + 1) + hx * ((ly + 1) + hy * (lz + 1));

  // halo nodes loaded by this thread
  long long hoff[KH];
  double hP[KH];
  bool hin[KH], hact[KH];
#pragma unroll
  for (int s = 0; s < KH; ++s) {
    const int h = t + kMvThreads * s;
    hact[s] = h < tl.halo;
    hin[s] = false;
    hoff[s] = 0;
    hP[s] = 0.0;
    if (hact[s]) {
      const int axh = h % hx, ayh = (h / hx) % hy, azh = h / (hx * hy);
      const int gx = ox + axh - 1, gy = oy + ayh - 1, gz = oz + azh - 1;
      if (gx >= 0 && gx < nn0 && gy >= 0 && gy < nn1 && gz >= 0 && gz < nn2) {
        hin[s] = true;
        hoff[s] = 3 * (gx + (long long)nn0 * (gy + (long long)nn1 * gz));
        hP[s] = on_dirichlet(op, gx, gy, gz) ? 0.0 : 1.0;
      }
    }
  }
  // halo values (c, g, f) of three consecutive levels and a fourth in flight:
  // the loads of a level are issued one level before its fields are formed
  double cm[KH], c0[KH], gm[KH], g0[KH], fm[KH], f0[KH], c1[KH], g1[KH], f1[KH], c2[KH], g2[KH], f2[KH];
#pragma unroll
  for (int s = 0; s < KH; ++s) {
    cm[s] = gm[s] = fm[s] = c0[s] = g0[s] = f0[s] = c1[s] = g1[s] = f1[s] = 0.0;
    if (hin[s] && n0 >= 1) {
      const double *p = x + 3LL * (n0 - 1) * N + hoff[s];
      cm[s] = p[0];
      gm[s] = p[1];
      fm[s] = p[2];
    }
    if (hin[s]) {
      const double *p = x + 3LL * n0 * N + hoff[s];
      c0[s] = p[0];
      g0[s] = p[1];
      f0[s] = p[2];
    }
    if (hin[s] && n0 < M) {
      const double *p = x + 3LL * (n0 + 1) * N + hoff[s];
      c1[s] = p[0];
      g1[s] = p[1];
      f1[s] = p[2];
    }
  }

  // Fields of level L from the held levels L - 1 (cm), L (c0) and L + 1 (c1)
  // into buffer buf; then the held levels move on by one, level L + 2 (c2,
  // requested one level earlier) taking the place of L + 1.
  auto fields = [&](int L, double2 *buf) {
    const bool hm = L >= 1, hp = L < M;
    const bool tend = (L == 0) || (L == M);
    // rows of the time stiffness St and mass Tt at level L
    const double stm = hm ? -mc.inv_tau : 0.0, st0 = tend ? mc.inv_tau : 2.0 * mc.inv_tau,
                 stp = hp ? -mc.inv_tau : 0.0;
    const double ttm = hm ? mc.tau6 : 0.0, tt0 = tend ? mc.tau3 : 2.0 * mc.tau3, ttp = hp ? mc.tau6 : 0.0;
    const bool mflag = !dto || hm;
#pragma unroll
    for (int s = 0; s < KH; ++s) {
      const double cp = hp ? c1[s] : 0.0, gp = hp ? g1[s] : 0.0, fp = hp ? f1[s] : 0.0;
      if (hact[s]) {
        const int h = t + kMvThreads * s;
        const double P = hP[s];
        const double gn = mflag ? g0[s] : 0.0;
        const double S2 = P * (gn + gp);
        const double stf = stm * fm[s] + st0 * f0[s] + stp * fp;
        const double ttf = ttm * fm[s] + tt0 * f0[s] + ttp * fp;
        const double U3 = mc.beta1 * stf - (dto ? ht * S2 : P * (ttm * gm[s] + tt0 * g0[s] + ttp * gp));
        buf[3 * h] = make_double2(P * (c0[s] - cm[s]) - ht * (fm[s] + f0[s]), P * (c0[s] + cm[s]));
        buf[3 * h + 1] = make_double2(P * (gn - gp), S2);
        buf[3 * h + 2] = mc.l2 ? make_double2(U3 + mc.beta2 * ttf, 0.0) : make_double2(U3, mc.beta2 * ttf);
      }
      cm[s] = c0[s];
      c0[s] = cp;
      c1[s] = c2[s];
      gm[s] = g0[s];
      g0[s] = gp;
      g1[s] = g2[s];
      fm[s] = f0[s];
      f0[s] = fp;
      f1[s] = f2[s];
    }
  };
  // level L of the halo into c2 (zero unless wanted)
  auto request = [&](int L, bool want) {
#pragma unroll
    for (int s = 0; s < KH; ++s) {
      c2[s] = g2[s] = f2[s] = 0.0;
      if (hin[s] && want) {
        const double *p = x + 3LL * L * N + hoff[s];
        c2[s] = p[0];
        g2[s] = p[1];
        f2[s] = p[2];
      }
    }
  };
  // Two field buffers: the fields of level n + 1 are written while the
  // outputs of level n read those of level n, so one barrier per level
  // separates the writes of a buffer from its reads.
  double2 *const buf0 = mv_lds, *const buf1 = mv_lds + 3 * tl.halo;
  request(n0 + 2, n0 + 2 <= M && n0 + 1 < n1);
  fields(n0, buf0);
  __syncthreads();
  for (int n = n0; n < n1; ++n) {
    const bool hp = n < M;
    const bool tend = (n == 0) || (n == M);
    const double2 *const cur = ((n - n0) & 1) ? buf1 : buf0;
    if (n + 1 < n1) {
      // level n + 3 feeds the fields of level n + 2 (formed only while that level is in this chunk)
      request(n + 3, n + 3 <= M && n + 2 < n1);
      fields(n + 1, ((n - n0) & 1) ? buf0 : buf1);
    }
    // rebuild the node's stencil weights every level instead of keeping them live
    asm volatile("" : "+v"(cx.m), "+v"(cx.k), "+v"(cx.c), "+v"(cy.m), "+v"(cy.k), "+v"(cy.c));
    asm volatile("" : "+v"(cz.m), "+v"(cz.k), "+v"(cz.c));
    if (own) {
      // Sum factorisation: B, K and N are tensor products of 1-D factors, so
      // each row of three x-neighbours is first contracted with the x factors
      // (off-centre entries are the same for every node, the centre ones are
      // the node's), then weighted by the (y, z) factors of the row.  The
      // variable diffusion A is applied point by point.
      double aC = 0.0, sC = 0.0, aG = 0.0, sG = 0.0, aF = 0.0;
      // The dz planes stay a loop: unrolled, the compiler requests the LDS
      // values of all nine rows at once and their registers leave one
      // wavefront per SIMD.  Rolled, the diffusion table of the node goes to
      // per-lane scratch (cached; 224 B) and two wavefronts fit
      // (174.7 / 642 us against 187.3 / 733 us on cube32x64 / cube48x96).
#pragma unroll 1
      for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
          double myz, kyz, nyz, vmyz;
          if (dy != 0 && dz != 0) {
            const double *c4 = mc.cyz[dy > 0][dz > 0];
            myz = c4[0];
            kyz = c4[1];
            nyz = c4[2];
            vmyz = c4[3];
          } else if (dy == 0 && dz != 0) {
            myz = cy.m * mc.h6[2];
            kyz = cy.k * mc.h6[2] - cy.m * mc.hinv[2];
            nyz = mc.v[1] * mc.h6[2] * cy.c + (0.5 * dz) * mc.v[2] * cy.m;
            vmyz = mc.v[0] * myz;
          } else if (dy != 0 && dz == 0) {
            myz = mc.h6[1] * cz.m;
            kyz = -mc.hinv[1] * cz.m + mc.h6[1] * cz.k;
            nyz = (0.5 * dy) * mc.v[1] * cz.m + mc.v[2] * mc.h6[1] * cz.c;
            vmyz = mc.v[0] * myz;
          } else {
            myz = cy.m * cz.m;
            kyz = cy.k * cz.m + cy.m * cz.k;
            nyz = mc.v[1] * cy.c * cz.m + mc.v[2] * cy.m * cz.c;
            vmyz = mc.v[0] * myz;
          }
          // N^T differs from N only in the sign of the off-centre convection entries
          double ntyz;
          if (dy != 0 && dz != 0) ntyz = -nyz;
          else if (dy == 0 && dz != 0) ntyz = mc.v[1] * mc.h6[2] * cy.c - (0.5 * dz) * mc.v[2] * cy.m;
          else if (dy != 0 && dz == 0) ntyz = -(0.5 * dy) * mc.v[1] * cz.m + mc.v[2] * mc.h6[1] * cz.c;
          else ntyz = nyz;
          const double2 *row = cur + 3 * (hc + hx * (dy + hy * dz));
          const double2 w1 = row[-3], w2 = row[-2], w3 = row[-1];   // x - 1
          const double2 c1 = row[0], c2 = row[1], c3 = row[2];      // x
          const double2 e1 = row[3], e2 = row[4], e3 = row[5];      // x + 1
          const int k0 = 3 * (dy + 1) + 9 * (dz + 1);
          const double mU1 = mc.h6[0] * (w1.x + e1.x) + cx.m * c1.x;
          const double mU2 = mc.h6[0] * (w2.x + e2.x) + cx.m * c2.x;
          const double mU3 = mc.h6[0] * (w3.x + e3.x) + cx.m * c3.x;
          const double mT = mc.h6[0] * (w3.y + e3.y) + cx.m * c3.y;
          const double kT = cx.k * c3.y - mc.hinv[0] * (w3.y + e3.y);
          const double mS1 = mc.h6[0] * (w1.y + e1.y) + cx.m * c1.y;
          const double cS1 = 0.5 * (e1.y - w1.y) + cx.c * c1.y;
          const double aS1 = A[k0] * w1.y + A[k0 + 1] * c1.y + A[k0 + 2] * e1.y;
          const double mS2 = mc.h6[0] * (w2.y + e2.y) + cx.m * c2.y;
          const double cS2 = 0.5 * (w2.y - e2.y) + cx.c * c2.y;
          const double aS2 = A[k0] * w2.y + A[k0 + 1] * c2.y + A[k0 + 2] * e2.y;
          aC += myz * mU1;
          aG += myz * mU2;
          aF += myz * (mU3 + kT) + kyz * mT;
          sC += aS1 + vmyz * cS1 + nyz * mS1;
          sG += aS2 + vmyz * cS2 + ntyz * mS2;
        }
      }
      const long long idx = (long long)n * N + j;
      const double *xs = x + 3 * idx;
      double *ys = y + 3 * idx;
      const double cj = xs[0], gj = xs[1];
      ys[0] = (n == 0 || !Pj) ? cj : aC + ht * sC;
      double g;
      if (!Pj) {
        g = gj;
      } else if (dto) {
        const double wn = tend ? ht : 2.0 * ht;   // trapezoid weight of level n
        g = aG + ht * sG + (n == 0 ? gj : 0.0) + wn * sens * cj;
      } else {
        g = hp ? aG + ht * sG + ht * sens * (cj + xs[3 * N]) : gj;
      }
      ys[1] = g;
      ys[2] = aF;
    }
    __syncthreads();
  }
}

template <int KH>
__global__ void __launch_bounds__(kMvThreads) matvec_tile_kernel(OpDev op, MvTile tl, MvConst mc,
                                                                 const double *__restrict__ Atab,
                                                                 const double *__restrict__ x,
                                                                 double *__restrict__ y) {
  matvec_tile_body<KH>(op, tl, mc, Atab, x, y, xcd_work_index());
}

// Batched form: the work items of all operators in one grid, operator i
// owning [w0_i, w0_i + nw_i).
template <int KH>
__global__ void __launch_bounds__(kMvThreads) matvec_batch_kernel(const MvBatchDesc *__restrict__ descs, int count,
                                                                  const int *__restrict__ act,
                                                                  const double *__restrict__ x,
                                                                  double *__restrict__ y) {
  const int w = xcd_work_index();
  cptr<MvBatchDesc> cd = as_const(descs);
  int i = 0;
  while (i + 1 < count && cd[i + 1].w0 <= w) ++i;
  if (!as_const(act)[i]) return;
  MvBatchDesc d = load_uniform(descs + i);
  // pointers read as pointers from the constant address space are taken to
  // address global memory (global loads); rebuilt from copied words they
  // would be generic, and generic loads also wait on the LDS counter
  d.op.a_elem = cd[i].op.a_elem;
  d.op.sensor = cd[i].op.sensor;
  matvec_tile_body<KH>(d.op, d.tl, d.mc, cd[i].atab, x + d.voff, y + d.voff, w - d.w0);
}

}  // namespace

MvTile choose_matvec_tile(const OpDev &d) {
  MvTile best{};
  double best_cost = 1e300;
  const int cap = kMvThreads;
  for (int tx = 1; tx <= std::min(d.nn[0], cap); ++tx)
    for (int ty = 1; ty <= std::min(d.nn[1], cap / tx); ++ty)
      for (int tz = 1; tz <= std::min(d.nn[2], cap / (tx * ty)); ++tz) {
        const int halo = (tx + 2) * (ty + 2) * (tz + 2);
        // at most three halo nodes per thread; two field buffers within 64 KB of LDS
        if (halo > 3 * kMvThreads || sizeof(double2) * 6 * (size_t)halo > 65536) continue;
        const long long ntiles = (long long)((d.nn[0] + tx - 1) / tx) * ((d.nn[1] + ty - 1) / ty) *
                                 ((d.nn[2] + tz - 1) / tz);
        const double cost = (double)ntiles * (halo + kMvThreads);
        // ties go to the widest x extent (longer contiguous rows of x and y)
        if (cost <= best_cost) {
          best_cost = cost;
          best.t[0] = tx;
          best.t[1] = ty;
          best.t[2] = tz;
        }
      }
  for (int a = 0; a < 3; ++a) best.nt[a] = (d.nn[a] + best.t[a] - 1) / best.t[a];
  best.ntiles = best.nt[0] * best.nt[1] * best.nt[2];
  best.halo = (best.t[0] + 2) * (best.t[1] + 2) * (best.t[2] + 2);
  const int levels = d.M + 1;
  int chunks = std::max(1, std::min(levels, (1024 + best.ntiles - 1) / best.ntiles));
  best.clen = (levels + chunks - 1) / chunks;
  best.nchunks = (levels + best.clen - 1) / best.clen;
  return best;
}

void matvec_device(const kkt_op *op, const double *x, double *y, hipStream_t s) {
  const OpDev &d = op->d;
  const MvTile &tl = op->mv;
  const long long grid = (long long)tl.ntiles * tl.nchunks;
  if (grid > INT32_MAX) throw Error(STKKT_EINVAL, "kkt_matvec: mesh too large");
  const size_t lds = sizeof(double2) * 6 * (size_t)tl.halo;   // two buffers of 48 B per halo node
  const int kh = (tl.halo + kMvThreads - 1) / kMvThreads;
  const double *atab = op->atab.as<double>();
  const MvConst mc = make_mv_const(d);
  if (kh == 1)
    hipLaunchKernelGGL(matvec_tile_kernel<1>, dim3((unsigned)grid), dim3(kMvThreads), lds, s, d, tl, mc, atab, x, y);
  else if (kh == 2)
    hipLaunchKernelGGL(matvec_tile_kernel<2>, dim3((unsigned)grid), dim3(kMvThreads), lds, s, d, tl, mc, atab, x, y);
  else
    hipLaunchKernelGGL(matvec_tile_kernel<3>, dim3((unsigned)grid), dim3(kMvThreads), lds, s, d, tl, mc, atab, x, y);
  STKKT_HIP(hipGetLastError());
}

void matvec_batch_prepare(const kkt_op *const *ops, const long long *voff, int count, const Allocator *al,
                          MvBatch &out, hipStream_t s) {
  std::vector<MvBatchDesc> d(count);
  long long w = 0;
  int halo = 0;
  for (int i = 0; i < count; ++i) {
    d[i] = MvBatchDesc{};
    d[i].w0 = (int32_t)w;
    if (!ops[i]) continue;   // empty slot: no work items
    d[i].op = ops[i]->d;
    d[i].tl = ops[i]->mv;
    d[i].mc = make_mv_const(ops[i]->d);
    d[i].atab = ops[i]->atab.as<double>();
    d[i].voff = voff[i];
    d[i].nw = ops[i]->mv.ntiles * ops[i]->mv.nchunks;
    w += d[i].nw;
    halo = std::max(halo, ops[i]->mv.halo);
  }
  STKKT_REQUIRE(w <= INT32_MAX, "batched matvec: too many work items");
  out.desc = DevBuf(al, sizeof(MvBatchDesc) * (size_t)count);
  STKKT_HIP(hipMemcpyAsync(out.desc.ptr, d.data(), sizeof(MvBatchDesc) * (size_t)count, hipMemcpyHostToDevice, s));
  halo = std::max(halo, 27);
  STKKT_HIP(hipStreamSynchronize(s));   // d is released on return
  out.count = count;
  out.items = w;
  out.lds = sizeof(double2) * 6 * (size_t)halo;
  out.kh = (halo + kMvThreads - 1) / kMvThreads;
}

void matvec_batch_run(const MvBatch &b, const double *x, double *y, const int *act, hipStream_t s) {
  if (b.items == 0) return;
  const MvBatchDesc *dd = b.desc.as<MvBatchDesc>();
  const dim3 grid((unsigned)b.items);
  if (b.kh == 1)
    hipLaunchKernelGGL(matvec_batch_kernel<1>, grid, dim3(kMvThreads), b.lds, s, dd, b.count, act, x, y);
  else if (b.kh == 2)
    hipLaunchKernelGGL(matvec_batch_kernel<2>, grid, dim3(kMvThreads), b.lds, s, dd, b.count, act, x, y);
  else
    hipLaunchKernelGGL(matvec_batch_kernel<3>, grid, dim3(kMvThreads), b.lds, s, dd, b.count, act, x, y);
  STKKT_HIP(hipGetLastError());
}

}  // namespace stkkt
