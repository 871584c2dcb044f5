// Operator assembly, right-hand side and the matrix-free space-time matvec.
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
// y = F_h x.  One thread per space-time node (n, j); the 27 spatial
// neighbours at levels n-1, n, n+1 are read through the caches.  Rows follow
// the block formula of kkt_block_c() with the time couplings fused:
//   C row (n >= 1, interior j): sum_i Pi[(B + tau/2 (A+N)) C_i^n + (-B + tau/2 (A+N)) C_i^{n-1}]
//                               - tau/2 B (f_i^{n-1} + f_i^n)
//   G row (interior j), DTO: sum_i Pi[[n>=1](B + tau/2(A+N^T)) G_i^n + [n<M](-B + tau/2 (A+N^T)) G_i^{n+1}]
//                            + [n=0] G_j^0 + w_n S_j C_j^n
//                       OTD (n < M): sum_i Pi[(B + tau/2(A+N^T)) G_i^n + (-B + tau/2(A+N^T)) G_i^{n+1}]
//                            + tau/2 S_j (C_j^n + C_j^{n+1});  n = M: G_j^M
//   f row: sum_i beta1 B (St f_i)^n + beta2 K (Tt f_i)^n
//          - DTO: tau/2 B Pi ([n>=1] G_i^n + [n<M] G_i^{n+1});  OTD: B Pi (Tt G_i)^n
//   Dirichlet rows of C and G, and the C row of level 0, are identity rows.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) matvec_kernel(OpDev op, const double *__restrict__ Atab,
                                                     const double *__restrict__ x, double *__restrict__ y) {
  const long long V = op.V;
  const int M = op.M;
  const double tau = op.tau, ht = 0.5 * tau;
  const bool dto = op.variant == STKKT_DTO;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < V;
       idx += (long long)gridDim.x * blockDim.x) {
    const int n = (int)(idx / op.N);
    const long long j = idx - (long long)n * op.N;
    const int jx = (int)(j % op.nn[0]);
    const int jy = (int)((j / op.nn[0]) % op.nn[1]);
    const int jz = (int)(j / ((long long)op.nn[0] * op.nn[1]));
    const bool Pj = !on_dirichlet(op, jx, jy, jz);
    const bool has_m = n >= 1, has_p = n <= M - 1;
    const double stm = has_m ? tstiff(tau, n, -1, M) : 0.0, st0 = tstiff(tau, n, 0, M),
                 stp = has_p ? tstiff(tau, n, 1, M) : 0.0;
    const double ttm = has_m ? tmass(tau, n, -1, M) : 0.0, tt0 = tmass(tau, n, 0, M),
                 ttp = has_p ? tmass(tau, n, 1, M) : 0.0;
    double accC = 0.0, accG = 0.0, accF = 0.0;
    for (int k = 0; k < 27; ++k) {
      const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
      const int ix = jx + dx, iy = jy + dy, iz = jz + dz;
      if (ix < 0 || ix >= op.nn[0] || iy < 0 || iy >= op.nn[1] || iz < 0 || iz >= op.nn[2]) continue;
      const double mx = mass1(op.h[0], jx, dx, op.nn[0]);
      const double my = mass1(op.h[1], jy, dy, op.nn[1]);
      const double mz = mass1(op.h[2], jz, dz, op.nn[2]);
      const double B = mx * my * mz;
      const double K = stiff1(op.h[0], jx, dx, op.nn[0]) * my * mz + mx * stiff1(op.h[1], jy, dy, op.nn[1]) * mz +
                       mx * my * stiff1(op.h[2], jz, dz, op.nn[2]);
      const double Nv = op.v[0] * conv1(jx, dx, op.nn[0]) * my * mz + op.v[1] * mx * conv1(jy, dy, op.nn[1]) * mz +
                        op.v[2] * mx * my * conv1(jz, dz, op.nn[2]);
      const double Nt = op.v[0] * conv1(ix, -dx, op.nn[0]) * my * mz + op.v[1] * mx * conv1(iy, -dy, op.nn[1]) * mz +
                        op.v[2] * mx * my * conv1(iz, -dz, op.nn[2]);
      const double A = Atab[27 * j + k];
      const double Pi = on_dirichlet(op, ix, iy, iz) ? 0.0 : 1.0;
      const long long i = ix + (long long)op.nn[0] * (iy + (long long)op.nn[1] * iz);
      const double *x0 = x + 3 * ((long long)n * op.N + i);
      const double c0 = x0[0], g0 = x0[1], f0 = x0[2];
      double cm = 0.0, fm = 0.0, gp = 0.0, fp = 0.0, gm = 0.0;
      if (has_m) {
        const double *xm = x0 - 3LL * op.N;
        cm = xm[0];
        gm = xm[1];
        fm = xm[2];
      }
      if (has_p) {
        const double *xp = x0 + 3LL * op.N;
        gp = xp[1];
        fp = xp[2];
      }
      const double AN = A + Nv, ANt = A + Nt;
      if (has_m) accC += Pi * ((B + ht * AN) * c0 + (-B + ht * AN) * cm) - ht * B * (fm + f0);
      if (dto) {
        accG += Pi * ((has_m ? (B + ht * ANt) * g0 : 0.0) + (has_p ? (-B + ht * ANt) * gp : 0.0));
        accF -= ht * B * Pi * ((has_m ? g0 : 0.0) + (has_p ? gp : 0.0));
      } else {
        if (has_p) accG += Pi * ((B + ht * ANt) * g0 + (-B + ht * ANt) * gp);
        accF -= B * Pi * (ttm * gm + tt0 * g0 + ttp * gp);
      }
      accF += op.beta1 * B * (stm * fm + st0 * f0 + stp * fp) + op.beta2 * K * (ttm * fm + tt0 * f0 + ttp * fp);
    }
    const double *xs = x + 3 * idx;
    double *ys = y + 3 * idx;
    const double sens = op.sensor[j];
    ys[0] = (n == 0 || !Pj) ? xs[0] : accC;
    double g;
    if (!Pj) {
      g = xs[1];
    } else if (dto) {
      g = accG + (n == 0 ? xs[1] : 0.0) + wtrap(tau, n, M) * sens * xs[0];
    } else {
      g = (n < M) ? accG + ht * sens * (xs[0] + xs[3 * (long long)op.N]) : xs[1];
    }
    ys[1] = g;
    ys[2] = accF;
  }
}

void matvec_device(const OpDev &d, const double *Atab, const double *x, double *y, hipStream_t s) {
  hipLaunchKernelGGL(matvec_kernel, dim3(blocks_for(d.V, 256, 1 << 16)), dim3(256), 0, s, d, Atab, x, y);
  STKKT_HIP(hipGetLastError());
}

}  // namespace stkkt
