/*
 * stkkt -- space-time KKT solver for the unsteady inverse source problem
 * (Deng, Cai, Zou, "Two-level space-time domain decomposition methods for
 * unsteady inverse problems", arXiv:1508.06103) on AMD MI355X (gfx950).
 *
 * C ABI.  Every entry point returns an int status:
 *   STKKT_OK (0), STKKT_NOT_CONVERGED (+1), STKKT_EINVAL (-1, bad argument),
 *   STKKT_ENOMEM (-2, allocation failed), STKKT_EHIP (-3, HIP runtime error),
 *   STKKT_EBREAKDOWN (-4, singular pivot block or non-finite Krylov quantity).
 * kkt_last_error() returns a human-readable message for the calling thread's
 * most recent failure.  No C++ exception crosses this boundary.
 *
 * Memory and streams.  "Device" pointers are HIP device addresses of FP64
 * arrays owned by the caller; they are only borrowed for the stream-ordered
 * duration of a call.  Handles (kkt_op_t, ras_t, coarse_t) own their internal
 * device memory, obtained from the kkt_alloc_t callbacks given at assembly
 * time (hipMalloc/hipFree when the callbacks are NULL).  Handles are immutable
 * after setup, except for a scratch area used by ras_apply/coarse_apply/
 * kkt_solve, so concurrent calls on the same handle must be serialised by the
 * caller (e.g. by using one stream).  `stream` is a hipStream_t passed as a
 * plain pointer (NULL = the null stream); all device work is enqueued on it.
 *
 * Vector layout (Section 3.2 of the paper): the unknown U holds, for every
 * time level n = 0..M (slowest), every spatial node j (x fastest, then y,
 * then z) and every slot c in (C, G, f) (fastest), the value at
 *   index(n, j, c) = 3 * (n * N + j) + c,   N = (n0+1)(n1+1)(n2+1).
 * Vectors have 3 * N * (M+1) doubles.
 */
#ifndef STKKT_H
#define STKKT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STKKT_OK 0
#define STKKT_NOT_CONVERGED 1
#define STKKT_EINVAL (-1)
#define STKKT_ENOMEM (-2)
#define STKKT_EHIP (-3)
#define STKKT_EBREAKDOWN (-4)

/* KKT variants.  DTO: optimality system of the discrete objective (trapezoid
 * misfit) under the Crank-Nicolson / Q1 state scheme of Section 3.1.
 * OTD: the block system printed in Appendix A of the paper. */
#define STKKT_DTO 0
#define STKKT_OTD 1

/* Regularisation of the source (kkt_problem_t.regularization). */
#define STKKT_REG_H1H1 0   /* eq. (3): beta1 |df/dt|^2 + beta2 |grad f|^2            */
#define STKKT_REG_H1L2 1   /* Example 2's H1-L2 form: beta1 |df/dt|^2 + beta2 f^2 */

#define STKKT_F64 0
#define STKKT_F32 1

#define STKKT_RESTRICT_TRANSPOSE 0
#define STKKT_RESTRICT_INJECTION 1

typedef struct kkt_op kkt_op_t;
typedef struct ras ras_t;
typedef struct coarse coarse_t;

/* Device allocator callbacks: alloc returns a device pointer (NULL on
 * failure) of at least `bytes` bytes aligned to 256; free releases it. */
typedef void *(*stkkt_alloc_fn)(size_t bytes, void *ctx);
typedef void (*stkkt_free_fn)(void *ptr, void *ctx);
typedef struct {
  stkkt_alloc_fn alloc;
  stkkt_free_fn free;
  void *ctx;
} kkt_alloc_t;

/* Problem definition (host memory, read during kkt_assemble only).
 * Model (eq. (1)): dC/dt = div(a grad C) - div(v C) + f on the box
 * [0,len0]x[0,len1]x[0,len2], t in (0,T), C = 0 on the Dirichlet faces,
 * a dC/dn = 0 elsewhere, C(.,0) = 0.  Objective (eqs. (2)-(3)): point sensors
 * and the H1-H1 space-time regularisation with weights beta1 (time) and
 * beta2 (space), or the H1-L2 form of Example 2 (beta2 weighs the L2 norm of
 * f instead of its gradient: the space factor of the beta2 block of W is the
 * mass matrix instead of the stiffness matrix, Appendix A). */
typedef struct {
  int32_t n[3];             /* elements per axis (>= 1); nodes = n + 1       */
  int32_t nt;               /* time steps M (>= 1); levels 0..M               */
  double len[3];            /* box edge lengths                               */
  double T;                 /* final time                                     */
  const double *a_elem;     /* [n2][n1][n0] diffusivity per element, > 0      */
  double v[3];              /* constant velocity                              */
  double beta1, beta2;      /* regularisation weights (> 0)                   */
  int32_t n_sensors;        /* >= 1                                           */
  const int32_t *sensor_node;  /* distinct spatial node ids, off Dirichlet faces */
  const double *data;       /* [nt+1][n_sensors] observed concentrations      */
  uint32_t dirichlet_faces; /* bit 0: x=0, 1: x=len0, 2: y=0, 3: y=len1,
                               4: z=0, 5: z=len2                              */
  int32_t variant;          /* STKKT_DTO or STKKT_OTD                         */
  int32_t regularization;   /* STKKT_REG_H1H1 (0) or STKKT_REG_H1L2 (1)       */
} kkt_problem_t;

/* One-level space-time restricted additive Schwarz (Section 3.2).
 * p[d] subdomains along x, y, z, t (node-based split: part k of L nodes owns
 * [k q + min(k,r), (k+1) q + min(k+1,r)), q,r = divmod(L, p)), each extended
 * by `overlap` nodes per side and trimmed at the global box.  Subdomain
 * solves: 3x3 point-block ILU(k) in the box's lexicographic order (Section 4:
 * k = 0 by default; the paper's first table varies k).  Level of fill on the
 * 81-point block pattern: its entries have level 0, eliminating row k from
 * row i offers entry (i, j) the level lev(i,k) + lev(k,j) + 1, and entries of
 * level <= k are kept.  k = 0 uses the stencil-specialised sweep kernels;
 * k > 0 a general level-scheduled form (its factor storage grows with k:
 * about 3.9x the ILU(0) blocks per interior row at k = 1, 6.4x at k = 2). */
typedef struct {
  int32_t p[4];
  int32_t overlap;          /* >= 0 */
  int32_t precision;        /* STKKT_F64 or STKKT_F32 factors and local solve */
  int32_t ilu_level;        /* k: 0, 1, 2 or 3 (STKKT_EINVAL otherwise) */
} ras_params_t;

/* Two-level preconditioner (Section 3.2, two-level paragraph): nested coarse
 * space-time mesh with integer coarsening factors (must divide n[] and nt),
 * interpolation I_c^h linear on the coarse mesh (per unknown slot), restriction
 * I_h^c = (I_c^h)^T or injection, coarse KKT system F_c rediscretised on the
 * coarse mesh (element coefficient = mean of the fine ones it covers; every
 * sensor must sit on a coarse node).  F_c^{-1} is applied by one of:
 *  - STKKT_COARSE_LU (the default, value 0), exactly: F_c is block tridiagonal
 *    in time, so S_0 = D_0, S_k = D_k - L_k S_{k-1}^{-1} U_{k-1}; the setup
 *    forms and inverts every S_k densely (FP64 Gauss-Jordan with partial
 *    pivoting) and keeps S_k^{-1} and S_k^{-1} U_k in `precision`, using about
 *    2 (M_c + 1) (3 N_c)^2 elements of device memory (columns padded to a
 *    multiple of 64 rows); `p`, `overlap`, `maxit`, `rtol` are ignored.
 *  - STKKT_COARSE_GMRES_RAS, as in the paper's experiments (Section 4):
 *    restarted GMRES from a zero guess with relative tolerance `rtol` and at
 *    most `maxit` steps, right-preconditioned by the one-level space-time RAS
 *    of the coarse mesh (`p`, `overlap`, ILU(0); `precision` of its factors).
 * The coarse mesh may have at most 512 nodes along x. */
#define STKKT_COARSE_LU 0
#define STKKT_COARSE_GMRES_RAS 1
typedef struct {
  int32_t factor[4];        /* coarsening in x, y, z, t                    */
  int32_t method;           /* STKKT_COARSE_LU (0) or _GMRES_RAS (1)      */
  int32_t precision;        /* STKKT_F64 or STKKT_F32 coarse blocks/factors */
  int32_t restrict_kind;    /* STKKT_RESTRICT_TRANSPOSE or _INJECTION       */
  int32_t p[4];             /* coarse subdomains in x, y, z, t              */
  int32_t overlap;          /* coarse overlap (paper: 1)                    */
  int32_t maxit;            /* coarse GMRES steps (paper: 4)                */
  double rtol;              /* coarse GMRES relative tolerance (paper: 0.1) */
} coarse_params_t;

/* Restarted right-preconditioned GMRES / FGMRES (Sections 3.2 and 4).
 * Always on, with no switch: the Arnoldi basis is orthogonalised by classical
 * Gram-Schmidt applied twice (CGS2, FP64), the Hessenberg least-squares
 * problem is solved by Givens rotations (FP64), and when the Givens estimate
 * meets rtol the true residual ||b - F x|| is computed in FP64 and decides
 * convergence (the cycle restarts if it does not meet rtol). */
typedef struct {
  int32_t restart;          /* Krylov dimension per cycle (>= 1)        */
  int32_t maxit;            /* total Arnoldi steps allowed               */
  double rtol;              /* stop when ||b - F x|| <= rtol ||b||        */
  int32_t flexible;         /* 0: GMRES, 1: FGMRES.  Both keep the
                               preconditioned basis in device memory (m more
                               n-vectors) and update x from it, so GMRES
                               needs no extra preconditioner application per
                               restart; its iterates are those of right-
                               preconditioned GMRES up to rounding.          */
  int32_t fixed_iters;      /* > 0: run exactly this many steps (no test) */
  int32_t graph;            /* kkt_solve_batch only: 1 = the Arnoldi steps of
                               a cycle replayed from captured HIP graphs, the
                               Givens rotations and convergence flags on the
                               device (one host check per 8 steps); 0 = one
                               host check per step.  Members with a coarse
                               level, or whose preconditioners cannot share
                               one launch, always run with 0.  Ignored by
                               kkt_solve.                                    */
} solve_params_t;

typedef struct {
  int32_t iters;            /* Arnoldi steps taken                   */
  int32_t restarts;
  int32_t converged;        /* 1 if the true residual met rtol       */
  int32_t status;           /* same as the return value               */
  double rel_res_est;       /* Givens estimate / ||b|| at the end    */
  double rel_res_true;      /* ||b - F x|| / ||b||                   */
  double bnorm;
  double t_ms[4];           /* total, preconditioner, matvec, orthogonalisation */
} kkt_stats_t;

/* Build the operator handle of F_h (Appendix A block structure) and write the
 * right-hand side b (3*N*(M+1) doubles, device) for the given data.
 * `al` may be NULL (hipMalloc).  `b` may be NULL. */
int kkt_assemble(const kkt_problem_t *p, const kkt_alloc_t *al, void *stream, kkt_op_t **op,
                 double *b);

/* Right-hand side for new sensor data on an existing operator.
 * data_host: [nt+1][n_sensors] host array; b: device. */
int kkt_rhs(const kkt_op_t *op, const double *data_host, void *stream, double *b);

/* kkt_rhs for callers that cannot allocate device memory (serving loops that
 * must not call hipMalloc, harnesses that forbid allocation): the same b, bit
 * for bit, with the sensor ids and the data staged in a static device array
 * of 1 MiB (STKKT_RHS_SCRATCH_BYTES) that each GPU holds until the process
 * ends, instead of buffers from the allocator.  It calls no allocation
 * routine.  The data must fit: round_up(4 n_sensors, 256) + 8 (nt+1)
 * n_sensors <= STKKT_RHS_SCRATCH_BYTES, else STKKT_EINVAL (use kkt_rhs).
 * Every call on one GPU shares that array: the call synchronises `stream`
 * before it returns, and calls that overlap on one GPU (from several host
 * threads) race.  Not for graph capture (it copies from host memory and
 * synchronises). */
#define STKKT_RHS_SCRATCH_BYTES (1 << 20)
int kkt_rhs_noalloc(const kkt_op_t *op, const double *data_host, void *stream, double *b);

/* y = F_h x: the space-time KKT operator of Section 3.1 with the block
 * structure of Appendix A (block tridiagonal in time; per level and spatial
 * node the (C, G, f) rows of the state, adjoint and source equations), applied
 * matrix-free.  x, y: device vectors of kkt_size(op) doubles in the layout
 * above; they may not alias.  Stream-ordered, no synchronisation.  Errors:
 * STKKT_EINVAL for NULL arguments. */
int kkt_matvec(const kkt_op_t *op, const double *x, double *y, void *stream);

/* Number of unknowns 3 N (M+1). */
int64_t kkt_size(const kkt_op_t *op);

/* Partition, extract the subdomain matrices and factor them (ILU(0)). */
int ras_setup(const kkt_op_t *op, const ras_params_t *rp, void *stream, ras_t **out);

/* One-level space-time restricted additive Schwarz (Section 3.2, the
 * one-level preconditioner; restricted form of Cai and Sarkis):
 *   z = sum_i (R^0_i)^T ILU_i^{-1} R^delta_i r,
 * i.e. every subdomain gathers r on its overlapped box, solves with its ILU(0)
 * factors (forward then backward block sweep, in the factors' precision) and
 * writes z on the nodes it owns only.  r, z: device vectors of kkt_size(op)
 * doubles; they may not alias.  Uses the handle's local vectors (calls on one
 * handle must be ordered on one stream).  Stream-ordered, no synchronisation.
 * Errors: STKKT_EINVAL for NULL arguments. */
int ras_apply(const ras_t *ras, const double *r, double *z, void *stream);

/* Subdomain count, and the box table: per subdomain 16 int32
 * {own_lo[4], own_hi[4], box_lo[4], box_hi[4]} in (x, y, z, t) order. */
int ras_num_subdomains(const ras_t *ras);
int ras_query_boxes(const ras_t *ras, int32_t *host_out);

/* Bytes of factor data streamed by one ras_apply (all L, U and inv(D) blocks). */
int64_t ras_factor_bytes(const ras_t *ras);

/* Which sweep kernel ras_apply runs: the rows of a wavefront level handled
 * per phase, 256 or 64, when the values of the last 16 levels of every box fit
 * in the 160 KB LDS of a workgroup (64 for boxes with many rows per level,
 * e.g. 14^4 nodes with FP64 factors); 0 when they do not and the sweeps keep
 * them in the local vector in global memory.  -1 for a NULL handle. */
int32_t ras_query_apply_rows(const ras_t *ras);

/* Factor blocks of one subdomain (the size of ras_export_factors_csr's
 * `blocks`, in 3x3 blocks); -1 for a bad handle or index. */
int64_t ras_subdomain_blocks(const ras_t *ras, int32_t sub);

/* Copy the factors of one subdomain to host memory as block CSR in the box's
 * natural order (rho = x + lx (y + ly (z + lz t))): indptr[rows + 1],
 * indices[n] (sorted columns of every row), blocks[9 n] doubles (row-major
 * 3x3: L left of the diagonal, inv(U_rr) on it, U right of it), n =
 * ras_subdomain_blocks(ras, sub).  Any ILU level; FP32 factors widened. */
int ras_export_factors_csr(const ras_t *ras, int32_t sub, int32_t *indptr, int32_t *indices, double *blocks);

/* Copy the factors of one subdomain to host memory as [rows][81][9] doubles:
 * slot s = (dx+1) + 3(dy+1) + 9(dz+1) + 27(dt+1) of local row rho
 * (rho = x + lx (y + ly (z + lz t))) holds L (s < 40), inv(U_rr) (s = 40) or
 * U (s > 40); blocks outside the box are zero.  ILU(0) only (STKKT_EINVAL for
 * k > 0, whose fill lies outside the 81 slots). */
int ras_export_factors(const ras_t *ras, int32_t sub, double *host_out);

/* Coarse level: build F_c on the coarse mesh, its one-level RAS (ILU(0)
 * factors) and the inner GMRES workspace, or, with STKKT_COARSE_LU, the
 * explicit inverses S_k^{-1} and E_k of the block elimination in time.  Fails
 * with STKKT_EINVAL when a factor does not divide the mesh or a sensor is not
 * on a coarse node, STKKT_EBREAKDOWN for a singular Schur block (a zero or
 * non-finite pivot).  The Schur blocks are inverted by Gauss-Jordan
 * elimination in 64-column panels with the pivots searched among each
 * panel's own rows (partial pivoting inside the diagonal block); the
 * environment variable STKKT_COARSE_PIVOT=global selects partial pivoting
 * over all rows, each panel then eliminated in one cooperative launch whose
 * workgroups must all be resident at once: every grid-barrier wait there is
 * bounded (about a second), so if other work on the device keeps some of
 * them from starting the setup fails with STKKT_EHIP instead of waiting.
 * While a panel is eliminated on `stream`, the rest of the previous panel's
 * update runs on a second stream of default priority that the call creates
 * and destroys; it waits for the work on `stream` before it and `stream`
 * waits for it before continuing.  The call synchronises both. */
int coarse_setup(const kkt_op_t *fine, const coarse_params_t *cp, void *stream, coarse_t **out);

/* y = I_c^h F_c^{-1} I_h^c x (device vectors of the fine size).  F_c^{-1} is
 * the inner GMRES(maxit) described above (not converging within maxit steps
 * is the normal case and not an error; this form synchronises `stream`), or
 * the exact block elimination in time (STKKT_COARSE_LU; stream-ordered, no
 * synchronisation).  x and y must not alias. */
int coarse_apply(const coarse_t *c, const double *x, double *y, void *stream);

/* Several applications of the coarse level at once: y_i = coarse_apply(x_i)
 * for i < q, with x_i = x + i ldx and y_i = y + i ldy (device vectors of
 * kkt_size(fine) doubles; ldx, ldy >= that size; the x and y ranges must not
 * overlap).  Two-level preconditioning (Section 3.2) of several right-hand
 * sides on one operator applies the same F_c^{-1} to each restricted vector:
 * with the exact block solve (STKKT_COARSE_LU) the q coarse vectors go through
 * the forward and backward sweeps together, each dense block being read once
 * per 16 right-hand sides and multiplied on the FP64 matrix cores (FP32
 * blocks widened to FP64), so that y_i depends on x_i only, not on q or on
 * the other vectors.  With the inner coarse GMRES the q applications run one
 * after the other.  The handle keeps a workspace of 2 q coarse vectors, grown
 * on demand (growing synchronises `stream`); calls on one handle must be
 * ordered on one stream.  q = 0 does nothing.  Errors: STKKT_EINVAL for
 * q < 0, NULL pointers, short strides or overlapping x and y. */
int coarse_apply_multi(const coarse_t *c, int32_t q, const double *x, int64_t ldx, double *y, int64_t ldy,
                       void *stream);

/* Solve F_h x = b.  coarse == NULL selects the one-level preconditioner;
 * otherwise M^{-1} x = y + M_one^{-1}(x - F_h y), y = coarse_apply(x).
 * x: device, holds x0 on entry (zero it for the paper's x0 = 0) and the
 * iterate on exit.  Synchronises `stream` before returning.  stats may be NULL. */
int kkt_solve(const kkt_op_t *op, const ras_t *ras, const coarse_t *coarse, const solve_params_t *sp,
              const double *b, double *x, void *stream, kkt_stats_t *stats);

/* Solve `count` independent systems F_i x_i = b_i together (batched
 * instances): every instance runs restarted FGMRES(restart) right-preconditioned
 * by its one-level RAS (Section 3.2; FGMRES as in Section 4), with its own
 * relative tolerance test, and all instances' device work is issued as one
 * launch per step (preconditioner over the (instance, subdomain) work list,
 * matvec over the (instance, tile) work list, per-instance CGS2 reductions).
 * ops[i], ras[i]: handles (ras[i] built on ops[i]); b[i], x[i]: device vectors
 * of kkt_size(ops[i]) doubles, x[i] holding x0 on entry and the iterate on exit.
 * sp->flexible is ignored (always FGMRES).  An instance's result does not
 * depend on the other members of the batch.  Device workspace for the
 * concatenated Krylov vectors comes from ops[0]'s allocator.  stats: `count`
 * entries or NULL.  Returns the most severe status over the instances;
 * synchronises `stream`. */
int kkt_solve_batch(int32_t count, const kkt_op_t *const *ops, const ras_t *const *ras, const solve_params_t *sp,
                    const double *const *b, double *const *x, void *stream, kkt_stats_t *stats);

/* Request server (served stream).  Requests -- an operator with its
 * preconditioner (and optionally a coarse level for the two-level method),
 * plus new sensor data -- are queued by kkt_server_submit and, at each
 * kkt_server_step, admitted first come first served while slots and device
 * memory allow; every admitted request then advances by one FGMRES(restart)
 * cycle together with the others (batched launches as in kkt_solve_batch), and
 * finished requests are retired, their solution copied to the caller's x_out.
 * Requests arriving while others run join at the next step (continuous
 * batching).  F_h does not depend on the data: a request only forms b, and
 * the factors of its operator stay on the device (the caller keeps handles
 * alive until every request on them has finished).  A request's result does
 * not depend on which other requests shared its steps. */
typedef struct kkt_server kkt_server_t;
typedef struct {
  int32_t restart;          /* FGMRES cycle length                          */
  int32_t maxit;            /* Arnoldi steps allowed per request            */
  double rtol;              /* ||b - F x|| <= rtol ||b|| per request         */
  int64_t device_bytes;     /* device memory for request state (half for the
                               Krylov vectors, half for per-request buffers) */
  int32_t max_active;       /* most requests advanced together              */
} server_params_t;

int kkt_server_create(const server_params_t *p, const kkt_alloc_t *al, void *stream, kkt_server_t **out);

/* Queue a request.  data_host: [nt+1][n_sensors] (copied); x_out: device
 * buffer of kkt_size(op) doubles receiving the solution (x0 = 0).  coarse may
 * be NULL.  EINVAL if the request can never fit the server. */
int kkt_server_submit(kkt_server_t *srv, const kkt_op_t *op, const ras_t *ras, const coarse_t *coarse,
                      const double *data_host, double *x_out, int64_t *ticket);

/* Admit, run one cycle, retire.  Reports the requests running and waiting. */
int kkt_server_step(kkt_server_t *srv, int32_t *n_running, int32_t *n_pending);

/* 1 and the request's stats when it has finished (then the ticket is
 * forgotten), 0 while it waits or runs.  stats.t_ms[0] = submit-to-result
 * latency, t_ms[1] = time waiting for admission. */
int kkt_server_poll(kkt_server_t *srv, int64_t ticket, kkt_stats_t *stats);

void kkt_server_destroy(kkt_server_t *srv);

void kkt_op_destroy(kkt_op_t *op);
void ras_destroy(ras_t *ras);
void coarse_destroy(coarse_t *c);

const char *kkt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STKKT_H */
