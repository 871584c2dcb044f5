"""The fully discretised space-time KKT system F_h U = b.

Unknown ordering (Section 3.2): time level n slowest, then spatial node j
(x fastest), then the slot c in (C, G, f) fastest:
    index(n, j, c) = 3*(n*N + j) + c.
F_h is block tridiagonal in time (Section 3.2) and is written here as a sum of
Kronecker products  T (time, (M+1)x(M+1))  x  S (space, NxN)  x  E_{c,c'} (3x3),
which is exactly the ordering above.

Spatial matrices (see ``fem``): A1 = B + tau/2 (A + N), A2 = -B + tau/2 (A + N)
(Appendix A, with E read as the Galerkin convection matrix N[j,i] =
(v.grad phi_i, phi_j) for the state and its transpose for the adjoint).
W = beta1 St x B + beta2 Tt x K (Appendix A, W^{nm} = beta1 L^{nm} + beta2 K^{nm}) for the
regularisation of eq. (3); for the H1-L2 regularisation of Example 2 (time
gradient and L2 norm of f) the space factor of the beta2 term is the mass
matrix: W = beta1 St x B + beta2 Tt x B.

Two variants:

* DTO (default): first-order conditions of the discrete Lagrangian of
    J_h(f) = 1/2 sum_n w_n (C^n - d^n)^T S (C^n - d^n) + 1/2 f^T W f
  subject to the Crank-Nicolson/Q1 state equation (Section 3.1 state scheme)
  with trapezoid weights w_n.  Rows per level n (interior node rows):
    C-slot: n = 0: C^0 = C_0;  n >= 1: A1 C^n + A2 C^{n-1} - tau/2 B (f^{n-1} + f^n) = 0
    G-slot: [n>=1] A1^T G^n + [n=0] G^0 + [n<M] A2^T G^{n+1} + w_n S C^n = w_n S d^n
    f-slot: (W f)^n - tau/2 B ([n>=1] G^n + [n<M] G^{n+1}) = 0
* OTD: the Appendix A system literally: G-slot rows
    n < M: A1^T G^n + A2^T G^{n+1} + tau/2 S (C^n + C^{n+1}) = tau/2 S (d^n + d^{n+1}),
    n = M: G^M = 0;  f-slot rows (W f)^n - sum_m Tt[n,m] B G^m = 0.

Dirichlet faces (Gamma_1): C- and G-slot rows of boundary nodes are identity
rows at every level and the C/G columns of boundary nodes are zero in every
other row (f has no Dirichlet nodes).  Sensors must sit off the Dirichlet faces.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import fem

DTO = 0
OTD = 1
H1H1 = 0
H1L2 = 1


def _E(c, cp):
    e = sp.lil_matrix((3, 3))
    e[c, cp] = 1.0
    return e.tocsr()


def _diag(v):
    return sp.diags(np.asarray(v, dtype=np.float64), format="csr")


@dataclass
class KKTTerms:
    """F_h = sum over terms of kron(T, S, E[c,c'])."""
    terms: list = field(default_factory=list)      # (T, S, c, cp)
    N: int = 0
    M: int = 0

    def add(self, T, S, c, cp):
        self.terms.append((sp.csr_matrix(T), sp.csr_matrix(S), c, cp))


def kkt_terms(prob, ops=None) -> KKTTerms:
    ops = ops if ops is not None else fem.spatial_ops(prob)
    M = prob.M
    tau = prob.T / M
    Nn = ops.B.shape[0]
    L = M + 1
    P = _diag(ops.interior.astype(np.float64))
    Q = _diag((~ops.interior).astype(np.float64))
    I = sp.identity(Nn, format="csr")
    S = _diag(ops.sensor)
    if np.any(ops.sensor[~ops.interior] != 0):
        raise ValueError("sensor on a Dirichlet face")
    AN = ops.A + ops.N
    A1 = (ops.B + 0.5 * tau * AN).tocsr()
    A2 = (-ops.B + 0.5 * tau * AN).tocsr()
    It = sp.identity(L, format="csr")
    Z0 = sp.csr_matrix(([1.0], ([0], [0])), shape=(L, L))
    ZM = sp.csr_matrix(([1.0], ([M], [M])), shape=(L, L))
    Tc1 = It - Z0                                               # levels n >= 1
    Tc2 = sp.diags([np.ones(M)], [-1], shape=(L, L), format="csr")   # (n, n-1)
    Tg2 = sp.diags([np.ones(M)], [1], shape=(L, L), format="csr")    # (n, n+1)
    Tt = fem.time_mass(M, tau)
    St = fem.time_stiff(M, tau)
    w = fem.trapezoid_weights(M, tau)
    t = KKTTerms(N=Nn, M=M)
    # C-slot rows (state equation), both variants
    t.add(Tc1, P @ A1 @ P, 0, 0)
    t.add(Tc2, P @ A2 @ P, 0, 0)
    t.add(Z0, I, 0, 0)
    t.add(Tc1, Q, 0, 0)
    t.add(Tc1 + Tc2, -0.5 * tau * (P @ ops.B), 0, 2)
    # f-slot: f-f coupling W, both variants
    t.add(prob.beta1 * St, ops.B, 2, 2)
    t.add(prob.beta2 * Tt, ops.B if getattr(prob, "reg", H1H1) == H1L2 else ops.K, 2, 2)
    if prob.variant == DTO:
        t.add(_diag(w), S, 1, 0)
        t.add(Tc1, P @ A1.T @ P, 1, 1)
        t.add(Z0, P, 1, 1)
        t.add(Tg2, P @ A2.T @ P, 1, 1)
        t.add(It, Q, 1, 1)
        t.add(Tc1 + Tg2, -0.5 * tau * (ops.B @ P), 2, 1)
    elif prob.variant == OTD:
        IM = It - ZM
        t.add(0.5 * tau * (IM + Tg2), S, 1, 0)
        t.add(IM, P @ A1.T @ P, 1, 1)
        t.add(Tg2, P @ A2.T @ P, 1, 1)
        t.add(IM, Q, 1, 1)
        t.add(ZM, I, 1, 1)
        t.add(-Tt, ops.B @ P, 2, 1)
    else:
        raise ValueError("unknown variant")
    return t


def assemble(prob, ops=None, terms=None) -> sp.csr_matrix:
    """F_h as scalar CSR (3V x 3V)."""
    terms = terms if terms is not None else kkt_terms(prob, ops)
    F = None
    for (T, S, c, cp) in terms.terms:
        blk = sp.kron(T, sp.kron(S, _E(c, cp), format="csr"), format="csr")
        F = blk if F is None else F + blk
    F = F.tocsr()
    F.sort_indices()
    return F


def rhs(prob, ops=None) -> np.ndarray:
    """b: sensor data enter the G-slot rows only (C_0 = 0, p = 0, q = 0)."""
    M = prob.M
    tau = prob.T / M
    Nn = prob.N
    d = np.zeros((M + 1, Nn))
    d[:, np.asarray(prob.sensor_node)] = prob.data
    b = np.zeros((M + 1, Nn, 3))
    if prob.variant == DTO:
        w = fem.trapezoid_weights(M, tau)
        b[:, :, 1] = w[:, None] * d
    else:
        b[:M, :, 1] = 0.5 * tau * (d[:M] + d[1:])
    return b.ravel()


def apply_terms(terms: KKTTerms, x: np.ndarray) -> np.ndarray:
    """y = F_h x evaluated term by term as T X_c' S^T (no global matrix)."""
    L = terms.M + 1
    X = x.reshape(L, terms.N, 3)
    Y = np.zeros_like(X)
    for (T, S, c, cp) in terms.terms:
        Y[:, :, c] += T @ (S @ X[:, :, cp].T).T
    return Y.ravel()


def box_submatrix(terms: KKTTerms, node_ids: np.ndarray, t0: int, t1: int) -> sp.csr_matrix:
    """Principal submatrix of F_h on (levels t0..t1-1) x (spatial nodes node_ids).

    node_ids must be listed in the box's lexicographic order; the local
    unknown order is then (level, node, slot) exactly like the global one.
    """
    F = None
    for (T, S, c, cp) in terms.terms:
        Tb = T[t0:t1][:, t0:t1]
        Sb = S[node_ids][:, node_ids]
        blk = sp.kron(Tb, sp.kron(Sb, _E(c, cp), format="csr"), format="csr")
        F = blk if F is None else F + blk
    F = F.tocsr()
    F.sort_indices()
    return F
