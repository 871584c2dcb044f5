"""Reduced-space view of the discrete problem (used only to pin the KKT system).

The traditional reduced-space approach of the paper's introduction eliminates
C through forward time marching and the multiplier through backward
(adjoint) marching.  Here, with the same Crank-Nicolson/Q1 state scheme as the
KKT system (Section 3.1) and C_0 = 0:

  state:   C^0 = 0;  n >= 1:  A1' C^n = -A2'' C^{n-1} + tau/2 P B (f^{n-1} + f^n)
           A1' = P A1 P + Q (identity on Dirichlet nodes), A2'' = P A2 P
  J_h(f) = 1/2 sum_n w_n (C^n - d^n)^T S (C^n - d^n) + 1/2 f^T W f
  grad J = W f + Phi^T Qw (Phi f - d),   Phi: f -> C (linear),  Qw = diag(w_n S)

Phi^T is applied by the adjoint (backward) march.  The minimiser of J_h solves
(W + Phi^T Qw Phi) f = Phi^T Qw d, done here by plain conjugate gradients.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


class Reduced:
    def __init__(self, prob, ops=None):
        self.prob = prob
        ops = ops if ops is not None else fem.spatial_ops(prob)
        self.ops = ops
        M = prob.M
        self.tau = tau = prob.T / M
        P = sp.diags(ops.interior.astype(np.float64))
        Q = sp.diags((~ops.interior).astype(np.float64))
        AN = ops.A + ops.N
        A1 = ops.B + 0.5 * tau * AN
        A2 = -ops.B + 0.5 * tau * AN
        self.A1p = (P @ A1 @ P + Q).tocsc()
        self.A2pp = (P @ A2 @ P).tocsr()
        self.PB = (P @ ops.B).tocsr()
        self.lu = spla.splu(self.A1p)
        self.w = fem.trapezoid_weights(M, tau)
        self.S = ops.sensor
        Tt = fem.time_mass(M, tau)
        St = fem.time_stiff(M, tau)
        self.Wt_beta1 = prob.beta1 * St
        self.Wt_beta2 = prob.beta2 * Tt
        # space factor of the beta2 term: K (eq. (3)) or the mass matrix (H1-L2 of Example 2)
        self.Ws = ops.B if getattr(prob, "reg", 0) == 1 else ops.K
        d = np.zeros((M + 1, prob.N))
        d[:, np.asarray(prob.sensor_node)] = prob.data
        self.d = d

    def W(self, f):
        """(beta1 St x B + beta2 Tt x K) f (or beta2 Tt x B, H1-L2) for f of shape (M+1, N)."""
        return self.Wt_beta1 @ (self.ops.B @ f.T).T + self.Wt_beta2 @ (self.Ws @ f.T).T

    def forward(self, f):
        M = self.prob.M
        C = np.zeros((M + 1, self.prob.N))
        for n in range(1, M + 1):
            rhs = -self.A2pp @ C[n - 1] + 0.5 * self.tau * (self.PB @ (f[n - 1] + f[n]))
            C[n] = self.lu.solve(rhs)
        return C

    def adjoint_apply(self, g):
        """Phi^T g by backward marching: solve E^T mu = g, return Bf^T mu."""
        M = self.prob.M
        mu = np.zeros((M + 2, self.prob.N))
        for n in range(M, 0, -1):
            rhs = g[n] - self.A2pp.T @ mu[n + 1]
            mu[n] = self.lu.solve(rhs, trans="T")
        out = np.zeros((M + 1, self.prob.N))
        for m in range(M + 1):
            acc = np.zeros(self.prob.N)
            if m >= 1:
                acc += mu[m]
            if m + 1 <= M:
                acc += mu[m + 1]
            out[m] = 0.5 * self.tau * (self.PB.T @ acc)
        return out

    def J(self, f):
        C = self.forward(f)
        r = C - self.d
        mis = 0.5 * np.sum(self.w[:, None] * self.S[None, :] * r * r)
        return mis + 0.5 * np.sum(f * self.W(f))

    def grad(self, f):
        C = self.forward(f)
        g = self.w[:, None] * self.S[None, :] * (C - self.d)
        return self.W(f) + self.adjoint_apply(g)

    def hess(self, f):
        C = self.forward(f)
        return self.W(f) + self.adjoint_apply(self.w[:, None] * self.S[None, :] * C)

    def cg(self, tol=1e-12, maxit=20000):
        """Solve (W + Phi^T Qw Phi) f = Phi^T Qw d by conjugate gradients."""
        shape = (self.prob.M + 1, self.prob.N)
        b = self.adjoint_apply(self.w[:, None] * self.S[None, :] * self.d)
        f = np.zeros(shape)
        r = b.copy()
        p = r.copy()
        rr = np.sum(r * r)
        bn = np.sqrt(np.sum(b * b))
        its = 0
        while np.sqrt(rr) > tol * bn and its < maxit:
            Ap = self.hess(p)
            alpha = rr / np.sum(p * Ap)
            f += alpha * p
            r -= alpha * Ap
            rr_new = np.sum(r * r)
            p = r + (rr_new / rr) * p
            rr = rr_new
            its += 1
        return f, its
