"""Right-preconditioned restarted GMRES and flexible GMRES (Saad 1993).

Section 3.2 solves F_h M^{-1} U' = b with U = M^{-1} U'; Section 4 uses
GMRES (one-level) and FGMRES (two-level) with relative tolerance 1e-6 and a
zero initial guess.  The paper does not name the orthogonalisation; this
oracle (and the GPU solver) use classical Gram-Schmidt applied twice (CGS2)
and Givens rotations on the Hessenberg matrix.  Stopping rule: the Givens
residual estimate |g_{j+1}| <= rtol ||b|| ends a cycle; the true residual
||b - F x|| <= rtol ||b|| then decides convergence, otherwise the method
restarts.  GMRES updates x += M^{-1}(V_k y); FGMRES keeps Z_j = M_j^{-1} v_j
and updates x += Z_k y.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Stats:
    iters: int = 0
    restarts: int = 0
    converged: bool = False
    rel_res_est: float = np.nan
    rel_res_true: float = np.nan
    history: list = field(default_factory=list)


def _givens(a, b):
    d = np.hypot(a, b)
    if d == 0.0:
        return 1.0, 0.0, 0.0
    return a / d, b / d, d


def gmres(A, Minv, b, *, restart=30, rtol=1e-6, maxit=10000, flexible=False, x0=None,
          fixed_iters=0):
    """Solve A x = b.  A, Minv: callables.  fixed_iters > 0 runs exactly that many
    Arnoldi steps (no convergence test) -- used for like-for-like comparisons."""
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    st = Stats()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        st.converged = True
        st.rel_res_est = st.rel_res_true = 0.0
        return np.zeros(n), st
    target = rtol * bnorm
    limit = fixed_iters if fixed_iters > 0 else maxit
    r = b - A(x) if np.any(x) else b.copy()
    beta = np.linalg.norm(r)
    st.rel_res_true = beta / bnorm
    if fixed_iters == 0 and beta <= target:
        st.converged = True
        st.rel_res_est = beta / bnorm
        return x, st
    m = restart
    while True:
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n)) if flexible else None
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        k = 0
        for j in range(m):
            z = Minv(V[j])
            if flexible:
                Z[j] = z
            w = A(z)
            h1 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h1
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h1 + h2
            hn = np.linalg.norm(w)
            col = np.zeros(m + 1)
            col[:j + 1] = h
            col[j + 1] = hn
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1]
                col[i] = t
            c, s, d = _givens(col[j], col[j + 1])
            cs[j], sn[j] = c, s
            col[j] = d
            col[j + 1] = 0.0
            H[:, j] = col
            g[j + 1] = -s * g[j]
            g[j] = c * g[j]
            st.iters += 1
            k = j + 1
            est = abs(g[j + 1])
            st.history.append(est / bnorm)
            done = st.iters >= limit
            if fixed_iters == 0 and (est <= target or hn == 0.0):
                done = True
            if done or hn == 0.0:
                break
            V[j + 1] = w / hn
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        if flexible:
            x = x + Z[:k].T @ y
        else:
            x = x + Minv(V[:k].T @ y)
        r = b - A(x)
        beta = np.linalg.norm(r)
        st.rel_res_est = abs(g[k]) / bnorm
        st.rel_res_true = beta / bnorm
        if fixed_iters > 0:
            st.converged = beta <= target
            if st.iters >= fixed_iters:
                return x, st
        elif beta <= target:
            st.converged = True
            return x, st
        if st.iters >= limit:
            return x, st
        st.restarts += 1
