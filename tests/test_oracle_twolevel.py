"""Pins of the oracle's interpolation, coarse operator, block LU and two-level method."""
import dataclasses

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import kkt, krylov, ras, twolevel
from workloads.generate import make_custom


def test_interpolation_reproduces_multilinear():
    prob = make_custom((4, 6, 2), 4, 1, lattice=1, sensors=np.array([2 + 7 * (3 + 7 * 1)]))
    fac = (2, 3, 2, 2)
    P = twolevel.prolongation(prob, fac)
    nx, ny, nz = prob.n
    cx, cy, cz, ct = nx // 2, ny // 3, nz // 2, prob.M // 2
    fun = lambda x, y, z, t: (1 + 2 * x) * (3 - y) * (0.5 + z) * (2 + 0.7 * t)

    def sample(nxs, nys, nzs, nts, hx, hy, hz, ht):
        T, Z, Y, X = np.meshgrid(np.arange(nts + 1) * ht, np.arange(nzs + 1) * hz, np.arange(nys + 1) * hy,
                                 np.arange(nxs + 1) * hx, indexing="ij")
        v = fun(X, Y, Z, T).ravel()
        return np.stack([v, 2 * v, -v], axis=1).ravel()
    h = (1 / nx, 1 / ny, 1 / nz, 1 / prob.M)
    coarse = sample(cx, cy, cz, ct, 2 * h[0], 3 * h[1], 2 * h[2], 2 * h[3])
    fine = sample(nx, ny, nz, prob.M, *h)
    np.testing.assert_allclose(P @ coarse, fine, rtol=1e-13)


def test_injection_picks_coarse_nodes():
    P = twolevel.injection_1d(3, 2).toarray()
    assert np.array_equal(np.argmax(P, axis=0), [0, 2, 4, 6])
    assert P.sum() == 4


def test_coarse_problem_mean_coefficient_and_sensors():
    nn = 9
    sens = np.array([2 + nn * (4 + nn * 6), 6 + nn * (2 + nn * 4)], dtype=np.int32)
    prob = make_custom((8, 8, 8), 8, 2, sensors=sens)
    cp = twolevel.coarse_problem(prob, (2, 2, 2, 4))
    a = prob.a_elem.reshape(8, 8, 8)
    assert np.isclose(cp.a_elem.reshape(4, 4, 4)[1, 2, 3], a[2:4, 4:6, 6:8].mean())
    assert list(cp.sensor_node) == [1 + 5 * (2 + 5 * 3), 3 + 5 * (1 + 5 * 2)]
    assert cp.M == 2


def test_block_tridiag_lu_exact():
    prob = make_custom((4, 4, 4), 6, 3, lattice=1, sensors=np.array([2 + 5 * (2 + 5 * 2)]))
    F = kkt.assemble(prob)
    lu = twolevel.BlockTridiagLU(F, prob.M + 1)
    e = np.random.default_rng(0).standard_normal(F.shape[0])
    x = lu.solve(e)
    assert np.linalg.norm(F @ x - e) <= 1e-10 * np.linalg.norm(e)
    xs = spla.splu(F.tocsc()).solve(e)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_two_level_with_identity_coarsening_is_exact():
    """Coarse mesh = fine mesh: y = F^{-1} x and x - F y = 0, so FGMRES takes one step."""
    prob = make_custom((3, 3, 3), 4, 5, lattice=1, sensors=np.array([1 + 4 * (2 + 4 * 1)]))
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    b = kkt.rhs(prob)
    R = ras.RAS(prob, (2, 2, 1, 2), 1, terms=terms)
    tl = twolevel.TwoLevel(prob, R.apply, lambda v: F @ v, (1, 1, 1, 1))
    x, st = krylov.gmres(lambda v: F @ v, tl, b, restart=10, rtol=1e-10, flexible=True)
    assert st.iters == 1 and st.converged


def test_two_level_fewer_iterations_than_one_level():
    """Paper Tables 3-4 trend: the coarse space-time correction cuts the iteration count."""
    nn = 13
    idx = [3, 6, 9]
    sens = np.array([i + nn * (j + nn * k) for k in idx for j in idx for i in idx], dtype=np.int32)
    prob = make_custom((12, 12, 12), 16, 4, sensors=sens)
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    b = kkt.rhs(prob)
    A = lambda v: F @ v
    R = ras.RAS(prob, (3, 3, 3, 4), 1, terms=terms)
    _, st1 = krylov.gmres(A, R.apply, b, restart=50, rtol=1e-6)
    tl = twolevel.TwoLevel(prob, R.apply, A, (3, 3, 3, 4))
    x2, st2 = krylov.gmres(A, tl, b, restart=50, rtol=1e-6, flexible=True)
    assert st1.converged and st2.converged
    assert st2.iters < st1.iters


def test_two_level_gmres_ras_coarse_solver():
    """The paper's coarse solver (GMRES(4), rtol 0.1, coarse RAS) still cuts iterations."""
    nn = 13
    idx = [3, 6, 9]
    sens = np.array([i + nn * (j + nn * k) for k in idx for j in idx for i in idx], dtype=np.int32)
    prob = make_custom((12, 12, 12), 16, 4, sensors=sens)
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    b = kkt.rhs(prob)
    A = lambda v: F @ v
    R = ras.RAS(prob, (3, 3, 3, 4), 1, terms=terms)
    _, st1 = krylov.gmres(A, R.apply, b, restart=50, rtol=1e-6)
    tl = twolevel.TwoLevel(prob, R.apply, A, (3, 3, 3, 4), coarse="gmres_ras", coarse_parts=(2, 2, 2, 2),
                           coarse_overlap=1, coarse_maxit=4, coarse_rtol=0.1)
    x, st2 = krylov.gmres(A, tl, b, restart=50, rtol=1e-6, flexible=True)
    assert st2.converged and st2.iters < st1.iters
    assert np.linalg.norm(b - F @ x) <= 1e-6 * np.linalg.norm(b)


def test_gmres_ras_coarse_exact_when_coarse_ras_is_exact():
    """2 x 2 x 2 coarse nodes: one coarse subdomain's ILU(0) is the exact block
    LU (every spatial pair is a stencil neighbour), so the paper's coarse
    solver -- GMRES right-preconditioned by that RAS -- must return
    F_c^{-1} r after its first step, equal to the exact block solve."""
    prob = make_custom((2, 2, 2), 8, 6, faces=0, sensors=np.array([0]))
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    R = ras.RAS(prob, (1, 1, 2, 2), 1, terms=terms)
    fac = (2, 2, 2, 2)
    gm = twolevel.TwoLevel(prob, R.apply, lambda v: F @ v, fac, coarse="gmres_ras", coarse_parts=(1, 1, 1, 1),
                           coarse_overlap=1, coarse_maxit=4, coarse_rtol=0.1)
    lu = twolevel.TwoLevel(prob, R.apply, lambda v: F @ v, fac, coarse="lu")
    assert gm.cprob.n == (1, 1, 1) and gm.cprob.M == 4
    r = np.random.default_rng(3).standard_normal(gm.Fc.shape[0])
    xg, xl = gm.coarse.solve(r), lu.coarse.solve(r)
    assert np.linalg.norm(xg - xl) <= 1e-12 * np.linalg.norm(xl)
    assert np.linalg.norm(gm.Fc @ xg - r) <= 1e-12 * np.linalg.norm(r)


def _min_residual_iterates(A, Minv, r, kmax):
    """Iterates of right-preconditioned GMRES from zero, by brute force: the
    k-th minimises |r - A Minv u| over u in span{r, (A Minv) r, ...,
    (A Minv)^{k-1} r}.  The basis is orthonormalised by numpy's QR and the
    least-squares problem solved by lstsq (no Arnoldi, no Givens)."""
    Q = (r / np.linalg.norm(r))[:, None]
    out = []
    for k in range(1, kmax + 1):
        AMQ = np.stack([A(Minv(Q[:, i])) for i in range(k)], axis=1)
        c = np.linalg.lstsq(AMQ, r, rcond=None)[0]
        x = Minv(Q @ c)
        out.append((x, np.linalg.norm(r - A(x))))
        Q = np.linalg.qr(np.concatenate([Q, AMQ[:, -1:]], axis=1))[0]
    return out


def test_gmres_ras_coarse_stopping_rule():
    """The paper's coarse solve (Section 4): GMRES from a zero guess with
    relative tolerance 0.1 and at most 4 steps.  On a coarse mesh where the
    coarse RAS is inexact, the result must be the brute-force minimal-residual
    iterate of the first step k whose residual |r - F_c x_k| (F_c assembled
    independently) is within rtol |r|, else of step 4: for rtol 0.1, for
    tolerances placed between consecutive residuals (stop at exactly k = 1..4),
    and for a tolerance no step reaches (4 steps, not more); with rtol 1 the
    zero guess is returned."""
    nn = 9
    idx = [2, 4, 6]
    sens = np.array([i + nn * (j + nn * k) for k in idx for j in idx for i in idx], dtype=np.int32)
    prob = make_custom((8, 8, 8), 8, 4, sensors=sens)
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    R = ras.RAS(prob, (2, 2, 2, 2), 1, terms=terms)
    tl = twolevel.TwoLevel(prob, R.apply, lambda v: F @ v, (2, 2, 2, 2), coarse="gmres_ras",
                           coarse_parts=(2, 2, 1, 2), coarse_overlap=1, coarse_maxit=4, coarse_rtol=0.1)
    cs = tl.coarse
    Fc = kkt.assemble(tl.cprob)
    b = kkt.rhs(prob)
    # a restricted random vector (no step reaches 0.1) and the restricted b (step 1 does)
    for r in (tl.R @ np.random.default_rng(5).standard_normal(F.shape[0]), tl.R @ b):
        rn = np.linalg.norm(r)
        its = _min_residual_iterates(lambda v: Fc @ v, cs.R.apply, r, 4)
        res = [rho / rn for _, rho in its]
        assert all(res[k + 1] < (1 - 1e-3) * res[k] for k in range(3)) and res[3] > 1e-4   # decreasing, inexact
        cases = [(0.1, next((k for k in range(4) if res[k] <= 0.1), 3)), (1e-9, 3)]
        cases += [(np.sqrt(res[k] * res[k - 1]), k) for k in range(1, 4)]
        for rtol, k in cases:
            cs.rtol = rtol
            x = cs.solve(r)
            xk, rho = its[k]
            assert np.linalg.norm(x - xk) <= 1e-8 * np.linalg.norm(xk), (rtol, k)
            assert abs(np.linalg.norm(r - Fc @ x) - rho) <= 1e-8 * rn, (rtol, k)
        cs.rtol = 1.0    # the zero guess already meets the tolerance: no step
        assert not np.any(cs.solve(r))
