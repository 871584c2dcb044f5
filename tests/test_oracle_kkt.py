"""Pins of the oracle's KKT system (DTO default, OTD structural checks).

The DTO system must be the first-order optimality system of the discrete
objective J_h under the Crank-Nicolson/Q1 state equation.  It is checked
against an independent reduced-space solve (forward/adjoint marching + CG),
against finite differences of J_h, against the forward and backward time
marches, and by the symmetry of its Lagrangian Hessian.
"""
import dataclasses
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import kkt, krylov, ras, reduced, fem
from workloads.generate import make_custom, OTD, DTO, H1L2

HERE = os.path.dirname(os.path.abspath(__file__))


def tiny(variant=DTO, n=(3, 2, 2), M=3, seed=11):
    return make_custom(n, M, seed, lattice=1, variant=variant)


def slot_swap_perm(nrows):
    p = np.arange(nrows).reshape(-1, 3).copy()
    p[:, [0, 1]] = p[:, [1, 0]]
    return p.ravel()


@pytest.mark.parametrize("shape", [((3, 2, 2), 3), ((2, 3, 4), 4), ((4, 4, 4), 5)])
def test_dto_lagrangian_hessian_symmetric(shape):
    prob = make_custom(shape[0], shape[1], 3, lattice=2)
    F = kkt.assemble(prob)
    H = F[slot_swap_perm(F.shape[0])]
    assert abs(H - H.T).max() <= 1e-15 * abs(F).max()


def test_dto_hessian_symmetric_cube8x16(cube8x16):
    prob, _ = cube8x16
    F = kkt.assemble(prob)
    H = F[slot_swap_perm(F.shape[0])]
    assert abs(H - H.T).max() <= 1e-15 * abs(F).max()


def test_apply_terms_and_box_submatrix():
    prob = make_custom((3, 4, 2), 4, 5, lattice=2)
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    x = np.random.default_rng(0).standard_normal(F.shape[0])
    assert np.abs(kkt.apply_terms(terms, x) - F @ x).max() < 1e-13
    sd = ras.Subdomain(0, (1, 1, 0, 1), (3, 3, 2, 3), (0, 1, 0, 1), (4, 4, 2, 4))
    nid = ras.box_node_ids(prob, sd)
    gi = ras.box_global_index(prob, sd)
    Fb = kkt.box_submatrix(terms, nid, sd.box_lo[3], sd.box_hi[3])
    assert abs(Fb - F[gi][:, gi]).max() == 0.0


def _solve_direct(prob):
    F = kkt.assemble(prob)
    b = kkt.rhs(prob)
    return F, b, np.linalg.solve(F.toarray(), b)


@pytest.mark.parametrize("shape", [((3, 2, 2), 3), ((4, 3, 3), 4)])
def test_dto_matches_reduced_cg(shape):
    prob = make_custom(shape[0], shape[1], 21, lattice=2)
    _, _, U = _solve_direct(prob)
    f_kkt = U.reshape(prob.M + 1, prob.N, 3)[:, :, 2]
    f_cg, its = reduced.Reduced(prob).cg(tol=1e-13)
    assert np.linalg.norm(f_kkt - f_cg) <= 1e-8 * np.linalg.norm(f_cg)


def test_dto_matches_reduced_cg_cube8x16(cube8x16):
    prob, s = cube8x16
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    b = kkt.rhs(prob)
    R = ras.RAS(prob, s.parts, s.overlap, terms=terms)
    U, st = krylov.gmres(lambda v: F @ v, R.apply, b, restart=s.restart, rtol=1e-12)
    assert st.converged
    f_kkt = U.reshape(prob.M + 1, prob.N, 3)[:, :, 2]
    f_cg, _ = reduced.Reduced(prob).cg(tol=1e-13)
    assert np.linalg.norm(f_kkt - f_cg) <= 1e-8 * np.linalg.norm(f_cg)


def test_fd_gradient_vanishes_at_kkt_solution():
    prob = make_custom((4, 3, 3), 4, 8, lattice=2)
    _, _, U = _solve_direct(prob)
    f = U.reshape(prob.M + 1, prob.N, 3)[:, :, 2]
    red = reduced.Reduced(prob)
    rng = np.random.default_rng(3)
    scale = np.linalg.norm(red.grad(np.zeros_like(f)))
    for _ in range(3):
        d = rng.standard_normal(f.shape)
        eps = 1e-2
        fd = (red.J(f + eps * d) - red.J(f - eps * d)) / (2 * eps)
        assert abs(fd) <= 1e-9 * scale * np.linalg.norm(d)


def test_fd_gradient_matches_adjoint_gradient():
    prob = make_custom((3, 3, 2), 5, 9, lattice=2)
    red = reduced.Reduced(prob)
    rng = np.random.default_rng(4)
    f = rng.standard_normal((prob.M + 1, prob.N))
    g = red.grad(f)
    for _ in range(3):
        d = rng.standard_normal(f.shape)
        eps = 1e-3
        fd = (red.J(f + eps * d) - red.J(f - eps * d)) / (2 * eps)
        assert abs(fd - np.sum(g * d)) <= 1e-9 * np.linalg.norm(g) * np.linalg.norm(d)


def test_state_and_adjoint_time_marching():
    prob = make_custom((4, 3, 3), 5, 12, lattice=2)
    F, b, U = _solve_direct(prob)
    X = U.reshape(prob.M + 1, prob.N, 3)
    C, G, f = X[:, :, 0], X[:, :, 1], X[:, :, 2]
    red = reduced.Reduced(prob)
    Cm = red.forward(f)
    assert np.linalg.norm(C - Cm) <= 1e-12 * np.linalg.norm(C)
    # backward march of the multiplier: A1'^T G^n = -A2''^T G^{n+1} - w_n S (C^n - d^n)
    g = red.w[:, None] * red.S[None, :] * (C - red.d)
    lam = np.zeros((prob.M + 2, prob.N))
    for n in range(prob.M, 0, -1):
        lam[n] = red.lu.solve(-red.A2pp.T @ lam[n + 1] - g[n], trans="T")
    P = red.ops.interior.astype(float)
    lam[0] = P * (-(red.A2pp.T @ lam[1]) - g[0])
    assert np.linalg.norm(G - lam[:-1]) <= 1e-11 * np.linalg.norm(G)


def test_paper_dof_count():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "paper_dof_counts.txt"))
            if l.strip() and not l.startswith("#")]
    from workloads.generate import Problem
    for nodes, levels, dof in rows:
        n = int(nodes) - 1
        p = Problem(n=(n, n, n), M=int(levels) - 1, a_elem=np.ones(1), v=(0, 0, 0), beta1=1, beta2=1,
                    sensor_node=np.zeros(0, np.int32), data=np.zeros((int(levels), 0)))
        assert p.unknowns == int(dof)


def test_otd_structure():
    """OTD shares the state rows and W with DTO; its G rows are the time-shifted
    transposed state operator (Appendix A: B1 = A1^T, B2 = A2^T), G^M = 0, and
    the f rows couple G through the space-time mass -Tt x B."""
    pd = make_custom((3, 3, 2), 4, 2, lattice=1, variant=DTO)
    po = make_custom((3, 3, 2), 4, 2, lattice=1, variant=OTD)
    Fd, Fo = kkt.assemble(pd).toarray(), kkt.assemble(po).toarray()
    N, M = pd.N, pd.M
    tau = pd.T / M
    idx = lambda n, c: 3 * (n * N + np.arange(N)) + c
    allc = lambda c: np.concatenate([idx(n, c) for n in range(M + 1)])
    # identical state rows and f-f blocks
    assert np.array_equal(Fd[allc(0)], Fo[allc(0)])
    assert np.array_equal(Fd[np.ix_(allc(2), allc(2))], Fo[np.ix_(allc(2), allc(2))])
    # G^M = 0 row
    assert np.array_equal(Fo[idx(M, 1)][:, idx(M, 1)], np.eye(N))
    assert np.abs(np.delete(Fo[idx(M, 1)], idx(M, 1), axis=1)).max() == 0
    # OTD G-G block at level n equals DTO's at level n+1 shifted by one level
    for n in range(M - 1):
        assert np.array_equal(Fo[np.ix_(idx(n, 1), idx(n, 1))], Fd[np.ix_(idx(n + 1, 1), idx(n + 1, 1))])
        assert np.array_equal(Fo[np.ix_(idx(n, 1), idx(n + 1, 1))], Fd[np.ix_(idx(n + 1, 1), idx(n + 2, 1))])
    # f-G coupling is minus the space-time mass matrix (columns on Dirichlet nodes removed)
    ops = fem.spatial_ops(po)
    Tt = fem.time_mass(M, tau).toarray()
    Bp = ops.B.toarray() * ops.interior[None, :]
    for n in range(M + 1):
        for m in range(M + 1):
            assert np.allclose(Fo[np.ix_(idx(n, 2), idx(m, 1))], -Tt[n, m] * Bp, rtol=0, atol=1e-16)


def test_otd_solution_close_to_dto():
    """Both variants discretise the same continuous optimality system."""
    pd = make_custom((4, 4, 4), 6, 30, lattice=2, variant=DTO)
    po = make_custom((4, 4, 4), 6, 30, lattice=2, variant=OTD)
    _, _, Ud = _solve_direct(pd)
    _, _, Uo = _solve_direct(po)
    Cd = Ud.reshape(-1, 3)[:, 0]
    Co = Uo.reshape(-1, 3)[:, 0]
    assert np.linalg.norm(Cd - Co) < 0.5 * np.linalg.norm(Cd)


def _lumped(nn, h):
    """Integrals of the 1-D hat functions on a uniform grid: h/2 at the ends, h inside."""
    w = np.full(nn, h)
    w[0] = w[-1] = h / 2
    return w


def test_h1l2_regularisation_block_closed_form():
    """The H1-L2 regularisation of Example 2 changes only the f-f block, by
    beta2 Tt x (B - K).  On f = 1 (C = G = 0) the f rows change by
    beta2 (integral of the time hat of level n) (integral of the space hat of
    node j), since the stiffness matrix annihilates constants: both integrals
    are products of 1-D lumped weights."""
    p1 = make_custom((3, 4, 2), 4, 5, lattice=2, length=(1.0, 0.7, 1.3), T=0.8)
    p2 = dataclasses.replace(p1, reg=H1L2)
    D = (kkt.assemble(p2) - kkt.assemble(p1)).tocoo()
    nz = np.abs(D.data) > 0
    assert nz.any() and np.all(D.row[nz] % 3 == 2) and np.all(D.col[nz] % 3 == 2)
    e = np.zeros(D.shape[0])
    e[2::3] = 1.0
    r = (D.tocsr() @ e).reshape(p1.M + 1, p1.N, 3)
    assert np.abs(r[:, :, :2]).max() == 0.0
    nx, ny, nz_ = p1.nodes
    wx = _lumped(nx, 1.0 / p1.n[0])
    wy = _lumped(ny, 0.7 / p1.n[1])
    wz = _lumped(nz_, 1.3 / p1.n[2])
    wt = _lumped(p1.M + 1, 0.8 / p1.M)
    space = (wz[:, None, None] * wy[None, :, None] * wx[None, None, :]).ravel()
    want = p1.beta2 * wt[:, None] * space[None, :]
    assert np.allclose(r[:, :, 2], want, rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("shape", [((3, 2, 2), 3), ((4, 3, 3), 4)])
def test_h1l2_matches_reduced_cg(shape):
    """The H1-L2 KKT solution minimises the reduced functional with the L2
    space term (reduced-space CG on the normal equations)."""
    prob = make_custom(shape[0], shape[1], 21, lattice=2, reg=H1L2)
    _, _, U = _solve_direct(prob)
    f_kkt = U.reshape(prob.M + 1, prob.N, 3)[:, :, 2]
    f_cg, its = reduced.Reduced(prob).cg(tol=1e-13)
    assert np.linalg.norm(f_kkt - f_cg) <= 1e-8 * np.linalg.norm(f_cg)


def _smooth_sensor_data(base, M, seed=1):
    """Sensor values sin(pi (t + phase_s)) amp_s, sampled at t^n = n/M: smooth in time."""
    rng = np.random.default_rng(seed)
    s = base.sensor_node.size
    amp = rng.uniform(0.5, 1.5, s)
    phase = rng.uniform(0.0, 1.0, s)
    t = np.arange(M + 1) * base.T / M
    return np.sin(np.pi * (t[:, None] + phase[None, :])) * amp[None, :]


def _otd_rhs_shifted(prob):
    """A planted mistake: the OTD data term of level n taken one level late
    (tau/2 S (d^{n+1} + d^{n+2}), last level repeated)."""
    M, tau = prob.M, prob.T / prob.M
    d = np.zeros((M + 1, prob.N))
    d[:, prob.sensor_node] = prob.data
    d = np.concatenate([d[1:], d[-1:]])
    b = np.zeros((M + 1, prob.N, 3))
    b[:M, :, 1] = 0.5 * tau * (d[:M] + d[1:])
    return b.ravel()


def _otd_rhs_rectangle(prob):
    """A planted mistake: the data term of level n as tau S d^n (left rectangle
    rule instead of the interval average of Appendix A)."""
    M, tau = prob.M, prob.T / prob.M
    d = np.zeros((M + 1, prob.N))
    d[:, prob.sensor_node] = prob.data
    b = np.zeros((M + 1, prob.N, 3))
    b[:M, :, 1] = tau * d[:M]
    return b.ravel()


def test_otd_rhs_second_order_in_time():
    """Appendix A's adjoint right-hand side tau/2 S (C^eps,n + C^eps,n+1) is the
    interval average of the data (Crank-Nicolson for the continuous adjoint
    equation of Section 2).  With the same spatial mesh, the OTD and DTO
    sources then discretise the same semi-discrete optimality system to second
    order in tau: on data smooth in time the relative gap |f_OTD - f_DTO|,
    sampled at common times, falls by about 4 per halving of tau.  A data term
    shifted by one level, or taken by the rectangle rule, is only first order
    (the gap halves), so either mistake in the oracle's OTD b fails here."""
    base = make_custom((3, 3, 3), 8, 5, lattice=2)
    orders = {"rhs": [], "shifted": [], "rectangle": []}
    prev = None
    for M in (16, 32, 64):
        pd = dataclasses.replace(base, M=M, data=_smooth_sensor_data(base, M), variant=DTO)
        po = dataclasses.replace(pd, variant=OTD)
        step = M // 8

        def f_of(prob, b):
            U = spla.spsolve(kkt.assemble(prob).tocsc(), b)
            return U.reshape(M + 1, prob.N, 3)[::step, :, 2]
        fd = f_of(pd, kkt.rhs(pd))
        gaps = {"rhs": f_of(po, kkt.rhs(po)), "shifted": f_of(po, _otd_rhs_shifted(po)),
                "rectangle": f_of(po, _otd_rhs_rectangle(po))}
        gaps = {k: np.linalg.norm(v - fd) / np.linalg.norm(fd) for k, v in gaps.items()}
        if prev is not None:
            for k in orders:
                orders[k].append(np.log2(prev[k] / gaps[k]))
        prev = gaps
    # observed orders at 16 -> 32 and 32 -> 64: about 1.74 and 1.92 for Appendix A's b
    assert orders["rhs"][-1] >= 1.8 and orders["rhs"][-1] > orders["rhs"][0]
    assert prev["rhs"] < 0.01
    for k in ("shifted", "rectangle"):
        assert orders[k][-1] <= 1.2, (k, orders[k])
