"""GPU parity of the two-level space-time preconditioner against the oracle.

The coarse correction y = I_c^h F_c^{-1} I_h^c x (F_c^{-1} = GMRES(maxit) from
zero, right-preconditioned by the coarse mesh's RAS) is compared element by
element; the two-level FGMRES solve is compared by iteration count and, at a
fixed number of Arnoldi steps, by its iterate.
"""
import sys

import numpy as np
import pytest

from oracle import kkt, krylov, ras as oras, twolevel
from workloads.generate import make_custom, make_problem, OTD

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def st():
    import paper_1508_06103_amd as st_mod
    assert torch.cuda.is_available()
    return st_mod


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _grid_sensors(n, fac, picks, faces=0b000011):
    """Sensor node ids on coarse nodes: picks = list of (I, J, K) coarse indices."""
    nn = (n[0] + 1, n[1] + 1)
    return np.array([I * fac[0] + nn[0] * (J * fac[1] + nn[1] * K * fac[2]) for I, J, K in picks], dtype=np.int32)


def case(name):
    if name == "cube8x16":
        return make_problem("cube8x16")[0], (2, 2, 2, 2), (2, 2, 2, 2)
    if name == "aniso":
        n, fac = (6, 6, 4), (3, 2, 2, 3)
        sens = _grid_sensors(n, fac, [(1, 0, 0), (1, 1, 1), (1, 2, 2), (1, 3, 1), (1, 1, 2)])
        return make_custom(n, 6, 11, sensors=sens), fac, (1, 2, 1, 2)
    if name == "partial_axes":
        # coarsening in y and z only: the transfers skip the x and t axes
        return make_problem("cube8x16")[0], (1, 2, 2, 1), (2, 2, 2, 2)
    if name == "same_mesh":
        # factor 1 everywhere: the coarse mesh is the fine mesh
        n = (3, 2, 3)
        return make_custom(n, 4, 13, lattice=2), (1, 1, 1, 1), (1, 1, 1, 1)
    if name == "otd_neumann":
        n, fac = (4, 6, 6), (2, 3, 2, 2)
        sens = _grid_sensors(n, fac, [(1, 1, 1), (0, 1, 2), (2, 0, 1), (1, 2, 3)])
        return make_custom(n, 8, 12, sensors=sens, variant=OTD, faces=0), fac, (2, 1, 2, 2)
    raise KeyError(name)


@pytest.mark.parametrize("name,restrict,rtol", [("cube8x16", "transpose", 1e-12), ("cube8x16", "transpose", 0.1),
                                                ("cube8x16", "injection", 1e-12), ("aniso", "transpose", 1e-12),
                                                ("otd_neumann", "transpose", 0.1),
                                                ("partial_axes", "transpose", 1e-12),
                                                ("same_mesh", "transpose", 1e-12)])
def test_coarse_correction(st, name, restrict, rtol):
    prob, fac, cparts = case(name)
    _say(f"case {name}: factor {fac} coarse parts {cparts} restrict {restrict} rtol {rtol}")
    op = st.KKTOperator(prob)
    kind = st.RESTRICT_TRANSPOSE if restrict == "transpose" else st.RESTRICT_INJECTION
    C = st.Coarse(op, fac, cparts, overlap=1, maxit=4, rtol=rtol, restrict=kind, method=st.COARSE_GMRES_RAS)
    F = kkt.assemble(prob)
    tl = twolevel.TwoLevel(prob, None, None, fac, restrict=restrict, coarse="gmres_ras", coarse_parts=cparts,
                           coarse_overlap=1, coarse_maxit=4, coarse_rtol=rtol)
    for seed in (1, 2):
        x = np.random.default_rng(seed).standard_normal(F.shape[0])
        y = C.apply(_dev(x)).cpu().numpy()
        y_ref = tl.coarse_correction(x)
        err = np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)
        # elementwise, per unknown slot (C, G, f)
        ys, yr = y.reshape(-1, 3), y_ref.reshape(-1, 3)
        slot_err = np.abs(ys - yr).max(axis=0) / np.abs(yr).max(axis=0)
        _say(f"  seed {seed}: coarse correction rel err {err:.2e}, per slot max "
             f"{', '.join(f'{e:.1e}' for e in slot_err)}")
        assert err <= 1e-10 and slot_err.max() <= 1e-9


@pytest.mark.parametrize("name,restart", [("cube8x16", 30), ("aniso", 20)])
def test_two_level_fgmres_parity(st, name, restart):
    prob, fac, cparts = case(name)
    parts = {"cube8x16": (2, 2, 2, 2), "aniso": (2, 2, 1, 2)}[name]
    _say(f"case {name}: two-level FGMRES({restart}), fine parts {parts}")
    op = st.KKTOperator(prob)
    pre = st.RAS(op, parts, 1)
    C = st.Coarse(op, fac, cparts, overlap=1, maxit=4, rtol=0.1, method=st.COARSE_GMRES_RAS)
    x, s = st.solve(op, pre, coarse=C, restart=restart, rtol=1e-6, flexible=True)
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    b = kkt.rhs(prob)
    A = lambda v: F @ v
    R = oras.RAS(prob, parts, 1, terms=terms)
    tl = twolevel.TwoLevel(prob, R.apply, A, fac, coarse="gmres_ras", coarse_parts=cparts, coarse_overlap=1,
                           coarse_maxit=4, coarse_rtol=0.1)
    xo, so = krylov.gmres(A, tl, b, restart=restart, rtol=1e-6, flexible=True)
    xg = x.cpu().numpy()
    res = np.linalg.norm(b - F @ xg) / np.linalg.norm(b)
    _say(f"  gpu its {s.iters} oracle its {so.iters} true res {res:.2e}")
    assert s.converged and res <= 1e-6
    assert abs(s.iters - so.iters) <= 1
    k = so.iters
    x2, _ = st.solve(op, pre, coarse=C, restart=restart, rtol=1e-6, flexible=True, fixed_iters=k)
    xo2, _ = krylov.gmres(A, tl, b, restart=restart, rtol=1e-6, flexible=True, fixed_iters=k)
    e = np.linalg.norm(x2.cpu().numpy() - xo2) / np.linalg.norm(xo2)
    _say(f"  fixed {k} iterations: rel diff {e:.2e}")
    assert e <= 1e-7


def test_two_level_cuts_iterations(st):
    """Space-time coarse correction reduces the FGMRES count of the one-level method."""
    nn = 13
    idx = [3, 6, 9]
    sens = np.array([i + nn * (j + nn * k) for k in idx for j in idx for i in idx], dtype=np.int32)
    prob = make_custom((12, 12, 12), 16, 4, sensors=sens)
    op = st.KKTOperator(prob)
    pre = st.RAS(op, (3, 3, 3, 4), 1)
    _, s1 = st.solve(op, pre, restart=50, rtol=1e-6)
    C = st.Coarse(op, (3, 3, 3, 4), (2, 2, 2, 2), overlap=1, maxit=4, rtol=0.1, method=st.COARSE_GMRES_RAS)
    x, s2 = st.solve(op, pre, coarse=C, restart=50, rtol=1e-6, flexible=True)
    _say(f"  one-level {s1.iters} its, two-level {s2.iters} its")
    assert s1.converged and s2.converged and s2.iters < s1.iters
    F = kkt.assemble(prob)
    b = kkt.rhs(prob)
    assert np.linalg.norm(b - F @ x.cpu().numpy()) <= 1e-6 * np.linalg.norm(b)


def test_coarse_errors(st):
    prob, fac, cparts = case("cube8x16")
    op = st.KKTOperator(prob)
    with pytest.raises(st.StkktError) as e:
        st.Coarse(op, (3, 2, 2, 2), cparts, method=st.COARSE_GMRES_RAS)          # 3 does not divide 8
    assert e.value.code == st.EINVAL
    n = (8, 8, 8)
    odd = make_custom(n, 8, 5, sensors=np.array([3 + 9 * (2 + 9 * 2)], dtype=np.int32))
    op_odd = st.KKTOperator(odd)
    with pytest.raises(st.StkktError):
        st.Coarse(op_odd, (2, 2, 2, 2), cparts, method=st.COARSE_GMRES_RAS)      # sensor at x = 3 is not a coarse node
    with pytest.raises(st.StkktError):
        st.Coarse(op, fac, cparts, maxit=0, method=st.COARSE_GMRES_RAS)
    C = st.Coarse(op, fac, cparts, method=st.COARSE_GMRES_RAS)
    other = st.KKTOperator(prob)
    pre_other = st.RAS(other, (2, 2, 2, 2), 1)
    with pytest.raises(st.StkktError):
        st.solve(other, pre_other, coarse=C, flexible=True)


@pytest.mark.parametrize("name,precision,tol", [("cube8x16", "f64", 1e-9), ("aniso", "f64", 1e-9),
                                                ("otd_neumann", "f64", 1e-9), ("cube8x16", "f32", 1e-4),
                                                ("partial_axes", "f64", 1e-9), ("same_mesh", "f64", 1e-9)])
def test_coarse_lu_correction(st, name, precision, tol):
    """Exact coarse solve (block elimination in time) against the oracle's block LU."""
    prob, fac, _ = case(name)
    _say(f"case {name}: coarse LU ({precision}), factor {fac}")
    op = st.KKTOperator(prob)
    C = st.Coarse(op, fac, method=st.COARSE_LU, precision=st.F64 if precision == "f64" else st.F32)
    tl = twolevel.TwoLevel(prob, None, None, fac, coarse="lu")
    for seed in (1, 2):
        x = np.random.default_rng(seed).standard_normal(prob.unknowns)
        y = C.apply(_dev(x)).cpu().numpy()
        y_ref = tl.coarse_correction(x)
        err = np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)
        _say(f"  seed {seed}: rel err {err:.2e}")
        assert err <= tol


def test_two_level_lu_fgmres_parity(st):
    prob, fac, cparts = case("cube8x16")
    op = st.KKTOperator(prob)
    pre = st.RAS(op, (2, 2, 2, 2), 1)
    C = st.Coarse(op, fac, method=st.COARSE_LU)
    x, s = st.solve(op, pre, coarse=C, restart=30, rtol=1e-6, flexible=True)
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    b = kkt.rhs(prob)
    A = lambda v: F @ v
    R = oras.RAS(prob, (2, 2, 2, 2), 1, terms=terms)
    tl = twolevel.TwoLevel(prob, R.apply, A, fac, coarse="lu")
    xo, so = krylov.gmres(A, tl, b, restart=30, rtol=1e-6, flexible=True)
    res = np.linalg.norm(b - F @ x.cpu().numpy()) / np.linalg.norm(b)
    _say(f"  two-level (coarse LU): gpu {s.iters} its, oracle {so.iters} its, true res {res:.2e}")
    assert s.converged and res <= 1e-6 and abs(s.iters - so.iters) <= 1
    k = so.iters
    x2, _ = st.solve(op, pre, coarse=C, restart=30, rtol=1e-6, flexible=True, fixed_iters=k)
    xo2, _ = krylov.gmres(A, tl, b, restart=30, rtol=1e-6, flexible=True, fixed_iters=k)
    e = np.linalg.norm(x2.cpu().numpy() - xo2) / np.linalg.norm(xo2)
    _say(f"  fixed {k} steps: rel diff {e:.2e}")
    assert e <= 1e-7


def _mid_case():
    """16^3 elements x 16 steps with sensors on coarse nodes: coarse level 8^3 x 8
    (2187 unknowns per level, 9 levels), so the dense block products span many
    row tiles and column chunks, with ragged tails."""
    n, fac = (16, 16, 16), (2, 2, 2, 2)
    sens = _grid_sensors(n, fac, [(1, 1, 1), (4, 4, 4), (6, 2, 5), (3, 7, 2), (5, 5, 6), (2, 6, 3)])
    return make_custom(n, 16, 5, sensors=sens), fac


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name,precision,tol", [("cube8x16", "f64", 1e-9), ("aniso", "f64", 1e-9),
                                                ("cube8x16", "f32", 1e-4), ("mid", "f64", 1e-9),
                                                ("mid", "f32", 1e-4)])
def test_coarse_lu_multi_rhs(st, name, precision, tol):
    """Several coarse right-hand sides in one pass over the dense blocks (matrix
    cores): sampled columns against the oracle's block LU, every column against
    the one-vector path, a column independent of the others and of its
    position (bit for bit), strided operands, more than 16 columns."""
    prob, fac = _mid_case() if name == "mid" else case(name)[:2]
    _say(f"case {name}: multi-RHS coarse LU ({precision}), factor {fac}")
    op = st.KKTOperator(prob)
    C = st.Coarse(op, fac, method=st.COARSE_LU, precision=st.F64 if precision == "f64" else st.F32)
    tl = twolevel.TwoLevel(prob, None, None, fac, coarse="lu")
    q, n = 19, prob.unknowns
    X = np.random.default_rng(31).standard_normal((q, n))
    Xd = _dev(X)
    Yh = C.apply_multi(Xd).cpu().numpy()
    for i in (0, 7, 16, 18):
        err = _rel(Yh[i], tl.coarse_correction(X[i]))
        _say(f"  column {i}: rel err vs oracle {err:.2e}")
        assert err <= tol
    worst = max(_rel(Yh[i], C.apply(Xd[i].contiguous()).cpu().numpy()) for i in range(q))
    _say(f"  largest rel diff to the one-vector path: {worst:.2e}")
    assert worst <= (1e-12 if precision == "f64" else tol)
    sub = C.apply_multi(Xd[[18, 3, 7]].contiguous()).cpu().numpy()
    assert np.array_equal(sub, Yh[[18, 3, 7]])
    one = C.apply_multi(Xd[5:6].contiguous()).cpu().numpy()
    assert np.array_equal(one[0], Yh[5])
    Xs = torch.zeros((q, n + 37), dtype=torch.float64, device="cuda")
    Xs[:, :n] = Xd
    Ys = torch.full((q, n + 11), 7.0, dtype=torch.float64, device="cuda")
    C.apply_multi(Xs[:, :n], Ys[:, :n])
    assert np.array_equal(Ys[:, :n].cpu().numpy(), Yh)
    assert bool(torch.all(Ys[:, n:] == 7.0))


def test_coarse_multi_rhs_gmres_and_errors(st):
    """With the inner coarse GMRES the applications run one by one (same result
    as apply); q = 0 does nothing; short strides and overlapping operands fail."""
    prob, fac, cparts = case("cube8x16")
    op = st.KKTOperator(prob)
    C = st.Coarse(op, fac, cparts, overlap=1, maxit=4, rtol=0.1, method=st.COARSE_GMRES_RAS)
    n = prob.unknowns
    Xd = _dev(np.random.default_rng(32).standard_normal((3, n)))
    Y = C.apply_multi(Xd)
    for i in range(3):
        assert torch.equal(Y[i], C.apply(Xd[i].contiguous()))
    C.apply_multi(Xd[:0])
    short = torch.as_strided(Xd, (2, n), (n - 1, 1))
    with pytest.raises(st.StkktError):
        C.apply_multi(short, torch.empty((2, n), dtype=torch.float64, device="cuda"))
    with pytest.raises(st.StkktError):
        C.apply_multi(Xd, Xd)


def test_coarse_lu_multi_rhs_injection(st):
    """Several right-hand sides with the injection restriction: columns against
    the oracle, and bit for bit equal to the one-vector path (FP64 blocks take
    the same matrix-core pass for one vector)."""
    prob, fac, _ = case("cube8x16")
    op = st.KKTOperator(prob)
    C = st.Coarse(op, fac, method=st.COARSE_LU, restrict=st.RESTRICT_INJECTION)
    tl = twolevel.TwoLevel(prob, None, None, fac, restrict="injection", coarse="lu")
    X = np.random.default_rng(33).standard_normal((3, prob.unknowns))
    Xd = _dev(X)
    Y = C.apply_multi(Xd)
    for i in range(3):
        assert _rel(Y[i].cpu().numpy(), tl.coarse_correction(X[i])) <= 1e-9
        assert torch.equal(Y[i], C.apply(Xd[i].contiguous()))


@pytest.mark.parametrize("name", ["aniso", "mid"])
def test_coarse_lu_panel_paths(st, name, monkeypatch):
    """The Gauss-Jordan inversion of the Schur blocks with partial pivoting
    over all rows, the panel eliminated by one cooperative launch (64, 128 or
    256 rows per workgroup) or by two launches per column: all give the same
    coarse correction, and it matches the oracle's block LU.  The default,
    pivots searched among each panel's own rows, matches both.  The mid case
    (2187 rows per block) spans 35 panels and 9 to 35 workgroups with ragged
    tails."""
    prob, fac = _mid_case() if name == "mid" else case(name)[:2]
    op = st.KKTOperator(prob)
    x = np.random.default_rng(77).standard_normal(prob.unknowns)
    xd = _dev(x)
    ys = {}
    for rows in ("0", "64", "128", "256"):
        monkeypatch.setenv("STKKT_COARSE_PANEL_ROWS", rows)
        _say(f"case {name}: coarse LU, panel rows {rows}")
        C = st.Coarse(op, fac, method=st.COARSE_LU)
        ys[rows] = C.apply(xd).cpu().numpy()
        del C
    monkeypatch.delenv("STKKT_COARSE_PANEL_ROWS")
    _say(f"case {name}: coarse LU, pivots within each panel (default)")
    C = st.Coarse(op, fac, method=st.COARSE_LU)
    ys["block"] = C.apply(xd).cpu().numpy()
    del C
    y_ref = twolevel.TwoLevel(prob, None, None, fac, coarse="lu").coarse_correction(x)
    err = _rel(ys["128"], y_ref)
    _say(f"  rel err vs oracle {err:.2e}")
    assert err <= 1e-9
    for rows in ("0", "64", "256"):
        d = _rel(ys[rows], ys["128"])
        _say(f"  panel rows {rows} vs 128: rel diff {d:.2e}")
        assert d <= 1e-12
    err_b, d_b = _rel(ys["block"], y_ref), _rel(ys["block"], ys["128"])
    _say(f"  pivots within panels: rel err vs oracle {err_b:.2e}, vs global pivoting {d_b:.2e}")
    assert err_b <= 1e-9 and d_b <= 1e-11


def test_coarse_lu_panel_barrier_timeout_is_reported(st, monkeypatch):
    """The cooperative panel elimination bounds every grid-barrier wait.  With
    the bound forced to zero polls from the host, a workgroup that has to wait
    gives up at once, the launch ends on every workgroup, and coarse_setup
    reports the failure; the next setup, with the default bound, is correct."""
    prob, fac = _mid_case()
    op = st.KKTOperator(prob)
    monkeypatch.setenv("STKKT_COARSE_PANEL_ROWS", "128")
    monkeypatch.setenv("STKKT_COARSE_SPIN_LIMIT", "0")
    _say("case mid: coarse LU with a zero barrier wait bound")
    with pytest.raises(st.StkktError) as ei:
        st.Coarse(op, fac, method=st.COARSE_LU)
    _say(f"  error: {ei.value}")
    assert "timed out" in str(ei.value)
    monkeypatch.delenv("STKKT_COARSE_SPIN_LIMIT")
    C = st.Coarse(op, fac, method=st.COARSE_LU)
    x = np.random.default_rng(78).standard_normal(prob.unknowns)
    y = C.apply(_dev(x)).cpu().numpy()
    err = _rel(y, twolevel.TwoLevel(prob, None, None, fac, coarse="lu").coarse_correction(x))
    _say(f"  default bound: rel err vs oracle {err:.2e}")
    assert err <= 1e-9
