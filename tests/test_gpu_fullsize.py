"""GPU checks at full size: cube32x64 (7,007,715 unknowns, 512 subdomains) and
cube48x96 (34,235,859 unknowns, two-level, the largest single-GPU workload).

The oracle cannot run the whole solve at these sizes in a test, so the matvec
is compared in full (level-by-level oracle), the preconditioner and its
factors on sampled subdomains, and the solves through their true residuals
(recomputed by the oracle) and, on a manufactured system, their error.
"""
import sys

import numpy as np
import pytest

from oracle import kkt, ras as oras
from workloads.generate import make_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full():
    import paper_1508_06103_amd as st
    prob, cfg = make_problem("cube32x64")
    _say(f"cube32x64: {prob.unknowns} unknowns; setting up on the GPU")
    op = st.KKTOperator(prob)
    pre = st.RAS(op, cfg.parts, cfg.overlap)
    torch.cuda.synchronize()
    terms = kkt.kkt_terms(prob)
    return st, prob, cfg, op, pre, terms


def test_fullsize_rhs_and_matvec(full):
    st, prob, cfg, op, pre, terms = full
    b_ref = kkt.rhs(prob)
    assert np.abs(op.b.cpu().numpy() - b_ref).max() <= 1e-15 * np.abs(b_ref).max()
    x = np.random.default_rng(7).standard_normal(prob.unknowns)
    y = op.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    y_ref = kkt.apply_terms(terms, x)
    err = np.abs(y - y_ref).max() / np.abs(y_ref).max()
    _say(f"  full-size matvec max rel err {err:.2e}")
    assert err <= 1e-13


def test_fullsize_boxes_bit_exact(full):
    st, prob, cfg, op, pre, terms = full
    subs = oras.subdomains(prob, cfg.parts, cfg.overlap)
    ref = np.array([list(s.own_lo) + list(s.own_hi) + list(s.box_lo) + list(s.box_hi) for s in subs])
    assert np.array_equal(pre.boxes(), ref)
    # factor storage is exactly the ILU(0) pattern: sum over boxes of prod(3 l - 2) blocks
    nblk = sum(int(np.prod([3 * l - 2 for l in s.dims])) for s in subs)
    assert pre.factor_bytes == nblk * 72


def test_fullsize_sampled_subdomains(full):
    st, prob, cfg, op, pre, terms = full
    subs = oras.subdomains(prob, cfg.parts, cfg.overlap)
    # one interior 12^4 box and one corner box
    cands = [i for i, s in enumerate(subs) if s.dims == (12, 12, 12, 12)]
    interior = cands[len(cands) // 2]
    pick = [0, interior]
    R = oras.RAS(prob, cfg.parts, cfg.overlap, terms=terms, subset=pick)
    r = np.random.default_rng(8).standard_normal(prob.unknowns)
    z = pre.apply(torch.from_numpy(r).cuda()).cpu().numpy()
    for sid in pick:
        zl = R.solve_sub(sid, r)
        own = R.own[sid]
        got = z[R.gidx[sid][own]]
        err = np.linalg.norm(got - zl[own]) / np.linalg.norm(zl[own])
        f_err = np.abs(pre.export_factors(sid) - R.ilu[sid].padded()).max() / np.abs(R.ilu[sid].padded()).max()
        _say(f"  sub {sid} dims {subs[sid].dims}: apply rel err {err:.2e}, factor max rel err {f_err:.2e}")
        assert err <= 1e-11 and f_err <= 1e-11


def test_fullsize_solve_true_residual(full):
    st, prob, cfg, op, pre, terms = full
    x, s = st.solve(op, pre, restart=cfg.restart, rtol=cfg.rtol)
    xh = x.cpu().numpy()
    b = kkt.rhs(prob)
    res = np.linalg.norm(b - kkt.apply_terms(terms, xh)) / np.linalg.norm(b)
    _say(f"  cube32x64 solve: {s.iters} its, {s.ms:.0f} ms, gpu res {s.rel_res_true:.2e}, oracle res {res:.2e}")
    assert s.converged and res <= 1e-6 * (1 + 1e-6)
    # deterministic: a second solve is bit-identical
    x2, s2 = st.solve(op, pre, restart=cfg.restart, rtol=cfg.rtol)
    assert s2.iters == s.iters and torch.equal(x, x2)


def test_fullsize_coarse_multi_rhs():
    """The exact coarse solve of the 48^3 x 96 two-level configuration (coarse
    12^3 x 24: 25 dense blocks of order 6591, FP32) with several right-hand
    sides per pass against the one-vector path, a column independent of the
    others bit for bit.  The coarse operator does not depend on the sensor
    data, so the operator is built with zero data (no forward model run)."""
    import paper_1508_06103_amd as st
    from workloads.generate import Problem, lattice_nodes
    n, M = 48, 96
    sensors = lattice_nodes(n, 5)   # the {8, ..., 40}^3 lattice: all on coarse nodes
    prob = Problem(n=(n, n, n), M=M, a_elem=np.ones(n ** 3), v=(1.0, 0.5, 0.25), beta1=1e-4, beta2=1e-4,
                   sensor_node=np.asarray(sensors, dtype=np.int32), data=np.zeros((M + 1, len(sensors))))
    op = st.KKTOperator(prob)
    C = st.Coarse(op, (4, 4, 4, 4), method=st.COARSE_LU, precision=st.F32)
    q = 5
    X = torch.randn(q, op.n, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    Y = C.apply_multi(X)
    worst = 0.0
    for i in range(q):
        y1 = C.apply(X[i].contiguous())
        worst = max(worst, (torch.linalg.norm(Y[i] - y1) / torch.linalg.norm(y1)).item())
    _say(f"  coarse 12^3 x 24, {q} vectors: largest rel diff to the one-vector path {worst:.2e}")
    assert worst <= 1e-4
    assert torch.equal(C.apply_multi(X[3:4].contiguous())[0], Y[3])


@pytest.fixture(scope="module")
def full48():
    """cube48x96 (34,235,859 unknowns) with the benchmark's operator."""
    import paper_1508_06103_amd as st
    prob, cfg = make_problem("cube48x96")
    _say(f"cube48x96: {prob.unknowns} unknowns")
    terms = kkt.kkt_terms(prob)
    return st, prob, cfg, terms


def test_fullsize48_manufactured_two_level_f64_and_f32(full48):
    """The largest single-GPU configuration end to end on a manufactured system
    F x* = b (x* a seeded smooth vector, b from the oracle's level-by-level
    product): two-level FGMRES(50) with the exact coarse LU (coarse 12^3 x 24),
    FP64 factors and FP32 factors.  Both true residuals, recomputed by the
    oracle, meet 1e-6; the C and f errors against x* and between the two
    paths are printed, and the mixed path's C and f lie within 1e-5 of the
    FP64 path's."""
    from workloads.generate import manufactured_solution
    st, prob, cfg, terms = full48
    xs = manufactured_solution(prob, seed=48)
    b = kkt.apply_terms(terms, xs)
    bd = torch.from_numpy(b).cuda()
    out = {}
    for name, prec in (("f64", st.F64), ("f32", st.F32)):
        op = st.KKTOperator(prob)
        pre = st.RAS(op, cfg.parts, cfg.overlap, precision=prec)
        C = st.Coarse(op, cfg.coarse_factor, method=st.COARSE_LU, precision=prec)
        x, s = st.solve(op, pre, bd, coarse=C, restart=cfg.restart, rtol=cfg.rtol, flexible=True)
        xh = x.cpu().numpy()
        res = np.linalg.norm(b - kkt.apply_terms(terms, xh)) / np.linalg.norm(b)
        e = [np.linalg.norm(xh[c::3] - xs[c::3]) / np.linalg.norm(xs[c::3]) for c in (0, 2)]
        _say(f"  {name}: {s.iters} its, {s.ms:.0f} ms ({pre.apply_rows} rows per phase), gpu res "
             f"{s.rel_res_true:.2e}, oracle res {res:.2e}, error vs x*: C {e[0]:.2e} f {e[1]:.2e}")
        assert s.converged and res <= 1e-6 * (1 + 1e-6)
        out[name] = xh
        C.close()
        pre.close()
        op.close()
        del x
        torch.cuda.empty_cache()
    d = [np.linalg.norm(out["f32"][c::3] - out["f64"][c::3]) / np.linalg.norm(out["f64"][c::3]) for c in (0, 2)]
    _say(f"  FP32 preconditioners vs FP64: C {d[0]:.2e} f {d[1]:.2e}")
    assert d[0] <= 1e-5 and d[1] <= 1e-5


def test_fullsize48_sampled_subdomains_ring64(full48):
    """The FP64 apply of cube48x96 runs the 64-row LDS ring: a corner box and an
    interior 14^4 box against the oracle's ILU(0) solves (owned rows, per slot),
    and their factors."""
    st, prob, cfg, terms = full48
    op = st.KKTOperator(prob)
    pre = st.RAS(op, cfg.parts, cfg.overlap)
    assert pre.apply_rows == 64
    subs = oras.subdomains(prob, cfg.parts, cfg.overlap)
    cands = [i for i, s in enumerate(subs) if s.dims == (14, 14, 14, 14)]
    pick = [0, cands[len(cands) // 2]]
    R = oras.RAS(prob, cfg.parts, cfg.overlap, terms=terms, subset=pick)
    r = np.random.default_rng(9).standard_normal(prob.unknowns)
    z = pre.apply(torch.from_numpy(r).cuda()).cpu().numpy()
    for sid in pick:
        zl = R.solve_sub(sid, r)
        own = R.own[sid]
        got, want = z[R.gidx[sid][own]].reshape(-1, 3), zl[own].reshape(-1, 3)
        slot = np.abs(got - want).max(axis=0) / np.abs(want).max(axis=0)
        fp = R.ilu[sid].padded()
        f_err = np.abs(pre.export_factors(sid) - fp).max() / np.abs(fp).max()
        _say(f"  sub {sid} dims {subs[sid].dims}: apply per slot max rel err "
             f"{', '.join(f'{e:.1e}' for e in slot)}, factor max rel err {f_err:.2e}")
        assert slot.max() <= 1e-10 and f_err <= 1e-11
    pre.close()
    op.close()
