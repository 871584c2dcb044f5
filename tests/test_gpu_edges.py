"""Degenerate inputs of the solvers on the GPU: zero right-hand sides, an
exact initial guess, the shortest restart, alone and inside a batch."""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import kkt, krylov, ras as oras
from workloads.generate import make_custom, make_problem

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


@pytest.fixture(scope="module")
def pair(st):
    """Two small operators with their preconditioners and exact solutions."""
    out = []
    for prob in (make_problem("cube8x16")[0], make_custom((5, 6, 7), 9, 3, lattice=2)):
        op = st.KKTOperator(prob)
        pre = st.RAS(op, (2, 2, 2, 2), 1)
        F = kkt.assemble(prob).tocsc()
        xs = spla.spsolve(F, kkt.rhs(prob))
        out.append((prob, op, pre, F, xs))
    return out


def test_zero_rhs_single(st, pair):
    prob, op, pre, F, xs = pair[0]
    b = torch.zeros(op.n, dtype=torch.float64, device="cuda")
    x = torch.full_like(b, 3.0)   # x0 is ignored when b = 0: the solution is 0
    x, s = st.solve(op, pre, b, x, restart=10, rtol=1e-6)
    _say(f"  zero b: {s.iters} its, converged {s.converged}")
    assert s.converged and s.iters == 0
    assert torch.count_nonzero(x).item() == 0


def test_exact_initial_guess_single(st, pair):
    prob, op, pre, F, xs = pair[1]
    x = torch.from_numpy(xs.copy()).to("cuda")
    x, s = st.solve(op, pre, None, x, restart=10, rtol=1e-6)
    _say(f"  exact x0: {s.iters} its, true res {s.rel_res_true:.2e}")
    assert s.converged and s.iters == 0
    assert np.array_equal(x.cpu().numpy(), xs)


@pytest.mark.parametrize("graph", [False, True])
def test_zero_rhs_and_exact_guess_in_batch(st, pair, graph):
    """A zero right-hand side and an exact initial guess leave a batch at once,
    without changing the result of the member that iterates.  The zero-b member
    starts from x0 = 3 and must come back with the solution x = 0, as kkt_solve
    returns it."""
    (p0, op0, pre0, F0, xs0), (p1, op1, pre1, F1, xs1) = pair
    b0 = torch.zeros(op0.n, dtype=torch.float64, device="cuda")
    x_exact = torch.from_numpy(xs1.copy()).to("cuda")
    xs, sts = st.solve_batch([op0, op1, op0], [pre0, pre1, pre0], [b0, op1.b, op0.b],
                             [torch.full_like(b0, 3.0), x_exact, torch.zeros_like(b0)], restart=12, rtol=1e-6,
                             graph=graph)
    _say(f"  batch: iters {[s.iters for s in sts]}")
    assert sts[0].converged and sts[0].iters == 0 and torch.count_nonzero(xs[0]).item() == 0
    assert sts[1].converged and sts[1].iters == 0 and np.array_equal(xs[1].cpu().numpy(), xs1)
    assert sts[2].converged and sts[2].iters > 0
    alone, s_alone = st.solve_batch([op0], [pre0], [op0.b], [torch.zeros_like(b0)], restart=12, rtol=1e-6,
                                    graph=graph)
    assert s_alone[0].iters == sts[2].iters
    assert np.array_equal(alone[0].cpu().numpy(), xs[2].cpu().numpy())


@pytest.mark.parametrize("graph", [False, True])
def test_restart_one_fixed_steps(st, pair, graph):
    """GMRES(1) (a cycle shorter than one captured graph) at a fixed step count
    against the oracle's FGMRES(1)."""
    prob, op, pre, F, xs = pair[0]
    R = oras.RAS(prob, (2, 2, 2, 2), 1)
    b = kkt.rhs(prob)
    k = 7
    xo, _ = krylov.gmres(lambda v: F @ v, R.apply, b, restart=1, rtol=1e-6, flexible=True, fixed_iters=k)
    xg, sg = st.solve_batch([op], [pre], restart=1, rtol=1e-6, fixed_iters=k, graph=graph)
    x1, s1 = st.solve(op, pre, restart=1, rtol=1e-6, fixed_iters=k)
    for name, x, s in (("batch", xg[0], sg[0]), ("single", x1, s1)):
        e = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
        _say(f"  {name} GMRES(1), {s.iters} steps: rel diff {e:.2e}")
        assert s.iters == k and s.restarts == k - 1
        assert e <= 1e-7


@pytest.mark.parametrize("where", ["single", "batch"])
def test_non_finite_initial_guess_is_breakdown(st, pair, where):
    """A NaN in x0 makes the initial residual non-finite: the solve stops at once
    with EBREAKDOWN (alone, and for that member only in a batch)."""
    prob, op, pre, F, xs = pair[0]
    x = torch.zeros(op.n, dtype=torch.float64, device="cuda")
    x[17] = float("nan")
    if where == "single":
        _, s = st.solve(op, pre, None, x, restart=10, rtol=1e-6, raise_on_fail=False)
        assert s.status == st.EBREAKDOWN and s.iters == 0 and not s.converged
        return
    good = torch.zeros_like(x)
    _, sts = st.solve_batch([op, op], [pre, pre], None, [x, good], restart=10, rtol=1e-6, raise_on_fail=False)
    _say(f"  batch statuses {[s.status for s in sts]}, iters {[s.iters for s in sts]}")
    assert sts[0].status == st.EBREAKDOWN and sts[0].iters == 0
    assert sts[1].converged and sts[1].status == st.OK
