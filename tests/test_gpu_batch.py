"""Batched instances on the GPU: parity of every instance with the oracle,
and each result the same alone and in the mix."""
import sys

import numpy as np
import pytest

from oracle import kkt, krylov, ras as oras
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


# uneven instances: shapes, variants and partitions differ; "tall" needs the
# apply kernel without the LDS ring
MIX = [
    ("cube8x16", None, (2, 2, 2, 2), 1),
    ("ragged", dict(n=(5, 6, 7), M=9, seed=3, lattice=2), (2, 3, 2, 3), 1),
    ("aniso_otd", dict(n=(7, 3, 4), M=6, seed=4, lattice=2, variant=OTD, faces=0b010011), (2, 1, 2, 2), 1),
    ("tall", dict(n=(2, 2, 40), M=24, seed=6, lattice=1), (1, 1, 2, 2), 1),
    ("small", dict(n=(4, 4, 4), M=5, seed=5, lattice=2, faces=0), (1, 2, 2, 1), 0),
]


def build(st, name, spec, parts, delta, precision):
    if spec is None:
        prob = make_problem(name)[0]
    else:
        spec = dict(spec)
        prob = make_custom(spec.pop("n"), spec.pop("M"), spec.pop("seed"), **spec)
    op = st.KKTOperator(prob)
    return prob, op, st.RAS(op, parts, delta, precision=precision)


def test_batch_matches_oracle_and_alone(st):
    built = [build(st, *m, precision=st.F64) for m in MIX]
    ops = [b[1] for b in built]
    pres = [b[2] for b in built]
    xs, sts = st.solve_batch(ops, pres, restart=20, rtol=1e-6)
    for (name, _, parts, delta), (prob, op, pre), x, s in zip(MIX, built, xs, sts):
        terms = kkt.kkt_terms(prob)
        F = kkt.assemble(prob, terms=terms)
        b = kkt.rhs(prob)
        R = oras.RAS(prob, parts, delta, terms=terms)
        A = lambda v: F @ v
        xo, so = krylov.gmres(A, R.apply, b, restart=20, rtol=1e-6, flexible=True)
        xg = x.cpu().numpy()
        res = np.linalg.norm(b - F @ xg) / np.linalg.norm(b)
        _say(f"  {name}: batch {s.iters} its, oracle {so.iters} its, true res {res:.2e}")
        assert s.converged and res <= 1e-6
        assert abs(s.iters - so.iters) <= 1
        # alone: a batch of one gives the identical result
        x1, s1 = st.solve_batch([op], [pre], restart=20, rtol=1e-6)
        assert s1[0].iters == s.iters
        assert np.array_equal(x1[0].cpu().numpy(), xg), name
        # like for like with the oracle at a fixed number of steps
        k = so.iters
        xf, _ = st.solve_batch([op], [pre], restart=20, rtol=1e-6, fixed_iters=k)
        xof, _ = krylov.gmres(A, R.apply, b, restart=20, rtol=1e-6, flexible=True, fixed_iters=k)
        e = np.linalg.norm(xf[0].cpu().numpy() - xof) / np.linalg.norm(xof)
        _say(f"    fixed {k} steps: rel diff {e:.2e}")
        assert e <= 1e-7


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_graph_matches_eager(st, prec):
    """Cycles replayed from captured graphs (rotations and flags on the device,
    one host check per 8 steps) give the same bits as host-checked steps; with
    a restart of 12 every cycle replays two graphs, and the solves take several
    cycles, so graphs are replayed repeatedly with the engine's own work and
    synchronisations in between."""
    mix = [m for m in MIX if m[0] != "tall"]   # members that share one apply launch
    precision = st.F64 if prec == "f64" else st.F32
    built = [build(st, *m, precision=precision) for m in mix]
    ops = [b[1] for b in built]
    pres = [b[2] for b in built]
    xe, se = st.solve_batch(ops, pres, restart=12, rtol=1e-8, graph=False)
    xg, sg = st.solve_batch(ops, pres, restart=12, rtol=1e-8, graph=True)
    for (name, *_), a, b, sa, sb in zip(mix, xe, xg, se, sg):
        _say(f"  {name} ({prec}): eager {sa.iters} its / {sa.restarts} restarts, graph {sb.iters} / {sb.restarts}")
        assert sa.converged and sb.converged
        assert sa.iters == sb.iters and sa.restarts == sb.restarts
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), name


def test_batch_fixed_steps_in_mix(st):
    """Fixed-step mode over the whole mix equals the oracle instance by instance."""
    built = [build(st, *m, precision=st.F64) for m in MIX[:3]]
    xs, sts = st.solve_batch([b[1] for b in built], [b[2] for b in built], restart=7, rtol=1e-6, fixed_iters=17)
    for (name, _, parts, delta), (prob, op, pre), x, s in zip(MIX, built, xs, sts):
        assert s.iters == 17 and s.restarts == 2
        F = kkt.assemble(prob)
        R = oras.RAS(prob, parts, delta)
        xo, _ = krylov.gmres(lambda v: F @ v, R.apply, kkt.rhs(prob), restart=7, rtol=1e-6, flexible=True,
                             fixed_iters=17)
        e = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
        _say(f"  {name}: 17 steps (restart 7), rel diff {e:.2e}")
        assert e <= 1e-7


def test_batch_mixed_precision(st):
    """FP32 preconditioners inside the FP64 batched FGMRES reach the FP64 tolerance."""
    built = [build(st, *m, precision=st.F32) for m in MIX]
    xs, sts = st.solve_batch([b[1] for b in built], [b[2] for b in built], restart=20, rtol=1e-6)
    for (name, *_), (prob, op, pre), x, s in zip(MIX, built, xs, sts):
        F = kkt.assemble(prob)
        b = kkt.rhs(prob)
        res = np.linalg.norm(b - F @ x.cpu().numpy()) / np.linalg.norm(b)
        _say(f"  {name}: {s.iters} its, true res {res:.2e}")
        assert s.converged and res <= 1e-6


def test_batch_instances_generator(st):
    """A slice of the 64-instance workload (uneven sizes, sensors, noise, beta)."""
    from workloads.generate import batch_instances
    probs = batch_instances(count=6, base_seed=3000, max_n=12, max_M=24)
    ops, pres = [], []
    for p in probs:
        op = st.KKTOperator(p)
        ops.append(op)
        pres.append(st.RAS(op, (2, 2, 2, 2), 1, precision=st.F32))
    xs, sts = st.solve_batch(ops, pres, restart=50, rtol=1e-6)
    for p, x, s in zip(probs, xs, sts):
        F = kkt.assemble(p)
        b = kkt.rhs(p)
        res = np.linalg.norm(b - F @ x.cpu().numpy()) / np.linalg.norm(b)
        _say(f"  {p.name}: n={p.n} M={p.M}: {s.iters} its, true res {res:.2e}")
        assert s.converged and res <= 1e-6


def test_batch_errors(st):
    prob, op, pre = build(st, *MIX[0], precision=st.F64)
    other = st.KKTOperator(prob)
    with pytest.raises(st.StkktError):
        st.solve_batch([op, other], [pre, pre])


def test_batch_mixed_phase_sizes_and_solo_members(st):
    """One batched launch serves members with different LDS needs: a single
    14^4-node box in FP64 (its ring fits only with 64-row phases) makes the
    whole launch use 64-row phases, and a member with ILU(1) factors (which
    have no ring) is launched on its own beside it.  Each member's result
    equals its solve alone, bit for bit, and meets the tolerance on the
    assembled operator."""
    mix = [("big14", dict(n=(13, 13, 13), M=13, seed=9, lattice=2), (1, 1, 1, 1), 0), MIX[0], MIX[1]]
    built = [build(st, *m, precision=st.F64) for m in mix[:2]]
    prob, op, _ = build(st, *mix[2], precision=st.F64)
    built.append((prob, op, st.RAS(op, mix[2][2], mix[2][3], precision=st.F64, ilu_level=1)))
    assert built[0][2].apply_rows == 64 and built[1][2].apply_rows == 256 and built[2][2].apply_rows == 0
    ops = [b[1] for b in built]
    pres = [b[2] for b in built]
    xs, sts = st.solve_batch(ops, pres, restart=20, rtol=1e-6)
    for (name, *_), (prob, op, pre), x, s in zip(mix, built, xs, sts):
        xg = x.cpu().numpy()
        F = kkt.assemble(prob)
        b = kkt.rhs(prob)
        res = np.linalg.norm(b - F @ xg) / np.linalg.norm(b)
        x1, s1 = st.solve_batch([op], [pre], restart=20, rtol=1e-6)
        _say(f"  {name}: {s.iters} its in the mix, {s1[0].iters} alone, true res {res:.2e}")
        assert s.converged and res <= 1e-6
        assert s1[0].iters == s.iters
        assert np.array_equal(x1[0].cpu().numpy(), xg), name
