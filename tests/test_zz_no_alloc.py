"""kkt_rhs_noalloc: the right-hand side without device allocation, against
kkt_rhs (bit for bit) and the oracle, on two calls in a row (the second with
a smaller input), plus the size limit of its static staging array."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import kkt
from workloads.generate import Problem, make_custom, make_problem, redraw_noise

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


def _counting_allocator(st):
    alloc = st.TorchAllocator()
    grant = alloc._alloc_cb
    calls = {"n": 0}

    def counted(nbytes, ctx):
        calls["n"] += 1
        return grant(nbytes, ctx)

    alloc._counted_cb = st.ALLOC_FN(counted)
    alloc.struct = st._Alloc(alloc._counted_cb, alloc._free_cb, None)
    return alloc, calls


def test_rhs_noalloc_matches_rhs(st):
    big, _ = make_problem("cube8x16")                      # 17 levels x 27 sensors
    small = make_custom((4, 4, 3), 6, 7, lattice=2)        # 7 levels x 8 sensors
    assert big.data.size > small.data.size
    for k, prob in enumerate((big, small)):
        alloc, calls = _counting_allocator(st)
        op = st.KKTOperator(prob, allocator=alloc)
        data = redraw_noise(prob, 600 + k)
        ref = op.rhs(data)
        out = torch.full_like(ref, float("nan"))
        torch.cuda.synchronize()
        before = calls["n"]
        op.rhs_noalloc(data, out)
        torch.cuda.synchronize()
        assert calls["n"] == before, "kkt_rhs_noalloc allocated through the allocator"
        want = kkt.rhs(dataclasses.replace(prob, data=data))
        err = np.abs(out.cpu().numpy() - want).max() / np.abs(want).max()
        _say(f"  call {k}: {prob.M + 1} levels x {prob.sensor_node.size} sensors: equal to kkt_rhs "
             f"{torch.equal(out, ref)}, vs oracle {err:.1e}")
        assert torch.equal(out, ref)
        assert err <= 1e-15


def test_rhs_noalloc_rejects_oversize_data(st):
    """(nt+1) x n_sensors beyond the 1 MiB staging array: EINVAL, b untouched."""
    n, M = 6, 1400
    nn = n + 1
    sens = np.array([i + nn * (j + nn * k) for k in range(1, 6) for j in range(1, 6) for i in range(1, 5)],
                    dtype=np.int32)   # 100 interior nodes
    prob = Problem(n=(n, n, n), M=M, a_elem=np.ones(n ** 3), v=(1.0, 0.5, 0.25), beta1=1e-4, beta2=1e-4,
                   sensor_node=sens, data=np.zeros((M + 1, sens.size)))
    op = st.KKTOperator(prob)
    assert 8 * (M + 1) * sens.size > st.RHS_SCRATCH_BYTES
    out = torch.full((op.n,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(st.StkktError) as e:
        op.rhs_noalloc(np.ones((M + 1, sens.size)), out)
    assert e.value.code == st.EINVAL and "kkt_rhs" in str(e.value)
    assert bool((out == 7.0).all())
    ok = op.rhs(np.ones((M + 1, sens.size)))   # the allocating form still serves it
    assert torch.count_nonzero(ok).item() > 0
