"""Pins of the oracle's GMRES / FGMRES, including the dense direct-solve check."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import kkt, krylov, ras
from workloads.generate import make_custom, DTO, OTD


def test_gmres_exact_in_n_steps():
    rng = np.random.default_rng(0)
    n = 12
    A = rng.standard_normal((n, n)) + 4 * np.eye(n)
    b = rng.standard_normal(n)
    x, st = krylov.gmres(lambda v: A @ v, lambda v: v, b, restart=n, rtol=1e-13)
    assert st.converged and st.iters <= n
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10)


def test_right_preconditioning_and_flexible():
    rng = np.random.default_rng(1)
    n = 40
    A = rng.standard_normal((n, n)) + 8 * np.eye(n)
    Dinv = 1.0 / np.diag(A)
    b = rng.standard_normal(n)
    ref = np.linalg.solve(A, b)
    x, st = krylov.gmres(lambda v: A @ v, lambda v: Dinv * v, b, restart=7, rtol=1e-12)
    assert st.converged and st.restarts > 0
    np.testing.assert_allclose(x, ref, rtol=1e-9)
    # a preconditioner that changes every call needs the flexible variant
    calls = [0]

    def varying(v):
        calls[0] += 1
        return (1.0 + 0.3 * np.sin(calls[0])) * Dinv * v
    x, st = krylov.gmres(lambda v: A @ v, varying, b, restart=7, rtol=1e-12, flexible=True)
    assert st.converged
    np.testing.assert_allclose(x, ref, rtol=1e-9)


def test_matches_scipy_gmres_solution():
    rng = np.random.default_rng(2)
    n = 60
    A = rng.standard_normal((n, n)) / np.sqrt(n) + 2 * np.eye(n)
    b = rng.standard_normal(n)
    x, st = krylov.gmres(lambda v: A @ v, lambda v: v, b, restart=20, rtol=1e-11)
    xs, info = spla.gmres(A, b, restart=20, rtol=1e-11, atol=0.0)
    assert info == 0 and st.converged
    np.testing.assert_allclose(x, xs, rtol=1e-8, atol=1e-10)


def test_fixed_iteration_mode():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30, 30)) + 6 * np.eye(30)
    b = rng.standard_normal(30)
    _, st = krylov.gmres(lambda v: A @ v, lambda v: v, b, restart=5, rtol=1e-14, fixed_iters=13)
    assert st.iters == 13 and st.restarts == 2


@pytest.mark.parametrize("variant", [DTO, OTD])
@pytest.mark.parametrize("shape", [((2, 2, 2), 2), ((3, 2, 3), 3), ((3, 3, 3), 4)])
def test_ras_gmres_matches_dense_direct(variant, shape):
    """Direct-solve check: GMRES + one-level RAS at rtol 1e-12 vs a dense solve."""
    prob = make_custom(shape[0], shape[1], 40 + shape[1], lattice=1, variant=variant)
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    b = kkt.rhs(prob)
    U = np.linalg.solve(F.toarray(), b)
    R = ras.RAS(prob, (2, 1, 2, 2), 1, terms=terms)
    x, st = krylov.gmres(lambda v: F @ v, R.apply, b, restart=30, rtol=1e-12)
    assert st.converged
    assert np.linalg.norm(x - U) <= 1e-9 * np.linalg.norm(U)
