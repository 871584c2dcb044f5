"""Pins of the oracle's finite-element matrices against brute-force quadrature.

The quadrature below evaluates trilinear basis functions and their gradients
directly (no Kronecker products, no 1-D element matrices), so a transposed
convection matrix, a wrong sign or a mis-scaled mass would fail here.
"""
import numpy as np
import pytest

from oracle import fem
from workloads.generate import Problem

GAUSS = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))   # on [0, 1], weights 1/2


def _brute(n, length, a_elem, v):
    nx, ny, nz = n
    h = [length[d] / n[d] for d in range(3)]
    NX, NY, NZ = nx + 1, ny + 1, nz + 1
    N = NX * NY * NZ
    B = np.zeros((N, N)); K = np.zeros((N, N)); A = np.zeros((N, N)); C = np.zeros((N, N))
    a = np.asarray(a_elem).reshape(nz, ny, nx)
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                nodes = []
                for lz in (0, 1):
                    for ly in (0, 1):
                        for lx in (0, 1):
                            nodes.append((lx, ly, lz, (ex + lx) + NX * ((ey + ly) + NY * (ez + lz))))
                for qz in GAUSS:
                    for qy in GAUSS:
                        for qx in GAUSS:
                            w = 0.125 * h[0] * h[1] * h[2]
                            q = (qx, qy, qz)
                            val, grad = {}, {}
                            for (lx, ly, lz, g) in nodes:
                                f = [q[0] if lx else 1 - q[0], q[1] if ly else 1 - q[1], q[2] if lz else 1 - q[2]]
                                df = [(1 if lx else -1) / h[0], (1 if ly else -1) / h[1], (1 if lz else -1) / h[2]]
                                val[g] = f[0] * f[1] * f[2]
                                grad[g] = np.array([df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]])
                            for (_, _, _, j) in nodes:
                                for (_, _, _, i) in nodes:
                                    B[j, i] += w * val[i] * val[j]
                                    K[j, i] += w * grad[i] @ grad[j]
                                    A[j, i] += w * a[ez, ey, ex] * grad[i] @ grad[j]
                                    C[j, i] += w * (np.asarray(v) @ grad[i]) * val[j]
    return B, K, A, C


def _prob(n, length, a, v, faces=0b11):
    return Problem(n=n, M=2, a_elem=a, v=v, beta1=1.0, beta2=1.0,
                   sensor_node=np.array([], dtype=np.int32), data=np.zeros((3, 0)),
                   length=length, dirichlet_faces=faces)


def test_spatial_matrices_match_quadrature():
    n = (2, 3, 2)
    length = (1.0, 1.5, 0.75)
    rng = np.random.default_rng(5)
    a = rng.uniform(0.5, 2.0, size=12)
    v = (0.7, -0.3, 1.1)
    ops = fem.spatial_ops(_prob(n, length, a, v))
    B, K, A, C = _brute(n, length, a, v)
    for name, got, ref in [("B", ops.B, B), ("K", ops.K, K), ("A", ops.A, A), ("N", ops.N, C)]:
        err = np.abs(got.toarray() - ref).max() / np.abs(ref).max()
        assert err < 1e-13, (name, err)


def test_convection_is_not_symmetric():
    """N[j,i] = (v.grad phi_i, phi_j): its transpose is a different matrix."""
    ops = fem.spatial_ops(_prob((3, 3, 3), (1, 1, 1), np.ones(27), (1.0, 0.5, 0.25)))
    assert np.abs((ops.N - ops.N.T).toarray()).max() > 1e-3


def test_time_matrices_match_quadrature():
    M, T = 5, 1.3
    tau = T / M
    Tt = fem.time_mass(M, tau).toarray()
    St = fem.time_stiff(M, tau).toarray()
    Tb = np.zeros((M + 1, M + 1)); Sb = np.zeros((M + 1, M + 1))
    for e in range(M):
        for q in GAUSS:
            w = 0.5 * tau
            phi = {e: 1 - q, e + 1: q}
            dphi = {e: -1 / tau, e + 1: 1 / tau}
            for i in phi:
                for j in phi:
                    Tb[i, j] += w * phi[i] * phi[j]
                    Sb[i, j] += w * dphi[i] * dphi[j]
    assert np.abs(Tt - Tb).max() < 1e-15
    assert np.abs(St - Sb).max() < 1e-13


@pytest.mark.parametrize("n", [(3, 4, 5), (8, 8, 8)])
def test_invariants(n):
    rng = np.random.default_rng(1)
    a = rng.uniform(0.3, 3.0, size=n[0] * n[1] * n[2])
    ops = fem.spatial_ops(_prob(n, (1.0, 1.0, 1.0), a, (1.0, 0.5, 0.25)))
    one = np.ones(ops.B.shape[0])
    assert np.abs(ops.A @ one).max() < 1e-12
    assert np.abs(ops.K @ one).max() < 1e-12
    assert np.abs(ops.N @ one).max() < 1e-14          # div v = 0
    assert abs(one @ ops.B @ one - 1.0) < 1e-13       # |Omega| = 1
    M, T = 7, 1.0
    tau = T / M
    assert np.abs(fem.time_stiff(M, tau) @ np.ones(M + 1)).max() < 1e-12
    assert abs(np.ones(M + 1) @ fem.time_mass(M, tau) @ np.ones(M + 1) - T) < 1e-14
    assert abs(fem.trapezoid_weights(M, tau).sum() - T) < 1e-14


def test_dirichlet_mask_faces():
    m = fem.dirichlet_mask((2, 2, 2), 0b000011)
    g = np.arange(27)
    i = g % 3
    assert np.array_equal(m, (i == 0) | (i == 2))
