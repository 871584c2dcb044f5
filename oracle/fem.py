"""Finite-element and time matrices of the space-time discretisation.

Space: uniform hexahedral mesh, trilinear (Q1) nodal basis phi_j, exact
integration, coefficient a constant per element.  Time: uniform partition
t^n = n*tau of [0, T] with piecewise-linear hat functions theta_n.

Definitions followed (Appendix A):
  A[j,i] = (a grad phi_i, grad phi_j)        stiffness with coefficient a
  B[j,i] = (phi_i, phi_j)                     mass
  K[j,i] = (grad phi_i, grad phi_j)           unit-coefficient stiffness
  N[j,i] = (v . grad phi_i, phi_j)            convection, row = test function
  time mass  Tt[n,m] = (theta_m, theta_n),  time stiffness St[n,m] = (theta_m', theta_n')
so that the space-time matrices of Appendix A are D^{nm} = Tt[n,m] B,
L^{nm} = St[n,m] B and K^{nm} = Tt[n,m] K.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


def mass_1d(ne: int, h: float) -> sp.csr_matrix:
    """Assembled 1-D P1 mass matrix on ne elements of length h."""
    Me = h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
    return _assemble_1d(ne, Me)


def stiff_1d(ne: int, h: float) -> sp.csr_matrix:
    """Assembled 1-D P1 stiffness matrix."""
    Ke = 1.0 / h * np.array([[1.0, -1.0], [-1.0, 1.0]])
    return _assemble_1d(ne, Ke)


def conv_1d(ne: int) -> sp.csr_matrix:
    """Assembled D[j,i] = int phi_j phi_i' (row = test, column = trial)."""
    De = 0.5 * np.array([[-1.0, 1.0], [-1.0, 1.0]])
    return _assemble_1d(ne, De)


def _assemble_1d(ne, Ee):
    rows, cols, vals = [], [], []
    for e in range(ne):
        for a in range(2):
            for b in range(2):
                rows.append(e + a)
                cols.append(e + b)
                vals.append(Ee[a, b])
    return sp.csr_matrix((vals, (rows, cols)), shape=(ne + 1, ne + 1))


def time_mass(M: int, tau: float) -> sp.csr_matrix:
    return mass_1d(M, tau)


def time_stiff(M: int, tau: float) -> sp.csr_matrix:
    return stiff_1d(M, tau)


def trapezoid_weights(M: int, tau: float) -> np.ndarray:
    """Lumped time mass (trapezoid rule) used for the discrete misfit."""
    w = np.full(M + 1, tau)
    w[0] = w[-1] = 0.5 * tau
    return w


def kron3(Z, Y, X):
    """Kronecker product with the x index fastest (node g = i + nx*(j + ny*k))."""
    return sp.kron(Z, sp.kron(Y, X, format="csr"), format="csr")


def stiffness_variable(n, h, a_elem) -> sp.csr_matrix:
    """A[j,i] = sum_e a_e int_e grad phi_i . grad phi_j on the Q1 hex mesh."""
    nx, ny, nz = n
    Me = [h[d] / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]]) for d in range(3)]
    Ke = [1.0 / h[d] * np.array([[1.0, -1.0], [-1.0, 1.0]]) for d in range(3)]
    # 8x8 element stiffness, local node l = lx + 2 ly + 4 lz
    Kel = (np.kron(Me[2], np.kron(Me[1], Ke[0])) + np.kron(Me[2], np.kron(Ke[1], Me[0]))
           + np.kron(Ke[2], np.kron(Me[1], Me[0])))
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    NX, NY = nx + 1, ny + 1
    loc = []
    for l in range(8):
        lx, ly, lz = l & 1, (l >> 1) & 1, (l >> 2) & 1
        loc.append((ex + lx) + NX * ((ey + ly) + NY * (ez + lz)))
    loc = np.stack(loc, axis=1)              # [nelem, 8]
    a = np.asarray(a_elem, dtype=np.float64).ravel()
    rows = np.repeat(loc, 8, axis=1).ravel()
    cols = np.tile(loc, (1, 8)).ravel()
    vals = (a[:, None] * Kel.ravel()[None, :]).ravel()
    N = NX * NY * (nz + 1)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


@dataclass
class SpatialOps:
    B: sp.csr_matrix
    K: sp.csr_matrix
    A: sp.csr_matrix
    N: sp.csr_matrix
    interior: np.ndarray      # bool[N], True off the Dirichlet faces
    sensor: np.ndarray        # float64[N], 1 at sensor nodes


def dirichlet_mask(n, faces) -> np.ndarray:
    nx, ny, nz = (k + 1 for k in n)
    g = np.arange(nx * ny * nz)
    i, j, k = g % nx, (g // nx) % ny, g // (nx * ny)
    m = np.zeros(g.size, dtype=bool)
    for bit, (arr, val) in enumerate([(i, 0), (i, nx - 1), (j, 0), (j, ny - 1), (k, 0), (k, nz - 1)]):
        if faces >> bit & 1:
            m |= arr == val
    return m


def spatial_ops(prob) -> SpatialOps:
    n = prob.n
    h = [prob.length[d] / n[d] for d in range(3)]
    M1 = [mass_1d(n[d], h[d]) for d in range(3)]
    K1 = [stiff_1d(n[d], h[d]) for d in range(3)]
    D1 = [conv_1d(n[d]) for d in range(3)]
    B = kron3(M1[2], M1[1], M1[0])
    K = kron3(M1[2], M1[1], K1[0]) + kron3(M1[2], K1[1], M1[0]) + kron3(K1[2], M1[1], M1[0])
    vx, vy, vz = prob.v
    Nc = (vx * kron3(M1[2], M1[1], D1[0]) + vy * kron3(M1[2], D1[1], M1[0])
          + vz * kron3(D1[2], M1[1], M1[0]))
    A = stiffness_variable(n, h, prob.a_elem)
    interior = ~dirichlet_mask(n, prob.dirichlet_faces)
    sensor = np.zeros(B.shape[0])
    sensor[np.asarray(prob.sensor_node)] = 1.0
    return SpatialOps(B=B.tocsr(), K=K.tocsr(), A=A, N=Nc.tocsr(), interior=interior, sensor=sensor)
