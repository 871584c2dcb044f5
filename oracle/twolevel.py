"""Two-level space-time preconditioner (Section 3.2, two-level paragraph).

Nested coarse mesh: every coarse space-time node is a fine node; the
coarsening factors (fx, fy, fz, ft) divide the element counts and M.
Interpolation I_c^h is linear on the coarse mesh, per unknown slot, i.e. a
tensor product of 1-D linear interpolations in x, y, z and t; restriction is
its transpose I_h^c = (I_c^h)^T (or plain injection as an option).
The coarse operator F_c is the same KKT system rediscretised on the coarse
mesh (coarse element coefficient = mean of the fine element coefficients it
contains; sensor matrix S_c = P_x^T S P_x, which is the coarse 0/1 diagonal
when every sensor sits on a coarse node -- required here).
F_c^{-1} is applied either exactly, by a block LU in time (S_0 = D_0,
S_k = D_k - L_k S_{k-1}^{-1} U_{k-1} with dense partial-pivoting LU of S_k),
or as in the paper's experiments (Section 4): restarted GMRES from a zero
guess with a loose tolerance and a few steps, right-preconditioned by the
one-level space-time RAS of the coarse mesh.
Multiplicative combination:
    y = I_c^h F_c^{-1} I_h^c x,    M^{-1} x = y + M_one^{-1} (x - F_h y).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import kkt as kkt_mod
from . import krylov
from . import ras as ras_mod


def interp_1d(nc: int, f: int) -> sp.csr_matrix:
    """(nc f + 1) x (nc + 1) linear interpolation, fine node i = f I + r."""
    nf = nc * f
    rows, cols, vals = [], [], []
    for i in range(nf + 1):
        I, r = divmod(i, f)
        if r == 0:
            rows.append(i); cols.append(I); vals.append(1.0)
        else:
            rows += [i, i]
            cols += [I, I + 1]
            vals += [1.0 - r / f, r / f]
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf + 1, nc + 1))


def injection_1d(nc: int, f: int) -> sp.csr_matrix:
    """Coarse value = fine value at the same node."""
    nf = nc * f
    return sp.csr_matrix((np.ones(nc + 1), (np.arange(nc + 1) * f, np.arange(nc + 1))), shape=(nf + 1, nc + 1))


def prolongation(prob, factors, kind=interp_1d) -> sp.csr_matrix:
    fx, fy, fz, ft = factors
    nx, ny, nz = prob.n
    Px = kind(nx // fx, fx)
    Py = kind(ny // fy, fy)
    Pz = kind(nz // fz, fz)
    Pt = kind(prob.M // ft, ft)
    P = sp.kron(Pt, sp.kron(Pz, sp.kron(Py, sp.kron(Px, sp.identity(3)))))
    return P.tocsr()


def coarse_problem(prob, factors):
    fx, fy, fz, ft = factors
    nx, ny, nz = prob.n
    if nx % fx or ny % fy or nz % fz or prob.M % ft:
        raise ValueError("coarsening factors must divide the mesh")
    ncx, ncy, ncz = nx // fx, ny // fy, nz // fz
    a = np.asarray(prob.a_elem).reshape(nz, ny, nx)
    ac = a.reshape(ncz, fz, ncy, fy, ncx, fx).mean(axis=(1, 3, 5)).ravel()
    NX, NY = nx + 1, ny + 1
    sn = np.asarray(prob.sensor_node)
    i, j, k = sn % NX, (sn // NX) % NY, sn // (NX * NY)
    if np.any(i % fx) or np.any(j % fy) or np.any(k % fz):
        raise ValueError("two-level setup needs every sensor on a coarse node")
    cs = (i // fx + (ncx + 1) * (j // fy + (ncy + 1) * (k // fz))).astype(np.int32)
    return dataclasses.replace(prob, n=(ncx, ncy, ncz), M=prob.M // ft, a_elem=ac, sensor_node=cs,
                               data=np.zeros((prob.M // ft + 1, cs.size)), f_true=None,
                               name=prob.name + "_coarse")


class BlockTridiagLU:
    """Exact F_c^{-1} via block LU over time levels (blocks of 3 N_c unknowns)."""

    def __init__(self, F: sp.csr_matrix, nlev: int):
        n = F.shape[0] // nlev
        self.n, self.nlev = n, nlev
        F = F.tocsr()
        blk = lambda a, b: F[a * n:(a + 1) * n, b * n:(b + 1) * n]
        self.L = [None] + [blk(k, k - 1) for k in range(1, nlev)]
        self.U = [blk(k, k + 1) for k in range(nlev - 1)] + [None]
        self.lu = []
        Sk = blk(0, 0).toarray()
        for k in range(nlev):
            if k > 0:
                Sk = blk(k, k).toarray() - self.L[k] @ sla.lu_solve(self.lu[k - 1], self.U[k - 1].toarray())
            self.lu.append(sla.lu_factor(Sk))

    def solve(self, r):
        n, nl = self.n, self.nlev
        R = r.reshape(nl, n)
        y = np.zeros((nl, n))
        for k in range(nl):
            rhs = R[k] - (self.L[k] @ y[k - 1] if k > 0 else 0.0)
            y[k] = sla.lu_solve(self.lu[k], rhs)
        x = np.zeros((nl, n))
        x[nl - 1] = y[nl - 1]
        for k in range(nl - 2, -1, -1):
            x[k] = y[k] - sla.lu_solve(self.lu[k], self.U[k] @ x[k + 1])
        return x.ravel()


class CoarseGmresRas:
    """F_c^{-1} r ~ GMRES(maxit) from zero, rtol, right-preconditioned by coarse RAS."""

    def __init__(self, cprob, Fc, parts, overlap, maxit=4, rtol=0.1):
        self.Fc = Fc
        self.R = ras_mod.RAS(cprob, parts, overlap)
        self.maxit = maxit
        self.rtol = rtol

    def solve(self, r):
        x, _ = krylov.gmres(lambda v: self.Fc @ v, self.R.apply, r, restart=self.maxit, rtol=self.rtol,
                            maxit=self.maxit)
        return x


class TwoLevel:
    """M^{-1} x = y + M_one^{-1}(x - F_h y),  y = P F_c^{-1} R x."""

    def __init__(self, prob, one_level, F_apply, factors, restrict="transpose", coarse="lu",
                 coarse_parts=None, coarse_overlap=1, coarse_maxit=4, coarse_rtol=0.1):
        self.P = prolongation(prob, factors)
        if restrict == "transpose":
            self.R = self.P.T.tocsr()
        elif restrict == "injection":
            self.R = prolongation(prob, factors, injection_1d).T.tocsr()
        else:
            raise ValueError(restrict)
        self.cprob = coarse_problem(prob, factors)
        self.Fc = kkt_mod.assemble(self.cprob)
        if coarse == "lu":
            self.coarse = BlockTridiagLU(self.Fc, self.cprob.M + 1)
        elif coarse == "gmres_ras":
            self.coarse = CoarseGmresRas(self.cprob, self.Fc, coarse_parts, coarse_overlap, coarse_maxit,
                                         coarse_rtol)
        else:
            raise ValueError(coarse)
        self.one = one_level
        self.F = F_apply

    def coarse_correction(self, x):
        return self.P @ self.coarse.solve(self.R @ x)

    def __call__(self, x):
        y = self.coarse_correction(x)
        return y + self.one(x - self.F(y))
