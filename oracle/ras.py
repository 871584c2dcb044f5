"""One-level space-time restricted additive Schwarz with 3x3 block ILU(0).

Section 3.2 (one-level preconditioner): the space-time box is split into
N_s spatial subdomains times N_t time intervals, each extended by ``delta``
whole mesh cells in x, y, z and t and trimmed at the global box; the
subdomain matrix is the principal submatrix of F_h on the extended box, and
the preconditioner restricts with overlap, solves approximately, and keeps the
owned (non-overlapping) part -- the restricted additive Schwarz of Cai and
Sarkis:  z = sum_i (R^0_i)^T  Mtilde_i^{-1}  R^delta_i r.
Mtilde_i^{-1} is ILU(k) (Section 4: ILU(k), k = 0 by default, the fill level
studied in the paper's first table) applied to 3x3 point blocks (C, G, f of
one space-time node, Section 3.2 ordering) in the box's natural
lexicographic order.  Level of fill (the usual symbolic rule): entries of the
81-point block pattern have level 0; eliminating row k from row i gives entry
(i, j) the level min(lev(i, j), lev(i, k) + lev(k, j) + 1); ILU(k) keeps the
entries of level <= k and is the incomplete factorisation on that pattern.

Partition rule per dimension with L nodes and p parts: q, r = divmod(L, p);
part k owns [k q + min(k, r), (k+1) q + min(k+1, r)).  Subdomain id =
kx + px (ky + py (kz + pz kt)).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import clib
from . import kkt as kkt_mod


def split(L: int, p: int):
    q, r = divmod(L, p)
    return [k * q + min(k, r) for k in range(p + 1)]


@dataclass
class Subdomain:
    sid: int
    own_lo: tuple   # (x, y, z, t), inclusive
    own_hi: tuple   # exclusive
    box_lo: tuple
    box_hi: tuple

    @property
    def dims(self):
        return tuple(self.box_hi[d] - self.box_lo[d] for d in range(4))

    @property
    def rows(self):
        d = self.dims
        return d[0] * d[1] * d[2] * d[3]


def subdomains(prob, parts, delta):
    nodes = (*prob.nodes, prob.M + 1)
    for d in range(4):
        if parts[d] < 1 or parts[d] > nodes[d]:
            raise ValueError("bad partition")
    cuts = [split(nodes[d], parts[d]) for d in range(4)]
    out = []
    px, py, pz, pt = parts
    for kt in range(pt):
        for kz in range(pz):
            for ky in range(py):
                for kx in range(px):
                    k = (kx, ky, kz, kt)
                    lo = tuple(cuts[d][k[d]] for d in range(4))
                    hi = tuple(cuts[d][k[d] + 1] for d in range(4))
                    blo = tuple(max(0, lo[d] - delta) for d in range(4))
                    bhi = tuple(min(nodes[d], hi[d] + delta) for d in range(4))
                    out.append(Subdomain(kx + px * (ky + py * (kz + pz * kt)), lo, hi, blo, bhi))
    return out


def box_node_ids(prob, sd: Subdomain):
    """Spatial node ids of the box in lexicographic (x fastest) order."""
    nx, ny, _ = prob.nodes
    xs = np.arange(sd.box_lo[0], sd.box_hi[0])
    ys = np.arange(sd.box_lo[1], sd.box_hi[1])
    zs = np.arange(sd.box_lo[2], sd.box_hi[2])
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return (X + nx * (Y + ny * Z)).ravel()


def box_global_index(prob, sd: Subdomain):
    """Global unknown index of every local unknown (level, node, slot order)."""
    nid = box_node_ids(prob, sd)
    ts = np.arange(sd.box_lo[3], sd.box_hi[3])
    g = (ts[:, None] * prob.N + nid[None, :]).ravel()
    return (3 * g[:, None] + np.arange(3)[None, :]).ravel()


def owned_mask(sd: Subdomain):
    """Local rows (block rows) inside the owned sub-box."""
    lx, ly, lz, lt = sd.dims
    T, Z, Y, X = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    c = [X.ravel(), Y.ravel(), Z.ravel(), T.ravel()]
    m = np.ones(c[0].size, dtype=bool)
    for d in range(4):
        g = c[d] + sd.box_lo[d]
        m &= (g >= sd.own_lo[d]) & (g < sd.own_hi[d])
    return m


# offsets in ascending neighbour order: slot s = (dx+1) + 3(dy+1) + 9(dz+1) + 27(dt+1)
OFFSETS = np.array([(dx, dy, dz, dt) for dt in (-1, 0, 1) for dz in (-1, 0, 1)
                    for dy in (-1, 0, 1) for dx in (-1, 0, 1)], dtype=np.int64)
DIAG_SLOT = 40


def block_pattern(dims):
    """Zero-fill ILU pattern: every in-box node pair within +-1 in all four coordinates.

    Returns (indptr, indices, slot) of the block CSR, columns sorted, plus the
    slot number (0..80) of every stored block.
    """
    lx, ly, lz, lt = dims
    n = lx * ly * lz * lt
    T, Z, Y, X = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    X, Y, Z, T = X.ravel(), Y.ravel(), Z.ravel(), T.ravel()
    cols = np.full((n, 81), -1, dtype=np.int64)
    for s, (dx, dy, dz, dt) in enumerate(OFFSETS):
        x, y, z, t = X + dx, Y + dy, Z + dz, T + dt
        ok = (x >= 0) & (x < lx) & (y >= 0) & (y < ly) & (z >= 0) & (z < lz) & (t >= 0) & (t < lt)
        cols[ok, s] = (x + lx * (y + ly * (z + lz * t)))[ok]
    valid = cols >= 0
    counts = valid.sum(axis=1)
    indptr = np.zeros(n + 1, dtype=np.int64)
    indptr[1:] = np.cumsum(counts)
    indices = cols[valid]
    slots = np.broadcast_to(np.arange(81), cols.shape)[valid]
    return indptr, indices, slots


_PATTERN_CACHE = {}


def ilu_pattern(dims, level):
    """Block pattern of ILU(level) on a box: (indptr, indices, lev) in block
    CSR form, columns sorted, lev the fill level of every entry.

    Symbolic elimination in the IKJ order (``oracle_iluk_symbolic`` in
    bilu.c): for every row i, the columns k < i of its current pattern are
    taken in ascending order (fill entries with k < i join as they appear),
    and every entry (k, j), j > k, of the already computed row k offers (i, j)
    the level lev(i, k) + lev(k, j) + 1; an entry is kept when its smallest
    offered level is <= level."""
    key = (tuple(int(d) for d in dims), int(level))
    if key in _PATTERN_CACHE:
        return _PATTERN_CACHE[key]
    indptr0, indices0, _ = block_pattern(dims)
    n = indptr0.size - 1
    ip0 = np.ascontiguousarray(indptr0, dtype=np.int32)
    ix0 = np.ascontiguousarray(indices0, dtype=np.int32)
    cap = max(4 * ix0.size, 1024)
    while True:
        indptr = np.zeros(n + 1, dtype=np.int64)
        indices = np.zeros(cap, dtype=np.int32)
        levs = np.zeros(cap, dtype=np.int32)
        nnz = clib.lib().oracle_iluk_symbolic(n, clib.ptr(ip0), clib.ptr(ix0), int(level), cap, clib.ptr(indptr),
                                              clib.ptr(indices), clib.ptr(levs))
        if nnz >= 0:
            break
        if cap > 64 * n * n:
            raise MemoryError("ilu_pattern")
        cap *= 2
    out = (indptr, indices[:nnz].astype(np.int64), levs[:nnz].astype(np.int64))
    _PATTERN_CACHE[key] = out
    return out


def block_values(A_box: sp.csr_matrix, indptr, indices):
    """Values of every pattern block (explicit zeros where F_h has none)."""
    nb = indptr.size - 1
    Ab = A_box.tobsr(blocksize=(3, 3))
    Ab.sort_indices()
    rows_b = np.repeat(np.arange(nb), np.diff(Ab.indptr))
    key_src = rows_b * nb + Ab.indices
    rows_p = np.repeat(np.arange(nb), np.diff(indptr))
    key_dst = rows_p * nb + indices
    pos = np.searchsorted(key_dst, key_src)
    if np.any(pos >= key_dst.size) or np.any(key_dst[np.minimum(pos, key_dst.size - 1)] != key_src):
        raise AssertionError("F_h has a block outside the 81-point space-time pattern")
    vals = np.zeros((key_dst.size, 3, 3))
    vals[pos] = Ab.data
    return vals


class SubdomainILU:
    """ILU(level) factors of one subdomain matrix (block CSR, IKJ order)."""

    def __init__(self, A_box: sp.csr_matrix, dims, level=0):
        self.dims = dims
        self.level = level
        if level == 0:
            indptr, indices, slots = block_pattern(dims)
            self.slots = slots
        else:
            indptr, indices, _ = ilu_pattern(dims, level)
            self.slots = None
        self.indptr = indptr.astype(np.int32)
        self.indices = indices.astype(np.int32)
        self.diagpos = (self.indptr[:-1] + np.array(
            [np.searchsorted(indices[indptr[i]:indptr[i + 1]], i) for i in range(indptr.size - 1)])).astype(np.int32)
        self.original = block_values(A_box, indptr, indices)
        self.vals = np.ascontiguousarray(self.original.copy())
        nrows = indptr.size - 1
        self.dinv = np.zeros((nrows, 3, 3))
        L = clib.lib()
        rc = L.oracle_bilu0(nrows, clib.ptr(self.indptr), clib.ptr(self.indices), clib.ptr(self.diagpos),
                            clib.ptr(self.vals), clib.ptr(self.dinv))
        if rc != 0:
            raise FloatingPointError(f"singular pivot block at local row {rc - 1}")

    def solve(self, r: np.ndarray) -> np.ndarray:
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty_like(r)
        clib.lib().oracle_bilu0_solve(self.indptr.size - 1, clib.ptr(self.indptr), clib.ptr(self.indices),
                                      clib.ptr(self.diagpos), clib.ptr(self.vals), clib.ptr(self.dinv),
                                      clib.ptr(r), clib.ptr(z))
        return z

    def csr(self):
        """(indptr, indices, blocks[nnz, 3, 3]): L blocks left of the diagonal,
        inv(U_ii) on it, U blocks right of it."""
        out = self.vals.copy()
        out[self.diagpos] = self.dinv
        return self.indptr.copy(), self.indices.copy(), out

    def padded(self) -> np.ndarray:
        """[rows, 81, 3, 3]: L blocks (slots < 40), inv(U_ii) (slot 40), U blocks (slots > 40)."""
        nrows = self.indptr.size - 1
        out = np.zeros((nrows, 81, 3, 3))
        rows = np.repeat(np.arange(nrows), np.diff(self.indptr))
        out[rows, self.slots] = self.vals
        out[:, DIAG_SLOT] = self.dinv
        return out

    def pattern_mask(self) -> np.ndarray:
        nrows = self.indptr.size - 1
        m = np.zeros((nrows, 81), dtype=bool)
        rows = np.repeat(np.arange(nrows), np.diff(self.indptr))
        m[rows, self.slots] = True
        return m


class RAS:
    """z = sum_i (R^0_i)^T ILU(k)_i^{-1} R^delta_i r."""

    def __init__(self, prob, parts, overlap, terms=None, subset=None, ilu_level=0):
        self.prob = prob
        self.terms = terms if terms is not None else kkt_mod.kkt_terms(prob)
        self.subs = subdomains(prob, parts, overlap)
        ids = range(len(self.subs)) if subset is None else subset
        self.ilu = {}
        self.gidx = {}
        self.own = {}
        for sid in ids:
            sd = self.subs[sid]
            nid = box_node_ids(prob, sd)
            A_box = kkt_mod.box_submatrix(self.terms, nid, sd.box_lo[3], sd.box_hi[3])
            self.ilu[sid] = SubdomainILU(A_box, sd.dims, ilu_level)
            self.gidx[sid] = box_global_index(prob, sd)
            self.own[sid] = np.repeat(owned_mask(sd), 3)

    def solve_sub(self, sid, r):
        return self.ilu[sid].solve(r[self.gidx[sid]])

    def apply(self, r):
        if len(self.ilu) != len(self.subs):
            raise RuntimeError("apply needs every subdomain factored")
        z = np.zeros_like(r)
        for sid in self.ilu:
            zl = self.solve_sub(sid, r)
            m = self.own[sid]
            z[self.gidx[sid][m]] = zl[m]
        return z
