"""Pins of the oracle's partition, ILU(0) and restricted additive Schwarz."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import kkt, ras, krylov
from workloads.generate import make_custom


def test_split_closed_form():
    assert ras.split(33, 4) == [0, 9, 17, 25, 33]
    assert ras.split(65, 8) == [0, 9, 17, 25, 33, 41, 49, 57, 65]
    assert ras.split(9, 2) == [0, 5, 9]


def test_cube32x64_boxes():
    """32^3 x 64 with 4x4x4x8 parts and overlap 2: boxes of at most 12^4 nodes."""
    class P:  # only sizes matter
        nodes = (33, 33, 33)
        M = 64
    subs = ras.subdomains(P, (4, 4, 4, 8), 2)
    assert len(subs) == 512
    xs = sorted({s.dims[0] for s in subs})
    assert xs == [10, 11, 12]
    assert max(s.rows for s in subs) == 12 ** 4
    # total block count of all box patterns: sum of prod_d (3 l_d - 2)
    tot = sum(int(np.prod([3 * l - 2 for l in s.dims])) for s in subs)
    assert tot == 538_724_729


def test_block_pattern_count_and_order():
    for dims in [(6, 6, 6, 10), (1, 3, 2, 4), (2, 1, 1, 1)]:
        indptr, indices, slots = ras.block_pattern(dims)
        assert indptr[-1] == np.prod([3 * l - 2 for l in dims])
        for i in range(indptr.size - 1):
            row = indices[indptr[i]:indptr[i + 1]]
            assert np.all(np.diff(row) > 0)
            assert np.all(np.diff(slots[indptr[i]:indptr[i + 1]]) > 0)
    # whole cube8x16 space-time box (9^3 nodes, 17 levels)
    indptr, _, _ = ras.block_pattern((9, 9, 9, 17))
    assert indptr[-1] == 25 ** 3 * 49 == 765_625


def test_owned_sets_partition_unknowns():
    prob = make_custom((4, 5, 3), 6, 1, lattice=2)
    for parts, delta in [((2, 2, 1, 3), 1), ((3, 1, 2, 2), 2), ((1, 1, 1, 1), 0)]:
        cover = np.zeros(prob.unknowns, dtype=int)
        for sd in ras.subdomains(prob, parts, delta):
            gi = ras.box_global_index(prob, sd)
            cover[gi[np.repeat(ras.owned_mask(sd), 3)]] += 1
        assert np.all(cover == 1)


def _reconstruct(ilu):
    """Dense L (unit lower) and U from the block factors."""
    n = ilu.indptr.size - 1
    Ld = np.eye(3 * n)
    Ud = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for p in range(ilu.indptr[i], ilu.indptr[i + 1]):
            j = ilu.indices[p]
            blk = ilu.vals[p]
            if j < i:
                Ld[3 * i:3 * i + 3, 3 * j:3 * j + 3] = blk
            else:
                Ud[3 * i:3 * i + 3, 3 * j:3 * j + 3] = blk
    return Ld, Ud


def test_bilu0_defining_property():
    """(L U)_ij = A_ij on every pattern block, and inv(U_ii) is the inverse."""
    prob = make_custom((3, 3, 3), 4, 2, lattice=2)
    terms = kkt.kkt_terms(prob)
    sd = ras.Subdomain(0, (0, 0, 0, 0), (3, 3, 3, 4), (0, 0, 0, 0), (3, 3, 3, 4))
    A = kkt.box_submatrix(terms, ras.box_node_ids(prob, sd), 0, 4)
    ilu = ras.SubdomainILU(A, sd.dims)
    Ld, Ud = _reconstruct(ilu)
    LU = Ld @ Ud
    Ad = A.toarray()
    n = ilu.indptr.size - 1
    scale = np.abs(Ad).max()
    for i in range(n):
        for p in range(ilu.indptr[i], ilu.indptr[i + 1]):
            j = ilu.indices[p]
            d = LU[3 * i:3 * i + 3, 3 * j:3 * j + 3] - Ad[3 * i:3 * i + 3, 3 * j:3 * j + 3]
            assert np.abs(d).max() <= 1e-13 * scale
        np.testing.assert_allclose(ilu.dinv[i] @ Ud[3 * i:3 * i + 3, 3 * i:3 * i + 3], np.eye(3), atol=1e-12)
    # the factorisation is incomplete: LU differs from A off the pattern
    assert np.abs(LU - Ad).max() > 1e-8 * scale


def test_bilu0_exact_on_chain():
    """A box that is one node wide in three dimensions is a block chain: ILU(0) = LU."""
    prob = make_custom((3, 3, 3), 8, 3, lattice=2)
    terms = kkt.kkt_terms(prob)
    sd = ras.Subdomain(0, (1, 1, 1, 0), (2, 2, 2, 9), (1, 1, 1, 0), (2, 2, 2, 9))
    A = kkt.box_submatrix(terms, ras.box_node_ids(prob, sd), 0, 9)
    ilu = ras.SubdomainILU(A, sd.dims)
    r = np.random.default_rng(0).standard_normal(A.shape[0])
    z = ilu.solve(r)
    np.testing.assert_allclose(A @ z, r, rtol=0, atol=1e-10 * np.abs(r).max())


def test_ras_zero_overlap_is_block_jacobi():
    prob = make_custom((4, 3, 3), 5, 4, lattice=2)
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    R = ras.RAS(prob, (2, 1, 2, 2), 0, terms=terms)
    r = np.random.default_rng(1).standard_normal(F.shape[0])
    z = R.apply(r)
    for sid, sd in enumerate(R.subs):
        gi = R.gidx[sid]
        ilu = ras.SubdomainILU(F[gi][:, gi], sd.dims)
        np.testing.assert_allclose(z[gi], ilu.solve(r[gi]), rtol=1e-13, atol=1e-13)


def test_ras_single_chain_subdomain_one_iteration():
    """2x2x2 spatial nodes: every spatial pair is a stencil neighbour, so the ILU(0)
    pattern already holds all the fill of block-tridiagonal-in-time LU; one subdomain
    then gives M^{-1} = F^{-1} and GMRES takes one step."""
    prob = make_custom((1, 1, 1), 12, 6, lattice=1, faces=0, sensors=np.array([0]))
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    b = kkt.rhs(prob)
    R = ras.RAS(prob, (1, 1, 1, 1), 0, terms=terms)
    x, st = krylov.gmres(lambda v: F @ v, R.apply, b, restart=10, rtol=1e-10)
    assert st.iters == 1 and st.converged


def test_overlap_reduces_iterations():
    """Paper Table 2 trend: larger overlap, fewer Krylov iterations."""
    prob = make_custom((8, 8, 8), 12, 3, lattice=3)
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    b = kkt.rhs(prob)
    its = []
    for delta in (0, 1, 2):
        R = ras.RAS(prob, (2, 2, 2, 2), delta, terms=terms)
        _, st = krylov.gmres(lambda v: F @ v, R.apply, b, restart=50, rtol=1e-6)
        assert st.converged
        its.append(st.iters)
    assert its[0] > its[1] >= its[2]


def _fill_path_levels(dims):
    """Brute force: the level of fill of entry (i, j) is the length of the
    shortest path from i to j in the graph of the 81-point block pattern whose
    interior vertices are all numbered below min(i, j), minus one (the graph
    model of level-based ILU of Hysom and Pothen); absent if no such path."""
    from collections import deque
    indptr, indices, _ = ras.block_pattern(dims)
    n = indptr.size - 1
    nbr = [[int(j) for j in indices[indptr[i]:indptr[i + 1]] if j != i] for i in range(n)]
    lev = {}
    for i in range(n):
        for j in range(n):
            if i == j:
                lev[(i, j)] = 0
                continue
            lo = min(i, j)
            dist = {i: 0}
            q = deque([i])
            while q:
                u = q.popleft()
                if u == j:
                    break
                for w in nbr[u]:
                    if w not in dist and (w < lo or w == j):
                        dist[w] = dist[u] + 1
                        q.append(w)
            if j in dist:
                lev[(i, j)] = dist[j] - 1
    return lev


@pytest.mark.parametrize("dims", [(3, 3, 2, 2), (2, 3, 3, 2)])
def test_iluk_pattern_matches_fill_paths(dims):
    """ILU(k) keeps exactly the entries whose shortest fill path has at most k
    interior vertices, with the level the path gives."""
    want = _fill_path_levels(dims)
    for k in range(4):
        indptr, indices, levs = ras.ilu_pattern(dims, k)
        got = {(i, int(indices[p])): int(levs[p]) for i in range(indptr.size - 1)
               for p in range(indptr[i], indptr[i + 1])}
        assert got == {key: l for key, l in want.items() if l <= k}, k
    assert np.array_equal(ras.ilu_pattern(dims, 0)[1], ras.block_pattern(dims)[1])


@pytest.mark.parametrize("level", [1, 2])
def test_iluk_product_matches_matrix_on_pattern(level):
    """ILU on the level-k pattern: (L U)_ij = A_ij for every (i, j) of the pattern."""
    prob = make_custom((6, 6, 6), 5, 13, lattice=2)
    terms = kkt.kkt_terms(prob)
    sd = ras.Subdomain(0, (1, 1, 1, 1), (6, 5, 5, 5), (1, 1, 1, 1), (6, 5, 5, 5))
    A = kkt.box_submatrix(terms, ras.box_node_ids(prob, sd), 1, 5).toarray()
    ilu = ras.SubdomainILU(sp.csr_matrix(A), sd.dims, level)
    n = ilu.indptr.size - 1
    L = np.eye(3 * n)
    U = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for p in range(ilu.indptr[i], ilu.indptr[i + 1]):
            j = ilu.indices[p]
            blk = ilu.vals[p]
            if j < i:
                L[3 * i:3 * i + 3, 3 * j:3 * j + 3] = blk
            else:
                U[3 * i:3 * i + 3, 3 * j:3 * j + 3] = blk
    LU = L @ U
    mask = np.zeros((3 * n, 3 * n), dtype=bool)
    for i in range(n):
        for j in ilu.indices[ilu.indptr[i]:ilu.indptr[i + 1]]:
            mask[3 * i:3 * i + 3, 3 * j:3 * j + 3] = True
    assert np.abs(LU - A)[mask].max() <= 1e-12 * np.abs(A).max()
    # and the pattern holds fill: the product differs from A somewhere off it
    assert np.abs(LU - A)[~mask].max() > 1e-8 * np.abs(A).max()
    assert mask.sum() > 9 * ras.block_pattern(sd.dims)[1].size


def test_iluk_becomes_exact_lu():
    """With a level above the box's row count every fill entry is kept:
    ILU(k) is the exact block LU and its solve is A^{-1}."""
    prob = make_custom((5, 5, 5), 5, 17, lattice=1)
    terms = kkt.kkt_terms(prob)
    sd = ras.Subdomain(0, (1, 1, 1, 1), (5, 4, 4, 4), (1, 1, 1, 1), (5, 4, 4, 4))
    A = kkt.box_submatrix(terms, ras.box_node_ids(prob, sd), 1, 4)
    nrows = int(np.prod(sd.dims))
    r = np.random.default_rng(4).standard_normal(A.shape[0])
    exact = np.linalg.solve(A.toarray(), r)
    errs = []
    for k in (0, 1, nrows):
        z = ras.SubdomainILU(A, sd.dims, k).solve(r)
        errs.append(np.linalg.norm(z - exact) / np.linalg.norm(exact))
    assert errs[-1] <= 1e-10
    assert errs[0] > errs[1] > errs[-1]


def test_iluk_reduces_iterations():
    """Paper's fill-level table trend: more fill, fewer Krylov iterations."""
    prob = make_custom((6, 6, 6), 8, 3, lattice=2)
    terms = kkt.kkt_terms(prob)
    F = kkt.assemble(prob, terms=terms)
    b = kkt.rhs(prob)
    its = []
    for k in (0, 1, 2):
        R = ras.RAS(prob, (2, 2, 2, 2), 1, terms=terms, ilu_level=k)
        _, st = krylov.gmres(lambda v: F @ v, R.apply, b, restart=50, rtol=1e-6)
        assert st.converged
        its.append(st.iters)
    assert its[0] > its[1] >= its[2], its
