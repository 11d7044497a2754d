"""Pins of the oracle's in-block pivoting (Bunch-Kaufman, the sytrf of the
paper's dense factorization task, restricted to segments of an interface)
against facts outside the oracle: LAPACK's complex symmetric sytrf through
scipy.linalg.ldl on a single block (same pivot rule, so the same pivots,
L and D), the reconstruction of the permuted K from the factor, dense
Gaussian elimination for the solve, and the no-pivot oracle where no
interchange is needed."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from paper_2002_05026_amd import instances as gen
from tests import dense_ref


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def _single_block(n, seed, shift=0.0):
    rng = np.random.default_rng(seed)
    M = _cn(rng, (n, n))
    A = np.tril(M) + np.tril(M, -1).T + shift * np.eye(n)
    K = A.reshape(-1, order="F").copy()
    return A, K


def full_factor(p, sizes, order, tile):
    """The factor in fully permuted form: the global permutation q (internal
    row -> user row) and L, D with K[q][:, q] = L D L^T.  Rows of a segment
    stored in columns left of it are in original order (the product form),
    so they are permuted here by the segment's interchanges."""
    sizes = np.asarray(sizes, dtype=np.int64)
    row0 = np.concatenate([[0], np.cumsum(sizes)])
    start, q = {}, []
    o = 0
    perms = {}
    for I in order:
        I = int(I)
        start[I] = o
        perm, doff = p.pivots(I)
        perms[I] = (perm, doff)
        q += list(row0[I] + perm)
        o += int(sizes[I])
    N = o
    L = np.zeros((N, N), dtype=np.complex128)
    D = np.zeros((N, N), dtype=np.complex128)
    for I in order:
        I = int(I)
        nI, s = int(sizes[I]), start[I]
        perm, doff = perms[I]
        blk = p.block(I, I)
        # segment id of each row; inside a segment rows are internal already
        seg = np.arange(nI) // tile
        inv = np.empty(nI, dtype=np.int64)
        inv[perm] = np.arange(nI)             # original index -> internal position
        for c in range(nI):
            for r in range(c + 1, nI):
                if r == c + 1 and doff[c] != 0:
                    continue
                ri = r if seg[r] == seg[c] else inv[r]   # stored by original index -> internal
                L[s + ri, s + c] = blk[r, c]
        L[s:s + nI, s:s + nI] += np.eye(nI)
        D[s:s + nI, s:s + nI] = np.diag(np.diag(blk))
        for k in range(nI - 1):
            if doff[k] != 0:
                D[s + k + 1, s + k] = D[s + k, s + k + 1] = doff[k]
        for J in p.struct(I):
            nJ, sJ = int(sizes[J]), start[J]
            permJ, _ = p.pivots(J)
            LJ = p.block(J, I)                # rows in J's original order
            L[sJ:sJ + nJ, s:s + nI] = LJ[permJ, :]
    return np.asarray(q), L, D


@pytest.mark.parametrize("n,seed", [(60, 1), (97, 2), (128, 3)])
def test_single_block_matches_lapack_sytrf(n, seed):
    # one interface of n <= 128 unknowns, not diagonally dominant: the oracle's
    # pivots, L and D equal LAPACK's (zsytrf via scipy.linalg.ldl)
    A, K = _single_block(n, seed)
    p = oracle.OraclePlan([n], np.zeros((0, 2), dtype=np.int32), [0])
    assert p.factor_bk(K, tile=128) == -1
    perm, doff = p.pivots(0)
    lu, d, sperm = sl.ldl(A, lower=True, hermitian=False)
    assert np.array_equal(perm, sperm)
    blk = p.block(0, 0)
    Lo = np.tril(blk, -1)
    for k in range(n - 1):
        if doff[k] != 0:
            Lo[k + 1, k] = 0
    Lo += np.eye(n)
    assert np.abs(Lo - lu[sperm]).max() <= 1e-12 * max(1.0, np.abs(lu).max())
    Dn = np.diag(np.diag(blk)) + np.diag(doff[:-1], -1) + np.diag(doff[:-1], 1)
    assert np.abs(Dn - d).max() <= 1e-12 * np.abs(d).max()
    assert np.count_nonzero(doff) >= 1  # the case exercises 2x2 pivots


@pytest.mark.parametrize("grid,lo,hi,tile", [((2, 2, 1), 20, 40, 16), ((2, 2, 2), 10, 30, 8),
                                             ((3, 3, 2), 4, 12, 128)])
def test_pivoted_factor_reconstructs_and_solves(grid, lo, hi, tile):
    # no diagonal shift: diagonal blocks are plain complex symmetric normal
    # matrices, which need interchanges; several segments per interface
    inst = gen.make_instance(grid, (lo, hi), 0.0, 3, 4100 + lo)
    order = oracle.nd_order(inst.grid)
    p = oracle.OraclePlan(inst.sizes, inst.pairs, order)
    assert p.factor_bk(inst.K, tile=tile) == -1
    q, L, D = full_factor(p, inst.sizes, order, tile)
    A = dense_ref.dense_K(inst.sizes, inst.pairs, inst.K)
    PAP = A[np.ix_(q, q)]
    assert np.linalg.norm(PAP - L @ D @ L.T) <= 1e-13 * np.linalg.norm(A) * max(1.0, np.abs(L).max())
    X = p.solve(inst.B)
    Xd = np.linalg.solve(A, inst.B.T).T
    assert (np.linalg.norm(X - Xd, axis=1) / np.linalg.norm(Xd, axis=1)).max() <= 1e-11
    assert oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, inst.B).max() <= 1e-14
    assert sum(np.count_nonzero(p.pivots(I)[1]) for I in range(inst.nb)) > 0


def test_pivoting_where_the_plain_factor_fails():
    # zero diagonal blocks: every first pivot of the no-pivot factorization
    # is zero, the pivoted one takes 2x2 pivots and solves
    inst = gen.make_instance((2, 2, 1), 12, 0.0, 2, 77)
    for i in range(inst.nb):
        inst.K[inst.offsets[i]:inst.offsets[i + 1]] = 0
        rng = np.random.default_rng(i)
        n = int(inst.sizes[i])
        H = _cn(rng, (n // 2, n // 2))
        blk = np.zeros((n, n), dtype=np.complex128)
        blk[n // 2:, :n // 2] = H
        blk[:n // 2, n // 2:] = H.T
        inst.K[inst.offsets[i]:inst.offsets[i + 1]] = blk.reshape(-1, order="F")
    order = oracle.nd_order(inst.grid)
    p0 = oracle.OraclePlan(inst.sizes, inst.pairs, order)
    assert p0.factor(inst.K) >= 0
    p = oracle.OraclePlan(inst.sizes, inst.pairs, order)
    assert p.factor_bk(inst.K, tile=128) == -1
    A = dense_ref.dense_K(inst.sizes, inst.pairs, inst.K)
    X = p.solve(inst.B)
    Xd = np.linalg.solve(A, inst.B.T).T
    assert (np.linalg.norm(X - Xd, axis=1) / np.linalg.norm(Xd, axis=1)).max() <= 1e-11


def test_no_interchange_reduces_to_the_plain_factor():
    # a block-dominant instance: Bunch-Kaufman keeps every diagonal pivot, so
    # the factor is the no-pivot oracle's
    inst = gen.make_instance((2, 2, 2), (10, 30), 8.0 * gen.COEF_PLAIN, 2, 99)
    order = oracle.nd_order(inst.grid)
    p0 = oracle.OraclePlan(inst.sizes, inst.pairs, order)
    assert p0.factor(inst.K) == -1
    p = oracle.OraclePlan(inst.sizes, inst.pairs, order)
    assert p.factor_bk(inst.K, tile=16) == -1
    for I in range(inst.nb):
        perm, doff = p.pivots(I)
        assert np.array_equal(perm, np.arange(inst.sizes[I])) and not np.any(doff)
        assert np.abs(p.block(I, I) - p0.block(I, I)).max() <= 1e-13 * np.abs(p0.block(I, I)).max()
        for J in p.struct(I):
            assert np.abs(p.block(J, I) - p0.block(J, I)).max() <= 1e-13
    assert np.abs(p.solve(inst.B) - p0.solve(inst.B)).max() <= 1e-12


def test_zero_column_reports_its_row():
    inst = gen.make_instance((2, 2, 1), 6, 0.0, 1, 5)
    I = int(oracle.nd_order(inst.grid)[0])
    blk = inst.K[inst.offsets[I]:inst.offsets[I + 1]].reshape(6, 6, order="F")
    blk[:, 2] = 0
    blk[2, :] = 0
    inst.K[inst.offsets[I]:inst.offsets[I + 1]] = blk.reshape(-1, order="F")
    # the row and column are zero inside the block only; the interface's
    # couplings to its neighbours are zeroed too so the column is singular
    for k, (a, b) in enumerate(inst.pairs.tolist()):
        o = int(inst.offsets[inst.nb + k])
        na, nbb = int(inst.sizes[a]), int(inst.sizes[b])
        B = inst.K[o:o + na * nbb].reshape(na, nbb, order="F")
        if a == I:
            B[2, :] = 0
        if b == I:
            B[:, 2] = 0
        inst.K[o:o + na * nbb] = B.reshape(-1, order="F")
    p = oracle.OraclePlan(inst.sizes, inst.pairs, oracle.nd_order(inst.grid))
    r = p.factor_bk(inst.K, tile=128)
    assert r == int(inst.row_offsets[I]) + 2
