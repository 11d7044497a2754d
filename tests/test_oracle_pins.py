"""Pins of the CPU oracle against facts fixed by the mathematics.

Nothing here compares the oracle with itself: every check is a closed form,
a hand-derived golden value (tests/golden), a brute-force dense algorithm, a
library routine on a special case that reduces to it, or an invariant.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2002_05026_amd import instances as gen
from tests import dense_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

GRIDS = [(2, 2, 1), (2, 2, 2), (3, 3, 2), (4, 4, 2), (8, 8, 1), (4, 4, 4), (6, 6, 6)]


def closed_form_ifaces(g):
    a, b, c = g
    return (a - 1) * b * c + a * (b - 1) * c + a * b * (c - 1)


def closed_form_pairs(g):
    # sum over domains of C(deg, 2), deg = number of face neighbours
    a, b, c = g
    tot = 0
    for x in range(a):
        for y in range(b):
            for z in range(c):
                deg = sum([x > 0, x < a - 1, y > 0, y < b - 1, z > 0, z < c - 1])
                tot += deg * (deg - 1) // 2
    return tot


@pytest.mark.parametrize("g", GRIDS)
def test_pattern_closed_forms(g):
    ifs = oracle.grid_interfaces(g)
    pairs = oracle.grid_pairs(g)
    assert ifs.shape[0] == closed_form_ifaces(g)
    assert pairs.shape[0] == closed_form_pairs(g)
    # generator and oracle enumerate independently and must agree
    assert np.array_equal(ifs, gen.grid_interfaces(g))
    assert np.array_equal(pairs, gen.grid_pairs(g))


def test_pattern_known_counts():
    # interface and pair counts of the five workloads and the batch grids
    want = {(2, 2, 1): (4, 4), (2, 2, 2): (12, 24), (3, 3, 2): (33, 92), (4, 4, 2): (64, 200),
            (8, 8, 1): (112, 292), (4, 4, 4): (144, 528), (6, 6, 6): (540, 2232)}
    for g, (ni, npr) in want.items():
        assert oracle.grid_interfaces(g).shape[0] == ni
        assert oracle.grid_pairs(g).shape[0] == npr


def test_golden_tiny():
    gd = json.load(open(os.path.join(GOLDEN, "tiny_2x2.json")))
    g = tuple(gd["grid"])
    assert oracle.grid_interfaces(g).tolist() == gd["interfaces"]
    assert oracle.grid_pairs(g).tolist() == gd["pairs"]
    order = oracle.nd_order(g)
    assert order.tolist() == gd["order"]
    nb = len(gd["interfaces"])
    p = oracle.OraclePlan([gd["n"]] * nb, gd["pairs"], order)
    for k, v in gd["S"].items():
        assert p.struct(int(k)) == v
    st = p.stats()
    assert st["fill_blocks"] == gd["fill_blocks"]
    assert st["L_blocks"] == gd["L_blocks"]
    assert (st["fact_tasks"], st["trsm_tasks"], st["update_tasks"]) == (
        gd["tasks"]["fact"], gd["tasks"]["trsm"], gd["tasks"]["update"])
    assert st["etree_height"] == gd["etree_height"]
    assert st["nnz_L"] == gd["nnz_L"]
    assert st["flops"] == pytest.approx(gd["flops"], rel=1e-12)


# fill blocks, elimination-tree height, max |S_I| at the workload grids
FILL = {(8, 8, 1): (468, 21, 11), (4, 4, 4): (1176, 35, 23), (6, 6, 6): (9344, 89, 53),
        (2, 2, 2): (16, 7, 5), (3, 3, 2): (112, 17, 11), (4, 4, 2): (288, 19, 11)}


@pytest.mark.parametrize("g", list(FILL))
def test_fill_bruteforce(g):
    pairs = oracle.grid_pairs(g)
    order = oracle.nd_order(g)
    nb = oracle.grid_interfaces(g).shape[0]
    assert sorted(order.tolist()) == list(range(nb))
    p = oracle.OraclePlan(np.ones(nb), pairs, order)
    st = p.stats()
    brute = dense_ref.brute_fill(nb, pairs, order)
    mine = {(J, I) for I in range(nb) for J in p.struct(I)}
    assert mine == brute
    fill, height, maxs = FILL[g]
    assert st["fill_blocks"] == fill
    assert st["L_blocks"] == fill + pairs.shape[0]
    assert st["etree_height"] == height
    assert st["max_S"] == maxs


def test_nd_separators_are_separators():
    # every interface of the low half and every interface of the high half of
    # the top split must never share a domain (no pattern edge across halves)
    for g in [(4, 4, 4), (8, 8, 1), (3, 3, 2)]:
        order = oracle.nd_order(g).tolist()
        pairs = oracle.grid_pairs(g)
        p = oracle.OraclePlan(np.ones(len(order)), pairs, order)
        # the elimination tree must be connected only through later blocks:
        # for each I, S_I holds only blocks later in the order
        pos = {I: k for k, I in enumerate(order)}
        for I in order:
            assert all(pos[J] > pos[I] for J in p.struct(I))


def _small(grid, lo, hi, seed, coef=gen.COEF_PLAIN, nrhs=3):
    return gen.make_instance(grid, (lo, hi), coef, nrhs, seed, with_c=True)


def _factor_check(inst, order=None):
    if order is None:
        order = oracle.nd_order(inst.grid) if inst.nb == gen.grid_interfaces(inst.grid).shape[0] \
            else np.arange(inst.nb)
    p = oracle.OraclePlan(inst.sizes, inst.pairs, order)
    assert p.factor(inst.K) == -1
    A = dense_ref.dense_K(inst.sizes, inst.pairs, inst.K)
    perm = dense_ref.perm_rows(inst.sizes, order)
    PAP = A[np.ix_(perm, perm)]
    # assemble the oracle's L and D in the permuted numbering
    N = inst.N
    sizes = inst.sizes.astype(np.int64)
    start = {}
    o = 0
    for I in order:
        start[int(I)] = o
        o += int(sizes[I])
    L = np.zeros((N, N), dtype=np.complex128)
    d = np.zeros(N, dtype=np.complex128)
    for I in order:
        I = int(I)
        nI, s = int(sizes[I]), start[I]
        Dg = p.block(I, I)
        L[s:s + nI, s:s + nI] = np.tril(Dg, -1) + np.eye(nI)
        d[s:s + nI] = np.diag(Dg)
        for J in p.struct(I):
            nJ, sJ = int(sizes[J]), start[J]
            L[sJ:sJ + nJ, s:s + nI] = p.block(J, I)
    return p, A, PAP, L, d, order


@pytest.mark.parametrize("case", ["tiny", "2x2x2", "3x3x2"])
def test_factor_unique_and_reconstructs(case):
    if case == "tiny":
        inst = gen.config_tiny(nrhs=2, with_c=True)
    elif case == "2x2x2":
        inst = _small((2, 2, 2), 10, 30, 11)
    else:
        inst = _small((3, 3, 2), 4, 12, 12)
    p, A, PAP, L, d, order = _factor_check(inst)
    # K = K^T exactly (complex symmetric, not Hermitian)
    assert np.array_equal(A, A.T)
    assert np.abs(A.imag).max() > 0.1
    # invariant: ||P K P^T - L D L^T||_F / ||K||_F <= 1e-13
    E = PAP - (L * d) @ L.T
    assert np.linalg.norm(E) / np.linalg.norm(A) <= 1e-13
    # uniqueness: the textbook dense scalar LDL^T gives the same L and D
    Lb, db = dense_ref.dense_ldlt_nopivot(PAP)
    assert np.abs(L - Lb).max() <= 1e-12 * max(1.0, np.abs(Lb).max())
    assert np.abs(d - db).max() <= 1e-12 * np.abs(db).max()
    # the LDL^T uses the transpose: the conjugate-transpose reconstruction must fail
    E2 = PAP - (L * d) @ L.conj().T
    assert np.linalg.norm(E2) / np.linalg.norm(A) > 1e-3


def test_solve_matches_dense_gauss():
    for inst in [gen.config_tiny(nrhs=3), _small((2, 2, 2), 10, 30, 21), _small((3, 3, 2), 3, 9, 22)]:
        order = oracle.nd_order(inst.grid)
        p = oracle.OraclePlan(inst.sizes, inst.pairs, order)
        assert p.factor(inst.K) == -1
        X = p.solve(inst.B)
        A = dense_ref.dense_K(inst.sizes, inst.pairs, inst.K)
        Xd = np.linalg.solve(A, inst.B.T).T
        fe = np.linalg.norm(X - Xd, axis=1) / np.linalg.norm(Xd, axis=1)
        assert fe.max() <= 1e-13
        eta = oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, inst.B)
        assert eta.max() <= 1e-15 * 10


def test_matvec_and_knorm_match_dense():
    inst = _small((3, 3, 2), 3, 9, 31)
    A = dense_ref.dense_K(inst.sizes, inst.pairs, inst.K)
    Y = oracle.matvec(inst.sizes, inst.pairs, inst.K, inst.B)
    assert np.abs(Y - (A @ inst.B.T).T).max() <= 1e-13 * np.abs(Y).max()
    assert oracle.k_norm_inf(inst.sizes, inst.pairs, inst.K) == pytest.approx(
        np.abs(A).sum(axis=1).max(), rel=1e-14)


def test_backward_error_against_dense_definition():
    # eta_inf = ||b - K x||_inf / (||K||_inf ||x||_inf + ||b||_inf) per column
    # (the normwise backward error that certifies every solution), evaluated
    # by hand on the dense assembled K with a residual planted exactly: x is
    # random, b = K x + r with a known r per column, so the expected value is
    # fixed before the oracle runs.  An inflated or deflated numerator or
    # denominator (a wrong norm of K, x or b) moves eta by far more than the
    # tolerance.
    inst = _small((3, 3, 2), 3, 9, 41, nrhs=4)
    A = dense_ref.dense_K(inst.sizes, inst.pairs, inst.K)
    rng = np.random.default_rng(17)
    X = (rng.standard_normal(inst.B.shape) + 1j * rng.standard_normal(inst.B.shape)) / np.sqrt(2)
    R = np.zeros_like(X)
    for j in range(X.shape[0]):
        R[j, rng.integers(inst.N)] = (0.05 + 0.1 * j) * np.exp(1j * rng.uniform(0, 2 * np.pi))
    B = (A @ X.T).T + R
    knorm = np.linalg.norm(A, np.inf)
    want = np.abs(R).max(axis=1) / (knorm * np.abs(X).max(axis=1) + np.abs(B).max(axis=1))
    got = oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, B)
    assert np.allclose(got, want, rtol=1e-12, atol=0), (got, want)
    # the planted eta is far from the values a wrong denominator would give
    alt = np.abs(R).max(axis=1) / (2 * knorm * np.abs(X).max(axis=1) + np.abs(B).max(axis=1))
    assert np.all(np.abs(alt / want - 1) > 1e-3)
    # a given ||K||_inf is used as given
    got2 = oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, B, knorm_inf=2 * knorm)
    assert np.allclose(got2, alt, rtol=1e-12, atol=0)
    # an exact solution has eta at rounding level
    Xe = np.linalg.solve(A, inst.B.T).T
    assert oracle.backward_error(inst.sizes, inst.pairs, inst.K, Xe, inst.B).max() <= 1e-15


def test_special_single_interface():
    # one interface: the method is a dense LDL^T of one block
    inst = gen.make_instance((2, 1, 1), 40, gen.COEF_PLAIN, 1, 5)
    p = oracle.OraclePlan(inst.sizes, inst.pairs, [0])
    assert p.factor(inst.K) == -1
    A = dense_ref.dense_K(inst.sizes, inst.pairs, inst.K)
    Lb, db = dense_ref.dense_ldlt_nopivot(A)
    Dg = p.block(0, 0)
    assert np.abs(np.tril(Dg, -1) + np.eye(40) - Lb).max() < 1e-12
    assert np.abs(np.diag(Dg) - db).max() < 1e-12 * np.abs(db).max()


def test_special_block_diagonal():
    # all off-diagonal blocks zero: L is block diagonal
    inst = _small((2, 2, 2), 5, 9, 41)
    inst.K[inst.offsets[inst.nb]:] = 0
    order = oracle.nd_order(inst.grid)
    p = oracle.OraclePlan(inst.sizes, inst.pairs, order)
    assert p.factor(inst.K) == -1
    for I in range(inst.nb):
        for J in p.struct(I):
            assert np.abs(p.block(J, I)).max() == 0.0
        Lb, db = dense_ref.dense_ldlt_nopivot(inst.diag_block(I))
        Dg = p.block(I, I)
        assert np.abs(np.diag(Dg) - db).max() < 1e-12 * np.abs(db).max()


def test_special_scalar_blocks():
    # all interfaces of size 1: a scalar sparse LDL^T
    inst = gen.make_instance((3, 3, 2), 1, gen.COEF_PLAIN, 2, 6)
    p, A, PAP, L, d, order = _factor_check(inst)
    Lb, db = dense_ref.dense_ldlt_nopivot(PAP)
    assert np.abs(L - Lb).max() < 1e-12
    assert np.abs(d - db).max() < 1e-12 * np.abs(db).max()


def test_special_real_spd_is_cholesky():
    # real SPD input: L diag(sqrt(d)) is the Cholesky factor (library routine)
    inst = _small((2, 2, 2), 5, 12, 51, coef=3.0)
    inst.K[:] = inst.K.real
    # make every diagonal sign positive: add 2*|shift| on the diagonal
    for I in range(inst.nb):
        n = int(inst.sizes[I])
        o = int(inst.offsets[I])
        blk = inst.K[o:o + n * n].reshape(n, n, order="F")
        blk[np.arange(n), np.arange(n)] = np.abs(blk[np.arange(n), np.arange(n)]) + 6 * math.sqrt(n)
    p, A, PAP, L, d, order = _factor_check(inst)
    assert np.all(np.linalg.eigvalsh(PAP.real) > 0)
    C = np.linalg.cholesky(PAP.real)
    assert np.abs(L.real * np.sqrt(d.real) - C).max() < 1e-12 * np.abs(C).max()


def test_zero_pivot_reports_global_index():
    inst = gen.make_instance((2, 2, 1), 1, gen.COEF_PLAIN, 1, 7)
    # interface 2 is eliminated first; zero its 1x1 diagonal block
    inst.K[inst.offsets[2]] = 0
    p = oracle.OraclePlan(inst.sizes, inst.pairs, oracle.nd_order(inst.grid))
    assert p.factor(inst.K) == 2
    inst2 = gen.config_tiny()
    inst2.K[:] = np.nan
    p2 = oracle.OraclePlan(inst2.sizes, inst2.pairs, oracle.nd_order(inst2.grid))
    assert p2.factor(inst2.K) == 2 * 48  # first row of interface 2


def _dense_grad(A, b, c):
    # J = Re(c^T x), x = A^{-1} b (holomorphic convention): dJ/db = lam,
    # dJ/dA = -lam x^T with lam = A^{-T} c
    x = np.linalg.solve(A, b)
    lam = np.linalg.solve(A.T, c)
    return x, lam, -np.outer(lam, x)


def test_gradient_identity_fd_and_dense():
    inst = _small((2, 2, 2), 6, 12, 61, nrhs=2)
    order = oracle.nd_order(inst.grid)
    p = oracle.OraclePlan(inst.sizes, inst.pairs, order)
    assert p.factor(inst.K) == -1
    X = p.solve(inst.B)
    Lam = p.solve(inst.C)
    # identity Re(c^T x) = Re(lam^T b) since K = K^T
    lhs = np.real(np.sum(inst.C * X))
    rhs = np.real(np.sum(Lam * inst.B))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    dK = oracle.grad_K(inst.sizes, inst.pairs, Lam, X, inst.K.shape[0])
    # against the dense gradient -lam x^T symmetrized over (I,J) and (J,I)
    A = dense_ref.dense_K(inst.sizes, inst.pairs, inst.K)
    G = np.zeros_like(A)
    for k in range(X.shape[0]):
        _, lam, g = _dense_grad(A, inst.B[k], inst.C[k])
        G += g
    Gs = 0.5 * (G + G.T)
    r0 = inst.row_offsets
    for I in range(inst.nb):
        blk = dK[inst.offsets[I]:inst.offsets[I + 1]].reshape(inst.sizes[I], inst.sizes[I], order="F")
        ref = Gs[r0[I]:r0[I + 1], r0[I]:r0[I + 1]]
        assert np.abs(blk - ref).max() <= 1e-11 * np.abs(Gs).max()
    for k, (I, J) in enumerate(inst.pairs.tolist()):
        o0, o1 = inst.offsets[inst.nb + k], inst.offsets[inst.nb + k + 1]
        blk = dK[o0:o1].reshape(inst.sizes[I], inst.sizes[J], order="F")
        ref = Gs[r0[I]:r0[I + 1], r0[J]:r0[J + 1]]
        assert np.abs(blk - ref).max() <= 1e-11 * np.abs(Gs).max()
    # central finite differences along a random symmetric pattern direction
    rng = np.random.default_rng(5)
    E = (rng.standard_normal(inst.K.shape) + 1j * rng.standard_normal(inst.K.shape))
    Ed = dense_ref.dense_K(inst.sizes, inst.pairs, E)
    h = 1e-6 * np.linalg.norm(inst.K) / np.linalg.norm(E)

    def J(Kflat):
        Ad = dense_ref.dense_K(inst.sizes, inst.pairs, Kflat)
        Xd = np.linalg.solve(Ad, inst.B.T)
        return np.real(np.sum(inst.C.T * Xd))

    fd = (J(inst.K + h * E) - J(inst.K - h * E)) / (2 * h)
    # directional derivative on the full symmetric matrix: <G_full, E_full>
    # with the bilinear pairing (no conjugate)
    ad = 0.0
    for I in range(inst.nb):
        blk = dK[inst.offsets[I]:inst.offsets[I + 1]].reshape(inst.sizes[I], inst.sizes[I], order="F")
        eb = Ed[r0[I]:r0[I + 1], r0[I]:r0[I + 1]]
        ad += np.real(np.sum(blk * eb))
    for k, (I, J_) in enumerate(inst.pairs.tolist()):
        o0, o1 = inst.offsets[inst.nb + k], inst.offsets[inst.nb + k + 1]
        blk = dK[o0:o1].reshape(inst.sizes[I], inst.sizes[J_], order="F")
        eb = Ed[r0[I]:r0[I + 1], r0[J_]:r0[J_ + 1]]
        ad += 2 * np.real(np.sum(blk * eb))
    assert abs(fd - ad) <= 1e-6 * abs(ad)


def test_generator_exact_symmetry_and_recipe():
    inst = gen.config_tiny()
    for I in range(inst.nb):
        blk = inst.diag_block(I)
        assert np.array_equal(blk, blk.T)
    # the diagonal shift: |diag - offdiag-noise| ~ |3+0.5j| sqrt(48)
    d = np.concatenate([np.diag(inst.diag_block(I)) for I in range(inst.nb)])
    assert np.median(np.abs(d)) > 0.7 * abs(gen.COEF_PLAIN) * math.sqrt(48)
    b = gen.config_batch(count=3, nrhs=1, size_range=(5, 10))
    assert len(b) == 3 and all(inst.grid in gen.BATCH_GRIDS for inst in b)


def test_flop_counts_at_mean_sizes():
    # factor flop split at uniform mean sizes (8 real flops per complex
    # multiply-add): diagonal (4/3) n^3, TRSM 4 n_J n_I^2, update
    # 8 n_J n_K n_I (4 n_J^2 n_I on the diagonal), in GFLOP
    want = {((8, 8, 1), 300): (4.032, 82.08, 628.128, 73.4568e6),
            ((4, 4, 4), 450): (17.496, 621.108, 8564.292, 359.6724e6),
            ((6, 6, 6), 500): (90.0, 5788.0, 162514.0, 2961.635e6)}
    for (g, n), (fd, ft, fu, nnz) in want.items():
        nb = oracle.grid_interfaces(g).shape[0]
        p = oracle.OraclePlan(np.full(nb, n), oracle.grid_pairs(g), oracle.nd_order(g))
        s = p.stats()
        assert s["flops_diag"] / 1e9 == pytest.approx(fd, rel=1e-9)
        assert s["flops_trsm"] / 1e9 == pytest.approx(ft, rel=1e-9)
        assert s["flops_update"] / 1e9 == pytest.approx(fu, rel=1e-9)
        assert s["nnz_L"] == pytest.approx(nnz, rel=1e-9)
