"""GPU: in-tile Bunch-Kaufman pivoting (d3m_options.pivot) against the
oracle's segment-restricted Bunch-Kaufman (the same pivot rule on the same
tiles): pivots, factor blocks and D element by element in FP64, and x.
Inputs without a diagonal shift need interchanges; zero diagonal blocks
break the unpivoted factorization and not the pivoted one."""
import numpy as np
import pytest

import oracle
from paper_2002_05026_amd import instances as gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _d3m():
    import paper_2002_05026_amd as d3m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert d3m.device_ok(), "libd3m.so has no usable gfx950 device"
    return d3m


def _run(d3m, inst, precision, tile, **opt):
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, tile=tile)
    K = torch.from_numpy(inst.K).cuda()
    B = torch.from_numpy(inst.B).cuda()
    f = d3m.Factor(plan, precision, nrhs_max=inst.B.shape[0], pivot=True, **opt)
    f.factorize(K)
    X = f.solve(B).cpu().numpy()
    return plan, f, X, f.status()


def _oracle_bk(inst, tile):
    p = oracle.OraclePlan(inst.sizes, inst.pairs, oracle.nd_order(inst.grid))
    assert p.factor_bk(inst.K, tile=tile) == -1
    return p


@pytest.mark.parametrize("grid,lo,hi,tile", [((2, 2, 2), 20, 70, 32), ((2, 2, 1), 100, 300, 128),
                                             ((3, 2, 2), 30, 90, 64)])
def test_pivoted_fp64_matches_oracle_elementwise(grid, lo, hi, tile):
    d3m = _d3m()
    inst = gen.make_instance(grid, (lo, hi), 0.0, 3, 3100 + lo)
    print(f"[case] pivot fp64 grid={grid} N={inst.N} tile={tile}", flush=True)
    plan, f, X, st = _run(d3m, inst, d3m.C128, tile)
    assert st["status"] == 0, st
    p = _oracle_bk(inst, tile)
    n2 = 0
    for I in range(inst.nb):
        perm, doff = f.pivots(I)
        operm, odoff = p.pivots(I)
        assert np.array_equal(perm, operm), I
        assert np.abs(doff - odoff).max() <= 1e-12 * max(1.0, np.abs(odoff).max())
        n2 += np.count_nonzero(odoff)
        g, o = f.block(I, I), p.block(I, I)
        low = np.tril(np.ones_like(o.real, dtype=bool))
        assert np.abs(g[low] - o[low]).max() <= 1e-12 * np.abs(o[low]).max(), I
        for J in p.struct(I):
            oJ = p.block(J, I)
            assert np.abs(f.block(J, I) - oJ).max() <= 1e-12 * max(1.0, np.abs(oJ).max()), (J, I)
    assert n2 > 0  # 2x2 pivots were taken
    Xo = p.solve(inst.B)
    assert (np.linalg.norm(X - Xo, axis=1) / np.linalg.norm(Xo, axis=1)).max() <= 1e-10
    assert oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, inst.B).max() <= 1e-12


def test_pivoted_mixed_refinement_certifies():
    d3m = _d3m()
    inst = gen.make_instance((2, 2, 2), (40, 150), 0.0, 4, 3200)
    print(f"[case] pivot c64 N={inst.N}", flush=True)
    plan, f, X, st = _run(d3m, inst, d3m.C64_IR, 64, tol=1e-10, max_iter=20)
    assert st["status"] == 0, st
    assert oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, inst.B).max() <= 1e-10


def test_pivoting_solves_where_the_plain_factor_fails():
    # zero diagonal blocks with an anti-diagonal coupling inside: the first
    # pivot of the unpivoted factorization is zero
    d3m = _d3m()
    inst = gen.make_instance((2, 2, 1), 40, 0.0, 2, 3300)
    rng = np.random.default_rng(5)
    for i in range(inst.nb):
        n = int(inst.sizes[i])
        H = (rng.standard_normal((n // 2, n // 2)) + 1j * rng.standard_normal((n // 2, n // 2))) / np.sqrt(2)
        blk = np.zeros((n, n), dtype=np.complex128)
        blk[n // 2:, :n // 2] = H
        blk[:n // 2, n // 2:] = H.T
        inst.K[inst.offsets[i]:inst.offsets[i + 1]] = blk.reshape(-1, order="F")
    print(f"[case] pivot zero-diagonal N={inst.N}", flush=True)
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, tile=32)
    K = torch.from_numpy(inst.K).cuda()
    f0 = d3m.Factor(plan, d3m.C128, nrhs_max=2)
    f0.factorize(K)
    f0.solve(torch.from_numpy(inst.B).cuda())
    assert f0.status()["status"] == 1  # D3M_ZERO_PIVOT without pivoting
    for prec in (d3m.C128, d3m.C64_IR):
        # one tile per interface: the whole diagonal block is the pivot search
        plan, f, X, st = _run(d3m, inst, prec, 64, tol=1e-10, max_iter=20)
        assert st["status"] == 0, st
        bound = 1e-12 if prec == d3m.C128 else 1e-10
        assert oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, inst.B).max() <= bound
    # pivoting is restricted to tiles: with tiles of 32 the first tile of each
    # interface, [0 H1; H1^T 0] with H1 of 20 x 12, has rank 24 < 32, and the
    # device reports the zero pivot where the oracle with the same tiles does
    plan, f, X, st = _run(d3m, inst, d3m.C128, 32)
    p = oracle.OraclePlan(inst.sizes, inst.pairs, oracle.nd_order(inst.grid))
    r = p.factor_bk(inst.K, tile=32)
    assert r >= 0 and st["status"] == 1 and st["pivot_row"] == r, (r, st)


def test_pivoting_on_a_dominant_input_keeps_the_diagonal():
    # block-dominant input: no interchange, and the factor is the unpivoted one
    d3m = _d3m()
    inst = gen.make_instance((2, 2, 2), (20, 70), 8.0 * gen.COEF_PLAIN, 2, 3400)
    print(f"[case] pivot dominant N={inst.N}", flush=True)
    plan, f, X, st = _run(d3m, inst, d3m.C128, 32)
    assert st["status"] == 0
    g = d3m.Factor(plan, d3m.C128, nrhs_max=2)
    g.factorize(torch.from_numpy(inst.K).cuda())
    Xg = g.solve(torch.from_numpy(inst.B).cuda()).cpu().numpy()
    for I in range(inst.nb):
        perm, doff = f.pivots(I)
        assert np.array_equal(perm, np.arange(inst.sizes[I])) and not np.any(doff)
        o = g.block(I, I)
        assert np.abs(f.block(I, I) - o).max() <= 1e-13 * np.abs(o).max()
    assert np.abs(X - Xg).max() <= 1e-12 * np.abs(Xg).max()
