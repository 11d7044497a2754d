"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Tolerances: FP64 path relative backward error eta_inf <= 1e-12 and
||x - x_oracle|| / ||x_oracle|| <= 1e-10 per column; factor entries L, D
against the oracle's (unique for a fixed elimination order) to 1e-12
relative; mixed precision: eta_inf <= 1e-10 after FP64 refinement and the
forward error against the oracle within kappa * eta.
"""
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


def _run(inst, precision, tile=0, nrhs=None, order=None, grid=True, **opt):
    d3m = _d3m()
    print(f"[case] grid={inst.grid} N={inst.N} prec={precision} tile={tile}", flush=True)
    plan = d3m.Plan(inst.sizes, inst.pairs, order=order, grid=inst.grid if (grid and order is None) else None,
                    tile=tile)
    B = inst.B if nrhs is None else inst.B[:nrhs]
    Kt = torch.from_numpy(inst.K).cuda()
    Bt = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    f = d3m.Factor(plan, precision, nrhs_max=Bt.shape[0], **opt)
    f.factorize(Kt)
    X = f.solve(Bt)
    st = f.status()
    return plan, f, Kt, Bt, X.cpu().numpy(), st


def _oracle_solution(inst, order, B):
    p = oracle.OraclePlan(inst.sizes, inst.pairs, order)
    assert p.factor(inst.K) == -1
    return p, p.solve(B)


def _fwd_err(X, Xo):
    return (np.linalg.norm(X - Xo, axis=1) / np.linalg.norm(Xo, axis=1)).max()


@pytest.mark.parametrize("tile", [0, 16, 32])
def test_tiny_fp64_factor_and_solve(tile):
    inst = gen.config_tiny(nrhs=3)
    plan, f, Kt, Bt, X, st = _run(inst, 0, tile=tile)
    assert st["status"] == 0, st
    order = oracle.nd_order(inst.grid)
    p, Xo = _oracle_solution(inst, order, inst.B)
    assert _fwd_err(X, Xo) <= 1e-10
    eta = oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, inst.B)
    assert eta.max() <= 1e-12
    # the device's own eta (its FP64 residual) certifies the same bound
    assert 0 <= st["eta"] <= 1e-12
    # factor entries, element by element (same elimination order)
    for I in range(inst.nb):
        g = f.block(I, I)
        o = p.block(I, I)
        low = np.tril(np.ones_like(o.real, dtype=bool))
        assert np.abs(g[low] - o[low]).max() <= 1e-12 * np.abs(o[low]).max()
        for J in p.struct(I):
            assert np.abs(f.block(J, I) - p.block(J, I)).max() <= 1e-12 * max(1.0, np.abs(p.block(J, I)).max())


@pytest.mark.parametrize("grid,lo,hi,tile", [((2, 2, 2), 20, 70, 32), ((3, 3, 2), 5, 40, 16),
                                              ((2, 2, 2), 100, 300, 0), ((4, 4, 2), 30, 90, 48)])
def test_small_fp64_parity(grid, lo, hi, tile):
    inst = gen.make_instance(grid, (lo, hi), gen.COEF_PLAIN, 5, 101 + lo)
    plan, f, Kt, Bt, X, st = _run(inst, 0, tile=tile)
    assert st["status"] == 0, st
    order = oracle.nd_order(inst.grid)
    p, Xo = _oracle_solution(inst, order, inst.B)
    assert _fwd_err(X, Xo) <= 1e-10
    assert oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, inst.B).max() <= 1e-12
    # a sample of factor blocks
    for I in list(range(inst.nb))[:: max(1, inst.nb // 4)]:
        o = p.block(I, I)
        g = f.block(I, I)
        low = np.tril(np.ones_like(o.real, dtype=bool))
        assert np.abs(g[low] - o[low]).max() <= 1e-12 * np.abs(o[low]).max()
        for J in p.struct(I)[:2]:
            assert np.abs(f.block(J, I) - p.block(J, I)).max() <= 1e-12 * max(1.0, np.abs(p.block(J, I)).max())


@pytest.mark.parametrize("grid,lo,hi,tile", [((2, 2, 2), 20, 70, 32), ((3, 3, 2), 60, 200, 0)])
def test_small_mixed_ir_parity(grid, lo, hi, tile):
    inst = gen.make_instance(grid, (lo, hi), gen.COEF_PRECISION, 4, 202 + lo)
    plan, f, Kt, Bt, X, st = _run(inst, 1, tile=tile, tol=1e-10, max_iter=10)
    assert st["status"] == 0, st
    assert 1 <= st["ir_iters"] <= 3, st
    eta = oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, inst.B)
    assert eta.max() <= 1e-10
    order = oracle.nd_order(inst.grid)
    p, Xo = _oracle_solution(inst, order, inst.B)
    # kappa <= ~20 for this recipe: forward error within 20 * 1e-10 (loose)
    assert _fwd_err(X, Xo) <= 1e-8


@pytest.mark.parametrize("precision", [0, 1])
def test_wide_rhs_parity(precision):
    # 100 right-hand sides: the FP64 residual runs in chunks of 64 columns
    # (one full, one ragged); every column must be certified
    inst = gen.make_instance((2, 2, 2), (40, 120), gen.COEF_PRECISION, 100, 505)
    plan, f, Kt, Bt, X, st = _run(inst, precision, tile=32, tol=1e-10, max_iter=10)
    assert st["status"] == 0, st
    eta = oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, inst.B)
    bound = 1e-12 if precision == 0 else 1e-10
    assert eta.max() <= bound
    assert 0 <= st["eta"] <= bound
    order = oracle.nd_order(inst.grid)
    p, Xo = _oracle_solution(inst, order, inst.B)
    assert _fwd_err(X, Xo) <= (1e-10 if precision == 0 else 1e-6)  # complex64: certified by eta below


def test_host_sync_refinement_matches_device_flag():
    inst = gen.make_instance((2, 2, 2), (30, 60), gen.COEF_PLAIN, 2, 303)
    _, _, _, _, X1, s1 = _run(inst, 1, tile=32)
    _, _, _, _, X2, s2 = _run(inst, 1, tile=32, ir_host_sync=True)
    assert s1["status"] == 0 and s2["status"] == 0
    assert s1["ir_iters"] == s2["ir_iters"]
    assert np.array_equal(X1, X2)


@pytest.mark.parametrize("precision", [0, 1])
def test_knorm_matches_oracle(precision):
    # ||K||_inf from the device (row tiles of 128 and ragged ones, all three
    # block modes) against the oracle's full symmetric row sums
    inst = gen.make_instance((3, 2, 2), (60, 300), gen.COEF_PRECISION, 1, 606)
    d3m = _d3m()
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid)
    f = d3m.Factor(plan, precision, nrhs_max=1)
    f.factorize(torch.from_numpy(inst.K).cuda())
    st = f.status()
    ref = oracle.k_norm_inf(inst.sizes, inst.pairs, inst.K)
    assert abs(st["knorm"] - ref) <= 1e-13 * ref, (st["knorm"], ref)


def test_determinism_bitwise():
    inst = gen.make_instance((3, 3, 2), (40, 150), gen.COEF_PLAIN, 3, 404)
    d3m = _d3m()
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, tile=32)
    Kt = torch.from_numpy(inst.K).cuda()
    Bt = torch.from_numpy(inst.B).cuda()
    xs = []
    for _ in range(3):
        f = d3m.Factor(plan, 0, nrhs_max=3)
        f.factorize(Kt)
        xs.append(f.solve(Bt).cpu().numpy())
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])
    # a different list schedule (sequential ticket order) gives the same bits
    plan2 = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, tile=32, sched=1)
    f2 = d3m.Factor(plan2, 0, nrhs_max=3)
    f2.factorize(Kt)
    assert np.array_equal(xs[0], f2.solve(Bt).cpu().numpy())


def test_zero_pivot_status():
    d3m = _d3m()
    inst = gen.make_instance((2, 2, 1), 1, gen.COEF_PLAIN, 1, 7)
    inst.K[inst.offsets[2]] = 0  # interface 2 is eliminated first
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid)
    f = d3m.Factor(plan, 0, nrhs_max=1)
    f.factorize(torch.from_numpy(inst.K).cuda())
    f.solve(torch.from_numpy(inst.B).cuda())
    st = f.status()
    assert st["status"] == 1 and st["pivot_row"] == 2


def test_minimum_degree_and_explicit_order():
    # no grid: the library orders by minimum degree; x is unique regardless
    inst = gen.make_instance((3, 3, 2), (20, 50), gen.COEF_PLAIN, 2, 505)
    plan, f, Kt, Bt, X, st = _run(inst, 0, tile=32, grid=False)
    assert st["status"] == 0
    _, Xo = _oracle_solution(inst, np.arange(inst.nb), inst.B)
    assert _fwd_err(X, Xo) <= 1e-10
    rng = np.random.default_rng(3)
    order = rng.permutation(inst.nb)
    plan, f, Kt, Bt, X2, st = _run(inst, 0, tile=16, order=order)
    assert st["status"] == 0
    p, Xo2 = _oracle_solution(inst, order, inst.B)
    assert _fwd_err(X2, Xo2) <= 1e-10
    I = int(order[0])
    assert np.abs(f.block(I, I) - np.tril(p.block(I, I))).max() <= 1e-12 * np.abs(p.block(I, I)).max()


def test_adjoint_against_oracle_gradient():
    d3m = _d3m()
    inst = gen.make_instance((2, 2, 2), (20, 60), gen.COEF_PLAIN, 3, 606, with_c=True)
    for prec in (0, 1):
        plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, tile=32)
        Kt = torch.from_numpy(inst.K).cuda()
        f = d3m.Factor(plan, prec, nrhs_max=3)
        f.factorize(Kt)
        X = f.solve(torch.from_numpy(inst.B).cuda())
        Lam, dK = f.adjoint(X, torch.from_numpy(inst.C).cuda())
        assert f.status()["status"] == 0
        p, Xo = _oracle_solution(inst, oracle.nd_order(inst.grid), inst.B)
        Lo = p.solve(inst.C)
        dKo = oracle.grad_K(inst.sizes, inst.pairs, Lo, Xo, inst.K.shape[0])
        tol = 1e-10 if prec == 0 else 1e-8
        assert _fwd_err(Lam.cpu().numpy(), Lo) <= tol
        g = dK.cpu().numpy()
        assert np.abs(g - dKo).max() <= tol * np.abs(dKo).max()


def test_batch_matches_single_runs():
    d3m = _d3m()
    insts = gen.config_batch(count=4, nrhs=2, size_range=(20, 60))
    factors, Ks, Bs, Xs = [], [], [], []
    for inst in insts:
        plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, tile=32)
        factors.append(d3m.Factor(plan, 1, nrhs_max=2))
        Ks.append(torch.from_numpy(inst.K).cuda())
        Bs.append(torch.from_numpy(inst.B).cuda())
        Xs.append(torch.empty_like(Bs[-1]))
    b = d3m.Batch(factors)
    b.run(Ks, Bs, Xs)
    for inst, f, K, B, X in zip(insts, factors, Ks, Bs, Xs):
        st = f.status()
        assert st["status"] == 0, st
        eta = oracle.backward_error(inst.sizes, inst.pairs, inst.K, X.cpu().numpy(), inst.B)
        assert eta.max() <= 1e-10


def test_forced_fp64_fallback_of_diagonal_tiles():
    # a growth threshold that every tile trips: each diagonal tile of the
    # complex64 factor is re-factored in FP64; refinement still certifies
    d3m = _d3m()
    inst = gen.make_instance((2, 2, 2), (40, 150), gen.COEF_PRECISION, 3, 1111)
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, tile=32)
    K = torch.from_numpy(inst.K).cuda()
    B = torch.from_numpy(inst.B).cuda()
    f = d3m.Factor(plan, 1, nrhs_max=3, growth_dmin=1e30)
    f.factorize(K)
    X = f.solve(B).cpu().numpy()
    st = f.status()
    assert st["status"] == 0 and st["fallbacks"] == plan.info["ntiles"], st
    assert oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, inst.B).max() <= 1e-10
    # the FP64 tiles make x0 at least as good as the plain complex64 factor
    g = d3m.Factor(plan, 1, nrhs_max=3)
    g.factorize(K)
    g.solve(B)
    sg = g.status()
    assert sg["fallbacks"] == 0
    assert st["eta_hist"][0] <= 2 * sg["eta_hist"][0]
    # with the fallback switched off nothing is re-factored
    h = d3m.Factor(plan, 1, nrhs_max=3, growth_dmin=1e30, fallback=False)
    h.factorize(K)
    h.solve(B)
    assert h.status()["fallbacks"] == 0
    # the other trigger, max|L| above its bound: every tile with a multiplier
    # trips (a one-row tile has none), and refinement still certifies
    q = d3m.Factor(plan, 1, nrhs_max=3, growth_lmax=1e-30)
    q.factorize(K)
    Xq = q.solve(B).cpu().numpy()
    sq = q.status()
    assert sq["status"] == 0 and 0 < sq["fallbacks"] <= plan.info["ntiles"], sq
    assert oracle.backward_error(inst.sizes, inst.pairs, inst.K, Xq, inst.B).max() <= 1e-10


@pytest.mark.parametrize("precision", [0, 1])
def test_rhs_groups_are_bitwise_the_ungrouped_solve(precision):
    # a grouped solve DAG computes every column with the same products in the
    # same order as the ungrouped one: bitwise equal results
    d3m = _d3m()
    inst = gen.make_instance((3, 2, 2), (40, 200), gen.COEF_PRECISION, 64, 707)
    K = torch.from_numpy(inst.K).cuda()
    xs = []
    for groups, nrhs in ((1, 64), (2, 64), (4, 64), (2, 37)):
        print(f"[case] rhs groups {groups} nrhs {nrhs} prec {precision}", flush=True)
        plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, rhs_groups=groups)
        f = d3m.Factor(plan, precision, nrhs_max=64)
        f.factorize(K)
        X = f.solve(torch.from_numpy(np.ascontiguousarray(inst.B[:nrhs])).cuda()).cpu().numpy()
        assert f.status()["status"] == 0
        xs.append(X)
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])
    assert np.array_equal(xs[0][:37], xs[3])
    eta = oracle.backward_error(inst.sizes, inst.pairs, inst.K, xs[1], inst.B)
    assert eta.max() <= (1e-12 if precision == 0 else 1e-10)


@pytest.mark.parametrize("solve_tile,merge", [(32, 1), (128, 4), (64, 16)])
def test_tuning_knobs_against_oracle(solve_tile, merge):
    d3m = _d3m()
    inst = gen.make_instance((3, 3, 2), (60, 200), gen.COEF_PLAIN, 4, 808)
    print(f"[case] knobs solve_tile {solve_tile} merge {merge}", flush=True)
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, solve_tile=solve_tile, merge=merge, rhs_groups=2)
    f = d3m.Factor(plan, 0, nrhs_max=4)
    f.factorize(torch.from_numpy(inst.K).cuda())
    X = f.solve(torch.from_numpy(inst.B).cuda()).cpu().numpy()
    assert f.status()["status"] == 0
    p, Xo = _oracle_solution(inst, oracle.nd_order(inst.grid), inst.B)
    assert _fwd_err(X, Xo) <= 1e-10


@pytest.mark.parametrize("solve_tile,nrhs,precision", [(32, 1, 0), (64, 3, 0), (128, 8, 0), (128, 9, 0),
                                                      (64, 1, 1), (128, 8, 1)])
def test_few_rhs_solve_products_against_oracle(solve_tile, nrhs, precision):
    # solve tasks with <= 8 right-hand-side columns take the vector product
    # path (up to 128 rows x 8 columns = two outputs per thread); 9 columns
    # take the MFMA tiles
    d3m = _d3m()
    inst = gen.make_instance((3, 3, 2), (60, 200), gen.COEF_PLAIN, nrhs, 909 + nrhs)
    print(f"[case] few-rhs solve_tile {solve_tile} nrhs {nrhs} precision {precision}", flush=True)
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, solve_tile=solve_tile)
    f = d3m.Factor(plan, precision, nrhs_max=nrhs)
    f.factorize(torch.from_numpy(inst.K).cuda())
    X = f.solve(torch.from_numpy(inst.B).cuda()).cpu().numpy()
    st = f.status()
    assert st["status"] == 0, st
    p, Xo = _oracle_solution(inst, oracle.nd_order(inst.grid), inst.B)
    assert _fwd_err(X, Xo) <= (1e-10 if precision == 0 else 1e-6)  # complex64: certified by eta below
    assert oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, inst.B).max() <= (1e-12 if precision == 0
                                                                                      else 1e-10)


def test_fp64_fallback_recovers_a_pivot_fp32_cannot_carry():
    # The first eliminated interface's diagonal block has small integer
    # entries (exact in complex64) and, at rows k, k+1, the pair
    # [[12288, 12289], [12289, 12290]] coupled to row k+2 by 64: the block is
    # well conditioned (cond ~3e3), but its pivot at k+1 is 12290 -
    # 12289^2/12288 = -1/12288, a cancellation to 8 digits.  FP32 elimination
    # cannot carry it: the multiplier 12289/12288 rounds at 6e-8, times 12289
    # that is an absolute error of 7e-4, several times the pivot itself.  The
    # growth check trips (min|d| < 1e-4 max|A|) and the tile is factored
    # again in FP64 from the stored entries, which are exact: D must then be
    # the oracle's FP64 elimination of K (rounded to complex64) to complex64
    # precision, and the solve must reach the tolerance.
    # The right pivot does not make the first solution better: below it L
    # grows by 1/|d| (L(k+2, k+1) = 64 * 12288), and the FP32 Schur updates
    # carry that growth either way; in-tile pivoting, which takes rows
    # k+1, k+2 as a 2x2 pivot, is what removes it (x0 at least 10x better).
    d3m = _d3m()
    inst = gen.make_instance((2, 2, 1), 40, gen.COEF_PLAIN, 2, 1212)
    order = oracle.nd_order(inst.grid)
    I = int(order[0])
    n = int(inst.sizes[I])
    rng = np.random.default_rng(5)
    R = rng.integers(-8, 9, size=(n, n)) + 1j * rng.integers(-8, 9, size=(n, n))
    A = np.tril(R, -1)
    A = A + A.T + np.diag(rng.integers(200, 260, size=n) * rng.choice([-1, 1], n)).astype(complex)
    k = n // 2
    A[k, :] = A[:, k] = A[k + 1, :] = A[:, k + 1] = 0
    A[k, k], A[k, k + 1], A[k + 1, k], A[k + 1, k + 1] = 12288, 12289, 12289, 12290
    A[k + 1, k + 2] = A[k + 2, k + 1] = 64
    assert np.linalg.cond(A) < 1e4
    inst.K[inst.offsets[I]:inst.offsets[I + 1]] = A.reshape(-1, order="F")
    ref = oracle.OraclePlan(inst.sizes, inst.pairs, order)
    assert ref.factor(inst.K.astype(np.complex64).astype(np.complex128)) < 0
    dref = np.diag(ref.block(I, I))
    assert abs(dref[k + 1] * 12288 + 1) <= 1e-6   # the cancellation costs FP64 ~8 digits too
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, tile=64)
    assert int(plan.order()[0]) == I
    K = torch.from_numpy(inst.K).cuda()
    B = torch.from_numpy(inst.B).cuda()
    st, err = {}, {}
    for mode in ("fallback", "plain", "pivot"):
        print(f"[case] integer block {mode}", flush=True)
        f = d3m.Factor(plan, d3m.C64_IR, nrhs_max=2, fallback=mode == "fallback", pivot=mode == "pivot",
                       max_iter=30)
        f.factorize(K)
        X = f.solve(B).cpu().numpy()
        st[mode] = f.status()
        if mode != "pivot":
            d = np.diag(f.block(I, I))
            err[mode] = (np.abs(d - dref) / np.abs(dref)).max()
        print(f"[case] {mode}: D error {err.get(mode)} status {st[mode]}", flush=True)
        assert st[mode]["status"] == 0, st[mode]
        assert oracle.backward_error(inst.sizes, inst.pairs, inst.K, X, inst.B).max() <= 1e-10
    assert st["fallback"]["fallbacks"] >= 1 and st["plain"]["fallbacks"] == 0
    assert err["fallback"] <= 1e-6, err   # FP64 elimination of exact entries, stored in complex64
    assert err["plain"] >= 0.5, err       # FP32 elimination: the pivot is wrong in its leading digit
    assert 10 * st["pivot"]["eta_hist"][0] <= min(st["fallback"]["eta_hist"][0], st["plain"]["eta_hist"][0]), st


@pytest.mark.parametrize("precision,tile", [(0, 16), (0, 0), (1, 32)])
def test_refactorize_with_a_new_K_matches_oracle(precision, tile):
    """A factor used again on a second K of the same structure: the fill-in
    blocks of L (not in K, stored by the first update of each of their tiles,
    not zeroed) must not keep anything of the first factorization."""
    d3m = _d3m()
    a = gen.make_instance((3, 3, 2), 40, gen.COEF_PLAIN, 2, 7)
    b = gen.make_instance((3, 3, 2), 40, gen.COEF_PLAIN, 2, 8)
    assert np.array_equal(a.sizes, b.sizes) and np.array_equal(a.pairs, b.pairs)
    print(f"[case] refactorize N={a.N} prec={precision} tile={tile}", flush=True)
    plan = d3m.Plan(a.sizes, a.pairs, grid=a.grid, tile=tile)
    assert plan.info["fill_blocks"] > 0
    f = d3m.Factor(plan, precision, nrhs_max=2)
    f.factorize(torch.from_numpy(a.K).cuda())
    f.factorize(torch.from_numpy(b.K).cuda())
    X = f.solve(torch.from_numpy(np.ascontiguousarray(b.B)).cuda()).cpu().numpy()
    st = f.status()
    assert st["status"] == 0, st
    order = oracle.nd_order(b.grid)
    _, Xo = _oracle_solution(b, order, b.B)
    eta = oracle.backward_error(b.sizes, b.pairs, b.K, X, b.B)
    assert eta.max() <= (1e-12 if precision == 0 else 1e-10)
    assert _fwd_err(X, Xo) <= (1e-10 if precision == 0 else 1e-8)
