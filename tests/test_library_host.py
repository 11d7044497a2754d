"""Host-side checks of the library (no GPU): exported C ABI, analysis
numbers against closed forms and the oracle's independent symbolic code,
the static race check of the task DAGs, and argument errors."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2002_05026_amd as d3m
from paper_2002_05026_amd import instances as gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "d3m.h")).read()
    names = set(re.findall(r"^(?:d3m_status|void|const char\*|int32_t)\s+(d3m_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 20
    lib = ctypes.CDLL(d3m.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(d3m.SIGNATURES) == names


@pytest.mark.parametrize("g,n", [((2, 2, 1), 48), ((8, 8, 1), 300), ((4, 4, 4), 450), ((6, 6, 6), 500),
                                 ((2, 2, 2), 300), ((3, 3, 2), 300), ((4, 4, 2), 300)])
def test_analysis_matches_oracle_and_closed_forms(g, n):
    nb = gen.grid_interfaces(g).shape[0]
    sizes = np.full(nb, n)
    pairs = gen.grid_pairs(g)
    p = d3m.Plan(sizes, pairs, grid=g)
    o = oracle.OraclePlan(sizes, pairs, oracle.nd_order(g))
    s = o.stats()
    assert np.array_equal(p.order(), oracle.nd_order(g))
    for k in ("fill_blocks", "L_blocks", "nnz_L", "etree_height", "max_S"):
        assert p.info[k] == s[k], k
    assert p.info["flops_factor"] == pytest.approx(s["flops"], rel=1e-12)
    for I in range(0, nb, max(1, nb // 7)):
        assert p.struct(I) == o.struct(I)
    assert p.info["k_len"] == gen.k_offsets(sizes, pairs)[-1]


@pytest.mark.parametrize("g,lo,hi,tile", [((2, 2, 1), 48, 48, 16), ((2, 2, 2), 20, 70, 16), ((3, 3, 2), 5, 60, 16),
                                          ((4, 4, 2), 20, 90, 32), ((3, 3, 2), 100, 300, 64),
                                          # 144 interfaces: the top of the tree takes unmerged updates
                                          ((4, 4, 4), 5, 20, 16)])
def test_task_dags_are_race_free(g, lo, hi, tile):
    inst = gen.make_instance(g, (lo, hi), gen.COEF_PLAIN, 1, 9)
    for sched in (0, 1):
        p = d3m.Plan(inst.sizes, inst.pairs, grid=g, tile=tile, sched=sched)
        assert p.check() == 0


def test_tiles_are_near_equal_multiples_of_16():
    # one interface of each size; tiles must cover it exactly
    sizes = np.array([1, 17, 128, 129, 200, 300, 450, 600, 700])
    pairs = np.array([[i + 1, i] for i in range(len(sizes) - 1)])
    p = d3m.Plan(sizes, pairs, order=np.arange(len(sizes)), tile=128)
    assert p.info["ntiles"] == sum((int(n) + 127) // 128 for n in sizes)


def test_argument_errors():
    sizes = np.array([3, 4, 5])
    with pytest.raises(d3m.D3MError) as e:
        d3m.Plan(sizes, [[0, 1], [1, 0]])
    assert e.value.code == -2  # duplicate pair
    with pytest.raises(d3m.D3MError) as e:
        d3m.Plan(sizes, [[1, 1]])
    assert e.value.code == -2  # self pair
    with pytest.raises(d3m.D3MError) as e:
        d3m.Plan(sizes, [[0, 3]])
    assert e.value.code == -2  # out of range
    with pytest.raises(d3m.D3MError) as e:
        d3m.Plan(sizes, [[0, 1]], order=[0, 0, 1])
    assert e.value.code == -2  # not a permutation
    with pytest.raises(d3m.D3MError) as e:
        d3m.Plan(sizes, [[0, 1]], tile=40)
    assert e.value.code == -1  # tile not a multiple of 16
    with pytest.raises(d3m.D3MError) as e:
        d3m.Plan(np.array([3, 0]), [[0, 1]])
    assert e.value.code == -1  # empty interface
    with pytest.raises(d3m.D3MError) as e:
        d3m.Plan(sizes, [[0, 1]], grid=(2, 2, 1))
    assert e.value.code == -2  # grid does not match the interface count
    # workspace checks happen before any device access
    p = d3m.Plan(sizes, [[0, 1], [1, 2]])
    lib = d3m.lib()
    need = p.workspace_bytes(d3m.C128, 4)
    h = ctypes.c_void_p()
    r = lib.d3m_factor_bind(p._h, 0, ctypes.c_void_p(256), need - 1, 4, None, ctypes.byref(h))
    assert r == -3
    r = lib.d3m_factor_bind(p._h, 0, ctypes.c_void_p(257), need, 4, None, ctypes.byref(h))
    assert r == -3
    r = lib.d3m_factor_bind(p._h, 0, ctypes.c_void_p(256), need, 129, None, ctypes.byref(h))
    assert r == -1  # nrhs above the maximum
    assert lib.d3m_status_string(3) == b"iterative refinement did not converge"


def test_minimum_degree_order_without_grid():
    inst = gen.make_instance((3, 3, 2), 10, gen.COEF_PLAIN, 1, 1)
    p = d3m.Plan(inst.sizes, inst.pairs)
    order = p.order()
    assert sorted(order.tolist()) == list(range(inst.nb))
    # the oracle's symbolic code on the same order gives the same fill
    o = oracle.OraclePlan(inst.sizes, inst.pairs, order)
    assert o.stats()["fill_blocks"] == p.info["fill_blocks"]


def test_batch_merge_keeps_every_task():
    insts = gen.config_batch(count=3, nrhs=1, size_range=(20, 40))
    plans = [d3m.Plan(i.sizes, i.pairs, grid=i.grid, tile=32) for i in insts]
    assert all(pl.info["ntask_factor"] > 0 for pl in plans)


def _primal_plan(inst, tile=32, **kw):
    """A partial-elimination plan of a primal instance: the domains' interior
    blocks first, then the interfaces in the library's nested-dissection
    order of the reduced matrix."""
    red = d3m.Plan(inst.sizes[:inst.nb], inst.pairs[:inst.npair_red], grid=inst.grid)
    order = [inst.nb + d for d in range(inst.ndom)] + red.order().tolist()
    return d3m.Plan(inst.sizes, inst.pairs, order=order, tile=tile, nelim=inst.ndom, **kw), red


@pytest.mark.parametrize("grid", [(2, 2, 1), (2, 2, 2), (3, 2, 2)])
def test_partial_elimination_plans(grid):
    inst = gen.make_primal_instance(grid, (20, 70), (30, 90), gen.COEF_PLAIN, 1, 7)
    plan, red = _primal_plan(inst)
    # the factor, forward and backward solve DAGs are race-free
    assert plan.check() == 0
    # factor work: only the interior blocks are eliminated
    n_in = inst.sizes[inst.nb:].astype(float)
    assert plan.info["flops_diag"] == pytest.approx((4.0 / 3.0 * n_in ** 3).sum(), rel=1e-12)
    fl_trsm = sum(4.0 * inst.sizes[I] * n_in[d] ** 2 for d in range(inst.ndom) for I in inst.dom_ifaces[d])
    assert plan.info["flops_trsm"] == pytest.approx(fl_trsm, rel=1e-12)


def test_partial_elimination_argument_errors():
    inst = gen.make_primal_instance((2, 2, 1), 8, 9, gen.COEF_PLAIN, 1, 8)
    red = d3m.Plan(inst.sizes[:inst.nb], inst.pairs[:inst.npair_red], grid=inst.grid)
    order = [inst.nb + d for d in range(inst.ndom)] + red.order().tolist()
    # the blocks left must be user ids 0..nred-1
    bad = list(reversed(order))
    with pytest.raises(d3m.D3MError) as e:
        d3m.Plan(inst.sizes, inst.pairs, order=bad, nelim=inst.ndom)
    assert e.value.code == -2
    # the pairs between the blocks left must come first
    pairs = np.concatenate([inst.pairs[inst.npair_red:], inst.pairs[:inst.npair_red]])
    with pytest.raises(d3m.D3MError):
        d3m.Plan(inst.sizes, pairs, order=order, nelim=inst.ndom)
    # a missing interface pair would be filled by the elimination
    pairs = np.concatenate([inst.pairs[1:inst.npair_red], inst.pairs[inst.npair_red:]])
    with pytest.raises(d3m.D3MError):
        d3m.Plan(inst.sizes, pairs, order=order, nelim=inst.ndom)
    with pytest.raises(d3m.D3MError):
        d3m.Plan(inst.sizes, inst.pairs, order=order, nelim=inst.nb + inst.ndom)


@pytest.mark.parametrize("solve_tile,merge,groups", [(32, 1, 2), (128, 4, 4), (64, 16, 2), (16, 8, 8)])
def test_tuning_knobs_keep_the_dags_race_free(solve_tile, merge, groups):
    inst = gen.make_instance((3, 2, 2), (20, 90), gen.COEF_PLAIN, 1, 55)
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, tile=32, solve_tile=solve_tile, merge=merge,
                    rhs_groups=groups)
    assert plan.check() == 0
    with pytest.raises(d3m.D3MError):
        d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, solve_tile=24)
    with pytest.raises(d3m.D3MError):
        d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, merge=17)
