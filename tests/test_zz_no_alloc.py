"""GPU: the allocation-free bind (d3m_factor_bind_static) through the C ABI
against the ordinary bind on a caller workspace, on two binds in a row (the
second plan smaller than the first): the same kernels on the same plan give
bitwise equal factors and solutions, and the earlier static factor is
refused once the array holds another."""
import ctypes

import numpy as np
import pytest

from paper_2002_05026_amd import instances as gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _d3m():
    import paper_2002_05026_amd as d3m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert d3m.device_ok(), "libd3m.so has no usable gfx950 device"
    return d3m


def _solve_static(d3m, plan, prec, K, B):
    lib = d3m.lib()
    opts = d3m.Options(1e-10, 10, 0, 0.0, 0.0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    assert lib.d3m_factor_bind_static(plan._h, prec, B.shape[0], ctypes.byref(opts), ctypes.byref(h)) == 0
    s = d3m._stream()
    assert lib.d3m_factorize(h, d3m._ptr(K), s) == 0
    X = torch.empty_like(B)
    assert lib.d3m_solve(h, d3m._ptr(K), d3m._ptr(B), d3m._ptr(X), B.shape[0], B.stride(0), s) == 0
    ri = d3m.RunInfo()
    assert lib.d3m_status_sync(h, ctypes.byref(ri)) == 0
    return h, X.cpu().numpy(), ri


def _solve_ws(d3m, plan, prec, K, B):
    f = d3m.Factor(plan, prec, nrhs_max=B.shape[0])
    f.factorize(K)
    X = f.solve(B)
    st = f.status()
    assert st["status"] == 0, st
    return X.cpu().numpy(), st


@pytest.mark.parametrize("prec", [0, 1])
def test_static_bind_matches_workspace_bind_twice(prec):
    d3m = _d3m()
    lib = d3m.lib()
    big = gen.make_instance((2, 2, 2), (40, 120), gen.COEF_PLAIN, 3, 91)
    small = gen.config_tiny(nrhs=2)
    prev = None
    for inst in (big, small):
        print(f"[case] static bind N={inst.N} prec={prec}", flush=True)
        plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid, tile=32)
        assert plan.workspace_bytes(prec, inst.B.shape[0]) <= d3m.STATIC_WS_BYTES
        K = torch.from_numpy(inst.K).cuda()
        B = torch.from_numpy(inst.B).cuda()
        h, Xs, ri = _solve_static(d3m, plan, prec, K, B)
        Xw, st = _solve_ws(d3m, plan, prec, K, B)
        assert np.array_equal(Xs, Xw)
        assert ri.eta == st["eta"] and ri.ir_iters == st["ir_iters"]
        if prev is not None:
            # the first static factor's array now holds the second one
            ri2 = d3m.RunInfo()
            assert lib.d3m_status_sync(prev, ctypes.byref(ri2)) == -4  # D3M_ERR_STATE
            lib.d3m_factor_destroy(prev)
        prev = h
        keep_plan = plan  # noqa: F841 (the factor refers to its plan)
    lib.d3m_factor_destroy(prev)


def test_static_bind_rejects_a_plan_beyond_the_array():
    d3m = _d3m()
    inst = gen.make_instance((2, 2, 2), (300, 600), gen.COEF_PLAIN, 1, 92)
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid)
    assert plan.workspace_bytes(0, 1) > d3m.STATIC_WS_BYTES
    with pytest.raises(d3m.D3MError) as e:
        d3m.Factor(plan, 0, nrhs_max=1, static_ws=True)
    assert e.value.code == -3  # D3M_ERR_WORKSPACE
