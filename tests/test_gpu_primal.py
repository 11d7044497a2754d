"""GPU: primal reduction (d3m_reduce) and recovery (d3m_recover) against the
oracle's plain definitions (per-domain Schur complements onto the
interfaces, the reduced right-hand sides, the interior back-substitution
and the port projections), with the reduced system solved by the library
itself, in FP64 and complex64 + FP64 refinement."""
import numpy as np
import pytest

import oracle
from oracle import primal
from paper_2002_05026_amd import instances as gen
from tests.test_library_host import _primal_plan

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _d3m():
    import paper_2002_05026_amd as d3m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert d3m.device_ok(), "libd3m.so has no usable gfx950 device"
    return d3m


@pytest.mark.parametrize("grid,ir,nr,tile", [((2, 2, 1), (20, 70), (30, 90), 32), ((2, 2, 2), (60, 200), (80, 260), 0),
                                             ((3, 3, 2), (40, 130), (100, 300), 64)])
def test_reduce_and_recover_match_the_oracle(grid, ir, nr, tile):
    d3m = _d3m()
    inst = gen.make_primal_instance(grid, ir, nr, gen.COEF_PLAIN, 3, 900 + ir[0], nports=3)
    print(f"[case] primal grid={grid} N={inst.N} tile={tile}", flush=True)
    plan, red = _primal_plan(inst, tile=tile)
    A = torch.from_numpy(inst.K).cuda()
    F = torch.from_numpy(inst.F).cuda()
    f = d3m.Factor(plan, d3m.C128, nrhs_max=3)
    Kred, G = f.reduce(A, F)
    assert f.status()["status"] == 0
    Ko, Go = primal.reduce(inst)
    Kg = Kred.cpu().numpy()
    assert np.abs(Kg - Ko).max() <= 1e-12 * np.abs(Ko).max()
    assert np.abs(G.cpu().numpy() - Go).max() <= 1e-12 * np.abs(Go).max()
    sizes, pairs, off = primal.reduced_layout(inst)
    p = oracle.OraclePlan(sizes, pairs, oracle.nd_order(grid))
    assert p.factor(Ko) == -1
    Uo = primal.recover(inst, p.solve(Go))
    So = primal.ports(inst, Uo)
    M = torch.from_numpy(inst.M).cuda()
    for prec in (d3m.C128, d3m.C64_IR):
        g = d3m.Factor(red, prec, nrhs_max=3, tol=1e-12 if prec == d3m.C64_IR else 1e-10)
        g.factorize(Kred)
        Xred = g.solve(G)
        assert g.status()["status"] == 0
        if prec == d3m.C64_IR:  # the forward part's z is used up by recover: reduce again
            f.reduce(A, F)
        U, S = f.recover(Xred, M)
        U = U.cpu().numpy()
        err = (np.linalg.norm(U - Uo, axis=1) / np.linalg.norm(Uo, axis=1)).max()
        assert err <= 1e-10, (prec, err)
        assert np.abs(S.cpu().numpy() - So).max() <= 1e-10 * np.abs(So).max()


def test_reduce_requires_its_order():
    d3m = _d3m()
    inst = gen.make_primal_instance((2, 2, 1), 8, 9, gen.COEF_PLAIN, 1, 11)
    plan, red = _primal_plan(inst)
    f = d3m.Factor(plan, d3m.C128, nrhs_max=1)
    A = torch.from_numpy(inst.K).cuda()
    with pytest.raises(d3m.D3MError):
        f.factorize(A)  # a partial plan factors through d3m_reduce only
    Xred = torch.zeros((1, int(inst.sizes[:inst.nb].sum())), dtype=torch.complex128, device="cuda")
    with pytest.raises(d3m.D3MError):
        f.recover(Xred)  # no reduction with right-hand sides yet
