"""Pins of the oracle's primal reduction and recovery against brute force:
the dense assembled primal matrix solved by Gaussian elimination, and the
Schur complement on all interface unknowns at once (one global dense
computation instead of the oracle's per-domain one)."""
import numpy as np
import pytest

import oracle
from oracle import primal
from paper_2002_05026_amd import instances as gen
from tests import dense_ref


def _inst(grid=(2, 2, 1), seed=1):
    return gen.make_primal_instance(grid, (5, 9), (6, 11), gen.COEF_PLAIN, 3, seed, nports=3)


@pytest.mark.parametrize("grid,seed", [((2, 2, 1), 1), ((2, 2, 2), 2), ((3, 2, 1), 3)])
def test_reduction_is_the_global_schur_complement(grid, seed):
    inst = _inst(grid, seed)
    A = dense_ref.dense_K(inst.sizes, inst.pairs, inst.K)
    NG = int(inst.row_offsets[inst.nb])
    S = A[:NG, :NG] - A[:NG, NG:] @ np.linalg.solve(A[NG:, NG:], A[NG:, :NG])
    g = inst.F[:, :NG] - (A[:NG, NG:] @ np.linalg.solve(A[NG:, NG:], inst.F[:, NG:].T)).T
    K, G = primal.reduce(inst)
    sizes, pairs, off = primal.reduced_layout(inst)
    Kd = dense_ref.dense_K(sizes, pairs, K)
    assert np.abs(Kd - S).max() <= 1e-13 * np.abs(S).max()
    assert np.abs(G - g).max() <= 1e-13 * np.abs(g).max()
    # the reduced pattern is the interfaces' (pairs sharing a domain), and K = K^T
    assert np.array_equal(pairs, gen.grid_pairs(grid))
    assert np.abs(S - S.T).max() <= 1e-13 * np.abs(S).max()


@pytest.mark.parametrize("grid,seed", [((2, 2, 1), 4), ((2, 2, 2), 5)])
def test_reduce_solve_recover_is_the_primal_solution(grid, seed):
    inst = _inst(grid, seed)
    A = dense_ref.dense_K(inst.sizes, inst.pairs, inst.K)
    Ud = np.linalg.solve(A, inst.F.T).T
    K, G = primal.reduce(inst)
    sizes, pairs, off = primal.reduced_layout(inst)
    p = oracle.OraclePlan(sizes, pairs, oracle.nd_order(grid))
    assert p.factor(K) == -1
    XG = p.solve(G)
    U = primal.recover(inst, XG)
    assert (np.linalg.norm(U - Ud, axis=1) / np.linalg.norm(Ud, axis=1)).max() <= 1e-12
    S = primal.ports(inst, U)
    assert np.abs(S - inst.M @ Ud.T).max() <= 1e-12 * np.abs(S).max()
    # each port lives on one domain's interior unknowns
    row0 = inst.row_offsets
    for q, d in enumerate(inst.port_domain):
        nz = np.nonzero(inst.M[q])[0]
        assert nz.min() >= row0[inst.nb + d] and nz.max() < row0[inst.nb + d + 1]
