"""The torch wrapper's gradient conventions, pinned on the CPU against
torch's own autograd through a dense assembly (a library routine), with the
oracle's holomorphic block gradient as input."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_05026_amd as d3m
from paper_2002_05026_amd import instances as gen
from paper_2002_05026_amd.autograd import flat_grad_from_dK


def _dense_torch(sizes, pairs, Kflat):
    """Differentiable dense assembly: diagonal blocks from their lower
    triangle, off-diagonal blocks mirrored."""
    sizes = [int(s) for s in sizes]
    r0 = np.concatenate([[0], np.cumsum(sizes)])
    N = int(r0[-1])
    rows = []
    o = 0
    blocks = {}
    for i, n in enumerate(sizes):
        B = Kflat[o:o + n * n].reshape(n, n).t()
        L = torch.tril(B)
        blocks[(i, i)] = L + torch.tril(B, -1).t()
        o += n * n
    for (i, j) in np.asarray(pairs).tolist():
        B = Kflat[o:o + sizes[i] * sizes[j]].reshape(sizes[j], sizes[i]).t()
        blocks[(i, j)] = B
        blocks[(j, i)] = B.t()
        o += sizes[i] * sizes[j]
    for i in range(len(sizes)):
        row = [blocks.get((i, j), torch.zeros(sizes[i], sizes[j], dtype=Kflat.dtype)) for j in range(len(sizes))]
        rows.append(torch.cat(row, dim=1))
    return torch.cat(rows, dim=0)


def test_wrapper_convention_matches_torch_autograd():
    inst = gen.make_instance((2, 2, 1), (5, 9), gen.COEF_PLAIN, 2, 77, with_c=True)
    K = torch.tensor(inst.K, requires_grad=True)
    B = torch.tensor(inst.B, requires_grad=True)
    C = torch.tensor(inst.C)
    A = _dense_torch(inst.sizes, inst.pairs, K)
    X = torch.linalg.solve(A, B.t()).t()
    J = torch.real((C * X).sum())
    J.backward()
    # holomorphic block gradient from the oracle
    p = oracle.OraclePlan(inst.sizes, inst.pairs, oracle.nd_order(inst.grid))
    assert p.factor(inst.K) == -1
    Xo = p.solve(inst.B)
    Lam = p.solve(inst.C)                    # G = conj(grad_X) = C for this J
    dK = oracle.grad_K(inst.sizes, inst.pairs, Lam, Xo, inst.K.shape[0])
    plan = d3m.Plan(inst.sizes, inst.pairs, grid=inst.grid)
    gK = torch.conj(flat_grad_from_dK(plan, torch.tensor(dK))).resolve_conj().numpy()
    gB = np.conj(Lam)
    assert np.abs(B.grad.numpy() - gB).max() <= 1e-12 * np.abs(gB).max()
    assert np.abs(K.grad.numpy() - gK).max() <= 1e-12 * np.abs(gK).max()
