"""The gradient conventions, pinned on the CPU against torch's own autograd
through a dense assembly (a library routine), with the oracle's holomorphic
block gradient as input: the stored-entry weights that d3m_adjoint applies
with d3m_options.dk_stored (strict lower of a diagonal block x2, its
diagonal x1, its upper triangle 0, off-diagonal blocks x2), and the
conjugation the torch wrapper applies."""
import numpy as np
import pytest
import torch

import oracle
from paper_2002_05026_amd import instances as gen


def stored_entry_grad(sizes, pairs, dK):
    """The stored-entry gradient from the symmetric block gradient (the rule
    d3m_adjoint follows with dk_stored), written out in numpy."""
    out = np.array(dK, copy=True)
    o = 0
    for n in [int(s) for s in sizes]:
        blk = out[o:o + n * n].reshape(n, n, order="F")
        w = 2.0 * np.tril(np.ones((n, n)), -1) + np.eye(n)
        out[o:o + n * n] = (blk * w).reshape(-1, order="F")
        o += n * n
    out[o:] *= 2.0
    return out


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
    gK = np.conj(stored_entry_grad(inst.sizes, inst.pairs, dK))
    gB = np.conj(Lam)
    assert np.abs(B.grad.numpy() - gB).max() <= 1e-12 * np.abs(gB).max()
    assert np.abs(K.grad.numpy() - gK).max() <= 1e-12 * np.abs(gK).max()
