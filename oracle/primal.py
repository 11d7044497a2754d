"""Plain definitions of the two steps around the dual factorization and
solution in D3M (Sec. II): the primal reduction and the primal recovery.

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU leg.

The primal matrix A is given in block form (see make_primal_instance of the
input generator): blocks 0..nb-1 are the interfaces, block nb + d the
interior unknowns of domain d, which couple only to the interfaces on d's
faces.  With Gamma the interface unknowns and i the interior ones:

* reduction (per domain: factor the regularized interior block, map its
  interfaces to its Dirichlet-to-Neumann contribution, assemble):
      K = A_GG - sum_d A_Gd A_dd^-1 A_dG,   g = f_G - sum_d A_Gd A_dd^-1 f_d
  K is block-sparse on the interface pairs that share a domain;
* recovery (per domain, once u_G = K^-1 g is known):
      u_d = A_dd^-1 (f_d - A_dG u_G);
* ports: S_pq = m_p^T u_q (bilinear), the projection of the solution for
  right-hand side q on the mode of port p.

Each dense solve uses numpy.linalg.solve (a library routine) on one
domain's interior block; nothing is blocked or reordered beyond that.
"""
from __future__ import annotations

import numpy as np


def _k_offsets(sizes, pairs):
    sizes = np.asarray(sizes, dtype=np.int64)
    nb = sizes.shape[0]
    off = np.zeros(nb + len(pairs) + 1, dtype=np.int64)
    for i in range(nb):
        off[i + 1] = off[i] + sizes[i] * sizes[i]
    for k, (i, j) in enumerate(np.asarray(pairs).reshape(-1, 2).tolist()):
        off[nb + k + 1] = off[nb + k] + sizes[i] * sizes[j]
    return off


def _diag(inst, i):
    n = int(inst.sizes[i])
    o = int(inst.offsets[i])
    low = np.tril(inst.K[o:o + n * n].reshape(n, n, order="F"))
    return low + np.tril(low, -1).T


def _pair(inst, k):
    i, j = (int(v) for v in inst.pairs[k])
    nblk = inst.sizes.shape[0]
    o = int(inst.offsets[nblk + k])
    return inst.K[o:o + int(inst.sizes[i]) * int(inst.sizes[j])].reshape(
        int(inst.sizes[i]), int(inst.sizes[j]), order="F")


def _interior_coupling(inst):
    """(d, I) -> A_dI (n_d x n_I) for the interfaces I of domain d."""
    out = {}
    for k in range(inst.npair_red, inst.pairs.shape[0]):
        a, b = (int(v) for v in inst.pairs[k])
        out[(a - inst.nb, b)] = _pair(inst, k)
    return out


def reduced_layout(inst):
    """Sizes, pairs and K offsets of the reduced matrix (the interfaces)."""
    sizes = inst.sizes[:inst.nb].copy()
    pairs = inst.pairs[:inst.npair_red].copy()
    return sizes, pairs, _k_offsets(sizes, pairs)


def reduce(inst):
    """The reduced matrix K (flat, in the library's K layout over the
    interfaces) and the reduced right-hand sides g (nrhs x N_G)."""
    nb = inst.nb
    sizes, pairs, off = reduced_layout(inst)
    row0 = inst.row_offsets
    blocks = {}
    for I in range(nb):
        blocks[(I, I)] = _diag(inst, I).copy()
    for k in range(inst.npair_red):
        I, J = (int(v) for v in inst.pairs[k])
        blocks[(I, J)] = _pair(inst, k).copy()
    C = _interior_coupling(inst)
    NG = int(row0[nb])
    G = np.array(inst.F[:, :NG], copy=True)
    for d in range(inst.ndom):
        Add = _diag(inst, nb + d)
        Gam = inst.dom_ifaces[d]
        Y = {J: np.linalg.solve(Add, C[(d, J)]) for J in Gam}   # A_dd^-1 A_dJ
        fd = inst.F[:, row0[nb + d]:row0[nb + d + 1]]
        z = np.linalg.solve(Add, fd.T)                         # A_dd^-1 f_d
        for I in Gam:
            for J in Gam:
                if I >= J:
                    blocks[(I, J)] -= C[(d, I)].T @ Y[J]
            G[:, row0[I]:row0[I + 1]] -= (C[(d, I)].T @ z).T
    K = np.empty(int(off[-1]), dtype=np.complex128)
    for I in range(nb):
        K[off[I]:off[I + 1]] = blocks[(I, I)].reshape(-1, order="F")
    for k, (I, J) in enumerate(pairs.tolist()):
        K[off[nb + k]:off[nb + k + 1]] = blocks[(I, J)].reshape(-1, order="F")
    return K, G


def recover(inst, XG):
    """The full primal solution U (nrhs x N) from the interface solution XG."""
    nb = inst.nb
    row0 = inst.row_offsets
    XG = np.atleast_2d(XG)
    U = np.zeros((XG.shape[0], inst.N), dtype=np.complex128)
    U[:, :row0[nb]] = XG
    C = _interior_coupling(inst)
    for d in range(inst.ndom):
        Add = _diag(inst, nb + d)
        r = np.array(inst.F[:, row0[nb + d]:row0[nb + d + 1]], copy=True)
        for I in inst.dom_ifaces[d]:
            r -= (C[(d, I)] @ XG[:, row0[I]:row0[I + 1]].T).T
        U[:, row0[nb + d]:row0[nb + d + 1]] = np.linalg.solve(Add, r.T).T
    return U


def ports(inst, U):
    """S (nports x nrhs), S_pq = m_p^T u_q."""
    return inst.M @ np.atleast_2d(U).T
