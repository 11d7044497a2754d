"""Seeded synthetic reduced matrices K for the dual block-LDL^T step of D3M.

This module builds *inputs* only: the domain grid, the interfaces between
face-adjacent domains, the block pattern of K (block (I,J) is nonzero when
interfaces I and J border a common domain, Sec. II and Fig. 1(b) of the
paper), the interface sizes and the random values of K, B and C.  It holds
none of the method's arithmetic (no ordering, fill, factorization or solve):
both the CPU reference solver of the tests and the GPU library receive what
it returns and compute everything else on their own.

Recipe (the paper's experiment, Sec. III, used a FEM-reduced K that is not
available; these synthetic matrices stand in for it):

* Interfaces are enumerated axis 0 first, then axis 1, then axis 2; within
  an axis the lower domain's coordinates run lexicographically (x slowest,
  z fastest).  Interface (ax, d) separates domain d and d + e_ax.
* Diagonal block K_II: upper triangle (with diagonal) iid CN(0,1), mirrored
  bitwise, plus a diagonal of s_k * coef * sqrt(n_I) with iid fair signs s_k.
* Off-diagonal stored block K_IJ (I > J): iid CN(0,1) / sqrt(max(n_I, n_J)).
* CN(0,1) = (N(0,1) + i N(0,1)) / sqrt(2).
* Draw order: sizes, then per interface (upper triangle re, im, then signs),
  then per pair in (J, I) lexicographic order (re, im), then B, then C.

K layout (one flat complex128 buffer, column-major blocks): the full
n_I x n_I diagonal block of every interface I in interface order, then the
n_I x n_J block K_IJ of every pair (I, J), I > J, in pair order.  K_JI =
K_IJ^T is implied, so K = K^T exactly.  Right-hand sides are stored as
(nrhs, N) arrays: each RHS vector is contiguous (an N x nrhs column-major
matrix).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

COEF_PLAIN = complex(3.0, 0.5)
COEF_PRECISION = 2.0 * COEF_PLAIN / abs(COEF_PLAIN)


def grid_interfaces(grid: Sequence[int]) -> np.ndarray:
    """Interfaces of a domain grid as rows (axis, x, y, z) of the lower domain."""
    a, b, c = (int(g) for g in grid)
    out = []
    for ax in range(3):
        for x in range(a):
            for y in range(b):
                for z in range(c):
                    d = [x, y, z]
                    d[ax] += 1
                    if d[0] < a and d[1] < b and d[2] < c:
                        out.append((ax, x, y, z))
    return np.asarray(out, dtype=np.int32).reshape(-1, 4)


def grid_pairs(grid: Sequence[int], ifaces: Optional[np.ndarray] = None) -> np.ndarray:
    """Pairs (I, J), I > J, of interfaces that border a common domain.

    Sorted by (J, I).  This is the nonzero block pattern of K off the diagonal.
    """
    if ifaces is None:
        ifaces = grid_interfaces(grid)
    a, b, c = (int(g) for g in grid)
    touching = {}
    for i, (ax, x, y, z) in enumerate(ifaces.tolist()):
        lo = (x, y, z)
        hi = [x, y, z]
        hi[ax] += 1
        for dom in (lo, tuple(hi)):
            touching.setdefault(dom, []).append(i)
    pairs = set()
    for lst in touching.values():
        for p in range(len(lst)):
            for q in range(p + 1, len(lst)):
                i, j = lst[p], lst[q]
                pairs.add((max(i, j), min(i, j)))
    pairs = sorted(pairs, key=lambda t: (t[1], t[0]))
    return np.asarray(pairs, dtype=np.int32).reshape(-1, 2)


def k_offsets(sizes: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """Offsets (in complex elements) of every block in the flat K layout."""
    sizes = np.asarray(sizes, dtype=np.int64)
    lens = [int(n) * int(n) for n in sizes]
    lens += [int(sizes[i]) * int(sizes[j]) for i, j in np.asarray(pairs).tolist()]
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    return off


def _cn(rng: np.random.Generator, shape) -> np.ndarray:
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * (1.0 / math.sqrt(2.0))


@dataclasses.dataclass
class Instance:
    grid: tuple
    ifaces: np.ndarray      # (nb, 4) int32
    sizes: np.ndarray       # (nb,) int32
    pairs: np.ndarray       # (npair, 2) int32, I > J
    offsets: np.ndarray     # (nb + npair + 1,) int64
    K: np.ndarray           # flat complex128
    B: np.ndarray           # (nrhs, N) complex128
    C: Optional[np.ndarray]  # (nrhs, N) complex128 or None
    coef: complex
    seed: object

    @property
    def nb(self) -> int:
        return int(self.sizes.shape[0])

    @property
    def N(self) -> int:
        return int(self.sizes.sum())

    @property
    def row_offsets(self) -> np.ndarray:
        o = np.zeros(self.nb + 1, dtype=np.int64)
        o[1:] = np.cumsum(self.sizes.astype(np.int64))
        return o

    def diag_block(self, i: int) -> np.ndarray:
        n = int(self.sizes[i])
        o = int(self.offsets[i])
        return self.K[o:o + n * n].reshape(n, n, order="F")

    def pair_block(self, k: int) -> np.ndarray:
        i, j = (int(v) for v in self.pairs[k])
        o = int(self.offsets[self.nb + k])
        return self.K[o:o + int(self.sizes[i]) * int(self.sizes[j])].reshape(
            int(self.sizes[i]), int(self.sizes[j]), order="F")


def make_instance(grid: Sequence[int], size_range, coef: complex, nrhs: int,
                  seed, with_c: bool = False, rng: Optional[np.random.Generator] = None
                  ) -> Instance:
    """Build one seeded instance.

    size_range: an int (all interfaces that size) or (lo, hi) inclusive.
    seed: an int or a numpy SeedSequence; ignored when rng is given.
    """
    grid = tuple(int(g) for g in grid)
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    ifaces = grid_interfaces(grid)
    nb = ifaces.shape[0]
    if isinstance(size_range, (int, np.integer)):
        sizes = np.full(nb, int(size_range), dtype=np.int32)
    else:
        lo, hi = size_range
        sizes = rng.integers(int(lo), int(hi) + 1, size=nb).astype(np.int32)
    pairs = grid_pairs(grid, ifaces)
    off = k_offsets(sizes, pairs)
    K = np.empty(int(off[-1]), dtype=np.complex128)
    for i in range(nb):
        n = int(sizes[i])
        iu, ju = np.triu_indices(n)
        vals = _cn(rng, iu.shape[0])
        blk = np.empty((n, n), dtype=np.complex128)
        blk[iu, ju] = vals
        blk[ju, iu] = vals
        signs = rng.integers(0, 2, size=n) * 2 - 1
        blk[np.arange(n), np.arange(n)] += signs * coef * math.sqrt(n)
        K[off[i]:off[i + 1]] = blk.reshape(-1, order="F")
    for k, (i, j) in enumerate(pairs.tolist()):
        ni, nj = int(sizes[i]), int(sizes[j])
        blk = _cn(rng, (ni, nj)) * (1.0 / math.sqrt(max(ni, nj)))
        K[off[nb + k]:off[nb + k + 1]] = blk.reshape(-1, order="F")
    N = int(sizes.sum())
    B = _cn(rng, (nrhs, N))
    C = _cn(rng, (nrhs, N)) if with_c else None
    return Instance(grid, ifaces, sizes, pairs, off, K, B, C, complex(coef), seed)


def subinstance(inst: Instance, keep: Sequence[int]) -> Instance:
    """Principal submatrix of K on the interfaces `keep` (renumbered in the
    given order), with the matching rows of B and C."""
    keep = [int(k) for k in keep]
    new_id = {old: new for new, old in enumerate(keep)}
    sizes = inst.sizes[keep].copy()
    pairs_new, src = [], []
    for k, (i, j) in enumerate(inst.pairs.tolist()):
        if i in new_id and j in new_id:
            a, b = new_id[i], new_id[j]
            pairs_new.append((a, b) if a > b else (b, a))
            src.append((k, a > b))
    order = sorted(range(len(pairs_new)), key=lambda t: (pairs_new[t][1], pairs_new[t][0]))
    pairs = np.asarray([pairs_new[t] for t in order], dtype=np.int32).reshape(-1, 2)
    src = [src[t] for t in order]
    off = k_offsets(sizes, pairs)
    nb = len(keep)
    K = np.empty(int(off[-1]), dtype=np.complex128)
    for a, old in enumerate(keep):
        K[off[a]:off[a + 1]] = inst.diag_block(old).reshape(-1, order="F")
    for k, (sk, same) in enumerate(src):
        blk = inst.pair_block(sk)
        if not same:
            blk = blk.T
        K[off[nb + k]:off[nb + k + 1]] = blk.reshape(-1, order="F")
    ro = inst.row_offsets
    rows = np.concatenate([np.arange(ro[o], ro[o + 1]) for o in keep])
    B = inst.B[:, rows].copy()
    C = inst.C[:, rows].copy() if inst.C is not None else None
    return Instance(inst.grid, inst.ifaces[keep].copy(), sizes, pairs, off, K, B, C,
                    inst.coef, inst.seed)


def box_interfaces(inst_or_ifaces, lo: Sequence[int], hi: Sequence[int]) -> list:
    """Interfaces whose two domains both lie in the box [lo, hi)."""
    ifaces = inst_or_ifaces.ifaces if isinstance(inst_or_ifaces, Instance) else inst_or_ifaces
    out = []
    for i, (ax, x, y, z) in enumerate(np.asarray(ifaces).tolist()):
        d0 = [x, y, z]
        d1 = [x, y, z]
        d1[ax] += 1
        if all(lo[t] <= d0[t] < hi[t] and lo[t] <= d1[t] < hi[t] for t in range(3)):
            out.append(i)
    return out


# The workloads: the paper's reduced matrices are replaced by these recipes.
def config_tiny(nrhs: int = 1, with_c: bool = False) -> Instance:
    """2x2 grid, 4 interfaces of 48 unknowns (the paper's four-domain example)."""
    return make_instance((2, 2, 1), 48, COEF_PLAIN, nrhs, 0, with_c)


def config_fp64(nrhs: int = 1, with_c: bool = False) -> Instance:
    """8x8x1 grid, 112 interfaces, n ~ U{200..400} (about 33k unknowns)."""
    return make_instance((8, 8, 1), (200, 400), COEF_PLAIN, nrhs, 1, with_c)


def config_precision(nrhs: int = 64, with_c: bool = False) -> Instance:
    """4x4x4 grid, 144 interfaces, n ~ U{300..600} (about 65k unknowns)."""
    return make_instance((4, 4, 4), (300, 600), COEF_PRECISION, nrhs, 2, with_c)


BATCH_GRIDS = ((2, 2, 2), (3, 3, 2), (4, 4, 2))


def config_batch(count: int = 32, nrhs: int = 16, size_range=(100, 500), indices=None) -> list:
    """Frequency sweep: instance k has f_k = 0.5 + 1.5 k/31 and a grid drawn
    uniformly from BATCH_GRIDS.  indices: build only these instances of the
    32 (else the first count)."""
    seqs = np.random.SeedSequence(3).spawn(32)
    out = []
    for k in (range(count) if indices is None else [int(i) for i in indices]):
        rng = np.random.Generator(np.random.PCG64(seqs[k]))
        g = BATCH_GRIDS[int(rng.integers(0, len(BATCH_GRIDS)))]
        f = 0.5 + 1.5 * k / 31.0
        out.append(make_instance(g, size_range, f * COEF_PLAIN, nrhs, seqs[k], rng=rng))
    return out


def config_diff(nrhs: int = 128, grid=(6, 6, 6), size_range=(300, 700)) -> Instance:
    """6x6x6 grid, 540 interfaces, n ~ U{300..700} (about 270k unknowns)."""
    return make_instance(grid, size_range, COEF_PLAIN, nrhs, 4, with_c=True)


# ---------------------------------------------------------------- primal (domain) matrices
def grid_domains(grid: Sequence[int]) -> np.ndarray:
    """Domains of the grid, lexicographic (x slowest)."""
    a, b, c = (int(g) for g in grid)
    return np.asarray([(x, y, z) for x in range(a) for y in range(b) for z in range(c)], dtype=np.int32)


def domain_interfaces(grid: Sequence[int], ifaces: Optional[np.ndarray] = None) -> list:
    """For each domain, the interfaces on its faces (increasing ids)."""
    if ifaces is None:
        ifaces = grid_interfaces(grid)
    doms = grid_domains(grid)
    index = {tuple(d): k for k, d in enumerate(doms.tolist())}
    out = [[] for _ in range(len(doms))]
    for i, (ax, x, y, z) in enumerate(np.asarray(ifaces).tolist()):
        d0 = [x, y, z]
        d1 = [x, y, z]
        d1[ax] += 1
        out[index[tuple(d0)]].append(i)
        out[index[tuple(d1)]].append(i)
    return [sorted(v) for v in out]


@dataclasses.dataclass
class PrimalInstance:
    """A synthetic primal (FEM-like) matrix in block form: blocks 0..nb-1
    are the interfaces, block nb + d the interior unknowns of domain d.  K
    uses the library's K layout over all blocks (pairs: the interface pairs
    first, as grid_pairs gives them, then (nb + d, I) for each domain d and
    interface I on its faces).  F: right-hand sides; M: port modes (one
    column per port, unit-norm, on the interior unknowns of one domain)."""
    grid: tuple
    nb: int                 # interfaces (the reduced blocks)
    ndom: int
    sizes: np.ndarray       # (nb + ndom,) int32
    pairs: np.ndarray       # (npair, 2) int32, first npair_red between interfaces
    npair_red: int
    offsets: np.ndarray
    K: np.ndarray
    F: np.ndarray           # (nrhs, N)
    M: np.ndarray           # (nports, N)
    port_domain: list
    dom_ifaces: list

    @property
    def N(self) -> int:
        return int(self.sizes.astype(np.int64).sum())

    @property
    def row_offsets(self) -> np.ndarray:
        o = np.zeros(self.sizes.shape[0] + 1, dtype=np.int64)
        o[1:] = np.cumsum(self.sizes.astype(np.int64))
        return o


def make_primal_instance(grid: Sequence[int], iface_range, interior_range, coef: complex, nrhs: int, seed,
                         nports: int = 4) -> PrimalInstance:
    """Synthetic primal matrix.  Interface diagonal blocks and the couplings
    between interfaces of one domain follow the reduced-matrix recipe (they
    stand for the assembled interface parts of the two domain matrices);
    each domain's interior block is symmetric complex normal plus the
    diagonal shift s_k coef sqrt(n_d) (the regularized domain matrix), and
    its coupling to each face interface is complex normal / sqrt(max(n_d,
    n_I)).  Draw order: interface sizes, interior sizes, interface blocks,
    interface pairs, interior blocks, interior-interface blocks, F, M."""
    grid = tuple(int(g) for g in grid)
    rng = np.random.Generator(np.random.PCG64(seed))
    ifaces = grid_interfaces(grid)
    nb = ifaces.shape[0]
    doms = grid_domains(grid)
    ndom = doms.shape[0]
    def draw_sizes(rng_, r, count):
        if isinstance(r, (int, np.integer)):
            return np.full(count, int(r), dtype=np.int32)
        return rng_.integers(int(r[0]), int(r[1]) + 1, size=count).astype(np.int32)
    s_if = draw_sizes(rng, iface_range, nb)
    s_in = draw_sizes(rng, interior_range, ndom)
    sizes = np.concatenate([s_if, s_in]).astype(np.int32)
    dif = domain_interfaces(grid, ifaces)
    red_pairs = grid_pairs(grid, ifaces)
    dom_pairs = [(nb + d, I) for d in range(ndom) for I in dif[d]]
    pairs = np.concatenate([red_pairs, np.asarray(dom_pairs, dtype=np.int32).reshape(-1, 2)]).astype(np.int32)
    off = k_offsets(sizes, pairs)
    K = np.empty(int(off[-1]), dtype=np.complex128)

    def sym_block(n):
        iu, ju = np.triu_indices(n)
        vals = _cn(rng, iu.shape[0])
        blk = np.empty((n, n), dtype=np.complex128)
        blk[iu, ju] = vals
        blk[ju, iu] = vals
        signs = rng.integers(0, 2, size=n) * 2 - 1
        blk[np.arange(n), np.arange(n)] += signs * coef * math.sqrt(n)
        return blk

    for i in range(nb):
        K[off[i]:off[i + 1]] = sym_block(int(sizes[i])).reshape(-1, order="F")
    npr = red_pairs.shape[0]
    for k in range(npr):
        i, j = (int(v) for v in pairs[k])
        ni, nj = int(sizes[i]), int(sizes[j])
        K[off[nb + ndom + k]:off[nb + ndom + k + 1]] = (
            _cn(rng, (ni, nj)) * (1.0 / math.sqrt(max(ni, nj)))).reshape(-1, order="F")
    for d in range(ndom):
        i = nb + d
        K[off[i]:off[i + 1]] = sym_block(int(sizes[i])).reshape(-1, order="F")
    for k in range(npr, pairs.shape[0]):
        i, j = (int(v) for v in pairs[k])
        ni, nj = int(sizes[i]), int(sizes[j])
        K[off[nb + ndom + k]:off[nb + ndom + k + 1]] = (
            _cn(rng, (ni, nj)) * (1.0 / math.sqrt(max(ni, nj)))).reshape(-1, order="F")
    N = int(sizes.astype(np.int64).sum())
    F = _cn(rng, (nrhs, N))
    row0 = np.concatenate([[0], np.cumsum(sizes.astype(np.int64))])
    # ports on the interiors of domains on the grid's x = 0 face, in turn
    face = [d for d in range(ndom) if doms[d][0] == 0]
    M = np.zeros((nports, N), dtype=np.complex128)
    pdom = []
    for q in range(nports):
        d = face[q % len(face)]
        n = int(sizes[nb + d])
        v = _cn(rng, n)
        M[q, row0[nb + d]:row0[nb + d + 1]] = v / np.linalg.norm(v)
        pdom.append(d)
    return PrimalInstance(grid, nb, ndom, sizes, pairs, int(npr), off, K, F, M, pdom, dif)


def config_primal(nrhs: int = 16, grid=(4, 4, 4), iface_range=(300, 600), interior_range=(300, 600),
                  nports: int = 8) -> PrimalInstance:
    """The primal reduction and recovery around the precision workload's
    grid: 4x4x4 domains, interfaces of n ~ U{300..600} and interiors of
    n ~ U{300..600} unknowns, coefficient 3 + 0.5j, 16 right-hand sides, 8
    ports on the x = 0 face."""
    return make_primal_instance(grid, iface_range, interior_range, COEF_PLAIN, nrhs, 5, nports)
