"""Brute-force dense helpers for the tests (numpy only).

They assemble the block-sparse K of an instance into a dense matrix and run
textbook dense algorithms on it; they share nothing with the oracle or the
GPU library and serve as independent pins on tiny inputs.
"""
import numpy as np


def dense_K(sizes, pairs, K):
    sizes = np.asarray(sizes, dtype=np.int64)
    nb = sizes.shape[0]
    r0 = np.zeros(nb + 1, dtype=np.int64)
    r0[1:] = np.cumsum(sizes)
    N = int(r0[-1])
    A = np.zeros((N, N), dtype=np.complex128)
    o = 0
    for i in range(nb):
        n = int(sizes[i])
        blk = np.asarray(K[o:o + n * n]).reshape(n, n, order="F")
        low = np.tril(blk)
        A[r0[i]:r0[i + 1], r0[i]:r0[i + 1]] = low + np.tril(low, -1).T
        o += n * n
    for i, j in np.asarray(pairs).reshape(-1, 2).tolist():
        ni, nj = int(sizes[i]), int(sizes[j])
        blk = np.asarray(K[o:o + ni * nj]).reshape(ni, nj, order="F")
        A[r0[i]:r0[i + 1], r0[j]:r0[j + 1]] = blk
        A[r0[j]:r0[j + 1], r0[i]:r0[i + 1]] = blk.T
        o += ni * nj
    return A


def perm_rows(sizes, order):
    """Row permutation p such that (P K P^T) = K[p][:, p]."""
    sizes = np.asarray(sizes, dtype=np.int64)
    r0 = np.zeros(sizes.shape[0] + 1, dtype=np.int64)
    r0[1:] = np.cumsum(sizes)
    return np.concatenate([np.arange(r0[i], r0[i + 1]) for i in order])


def dense_ldlt_nopivot(A):
    """Textbook right-looking scalar LDL^T (transpose, no pivoting)."""
    A = np.array(A, dtype=np.complex128, copy=True)
    N = A.shape[0]
    L = np.eye(N, dtype=np.complex128)
    d = np.zeros(N, dtype=np.complex128)
    for k in range(N):
        d[k] = A[k, k]
        col = A[k + 1:, k].copy()
        L[k + 1:, k] = col / d[k]
        A[k + 1:, k + 1:] -= np.outer(col, col) / d[k]
    return L, d


def brute_fill(nb, pairs, order):
    """Boolean block elimination on a dense adjacency matrix.

    Returns the set of (later, earlier) block pairs of L (original + fill)."""
    adj = np.zeros((nb, nb), dtype=bool)
    for i, j in np.asarray(pairs).reshape(-1, 2).tolist():
        adj[i, j] = adj[j, i] = True
    pos = np.empty(nb, dtype=np.int64)
    pos[np.asarray(order)] = np.arange(nb)
    blocks = set()
    for k in range(nb):
        I = int(order[k])
        later = [J for J in range(nb) if adj[I, J] and pos[J] > k]
        for J in later:
            blocks.add((J, I))
        for a in later:
            for b in later:
                if a != b:
                    adj[a, b] = True
    return blocks
