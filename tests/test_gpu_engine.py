"""Kernel unit parity of the MFMA tile engine (complex GEMM with the modes
the task bodies use) against numpy on random complex operands."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _d3m():
    import paper_2002_05026_amd as d3m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return d3m


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


CASES = [(16, 16, 4), (128, 128, 64), (100, 37, 53), (1, 1, 1), (128, 1, 300), (33, 128, 16), (7, 120, 0)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("m,n,k", CASES)
@pytest.mark.parametrize("amode", [0, 1])
@pytest.mark.parametrize("scaled", [False, True])
def test_engine_modes(prec, m, n, k, amode, scaled):
    d3m = _d3m()
    print(f"[engine] prec={prec} m={m} n={n} k={k} amode={amode} scaled={scaled}", flush=True)
    rng = np.random.default_rng(m * 1000 + n * 10 + k)
    A = _cn(rng, (m, k))
    Bm = _cn(rng, (n, k))
    d = _cn(rng, (k,)) + 1.5
    C0 = _cn(rng, (m, n))
    lda = (m + 3) if amode == 0 else (k + 5)
    Abuf = np.zeros(max(lda * max(k if amode == 0 else m, 1), 1), dtype=np.complex128)
    if amode == 0:
        for p in range(k):
            Abuf[p * lda:p * lda + m] = A[:, p]
    else:
        for i in range(m):
            Abuf[i * lda:i * lda + k] = A[i, :]
    ldb = n + 2
    Bbuf = np.zeros(max(ldb * k, 1), dtype=np.complex128)
    for p in range(k):
        Bbuf[p * ldb:p * ldb + n] = Bm[:, p]
    ldc = m + 1
    Cbuf = np.zeros(ldc * n, dtype=np.complex128)
    for j in range(n):
        Cbuf[j * ldc:j * ldc + m] = C0[:, j]
    dt = torch.complex128 if prec == 0 else torch.complex64
    tA = torch.from_numpy(Abuf).to(dt).cuda()
    tB = torch.from_numpy(Bbuf).to(dt).cuda()
    tC = torch.from_numpy(Cbuf).to(dt).cuda()
    td = torch.from_numpy(d if k else np.ones(1, dtype=np.complex128)).to(dt).cuda()
    alpha, beta = -0.5, 1.0
    d3m.debug_gemm(tA, tB, tC, m, n, k, amode=amode, d=td if scaled else None, alpha=alpha, beta=beta,
                   lda=lda, ldb=ldb, ldc=ldc)
    torch.cuda.synchronize()
    got = tC.cpu().numpy().astype(np.complex128)
    As = A * d[None, :] if scaled else A
    ref = alpha * (As @ Bm.T) + beta * C0
    G = np.stack([got[j * ldc:j * ldc + m] for j in range(n)], axis=1)
    tol = 1e-13 if prec == 0 else 3e-6
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(G - ref).max() <= tol * scale * max(1, k) ** 0.5
    # padding rows of C untouched
    for j in range(n):
        assert got[j * ldc + m] == Cbuf[j * ldc + m].astype(np.complex64 if prec else np.complex128)


@pytest.mark.parametrize("prec", [0, 1])
def test_engine_symmetric_lower_mode(prec):
    d3m = _d3m()
    rng = np.random.default_rng(9)
    nI, i0, m, n = 150, 40, 70, 20
    S = _cn(rng, (nI, nI))
    S = np.tril(S) + np.tril(S, -1).T
    Sbuf = np.asfortranarray(np.tril(S) + np.triu(np.full((nI, nI), np.nan + 0j), 1)).reshape(-1, order="F")
    Bm = _cn(rng, (n, nI))
    dt = torch.complex128 if prec == 0 else torch.complex64
    tS = torch.from_numpy(Sbuf).to(dt).cuda()
    tB = torch.from_numpy(np.asfortranarray(Bm).reshape(-1, order="F")).to(dt).cuda()
    tC = torch.zeros(m * n, dtype=dt).cuda()
    d3m.debug_gemm(tS, tB, tC, m, n, nI, amode=2, i0=i0, lda=nI, ldb=n, ldc=m)
    torch.cuda.synchronize()
    G = tC.cpu().numpy().reshape(m, n, order="F")
    ref = S[i0:i0 + m, :] @ Bm.T
    tol = 1e-13 if prec == 0 else 3e-6
    assert np.all(np.isfinite(G))  # the NaN upper triangle is never read
    assert np.abs(G - ref).max() <= tol * np.abs(ref).max() * 13
