"""MFMA FP64 GEMM and the batched Jacobi eigensolver against numpy."""
import numpy as np
import pytest

import paper_1902_07455_amd as P

pytestmark = pytest.mark.gpu

# every wave layout of the FP64 kernel: m, n <= 32 (K split in the block),
# n <= 32 with m <= 64 / m > 64, m <= 32 with n <= 64 / n > 64, 64 x 64, the
# 96 x 96 tile kernel (a side of 65..96, the other of 65..96 or above 128),
# the 80 x 128 tile kernel (m of 65..80, n of at least 128) and the 128 x 128
# tile kernel
SHAPES = [(1, 1, 1), (5, 7, 3), (64, 64, 16), (65, 63, 17), (100, 30, 4050), (2430, 30, 180),
          (30, 30, 24300), (180, 20, 2700), (1, 1, 24300), (7, 200, 1), (45, 26, 135), (26, 45, 135),
          (64, 32, 2025), (32, 64, 300), (33, 33, 97), (16, 16, 135),
          # 96 x 96 tiles, ragged edges and split K
          (96, 96, 16), (73, 73, 811), (90, 65, 90), (85, 1500, 73), (1500, 96, 33), (90, 200, 500),
          # 80 x 128 tiles (m of 65..80, n >= 128), ragged edges and split K
          (73, 1500, 73), (80, 128, 16), (65, 300, 500), (73, 128, 73),
          # 128 x 128 tiles (m, n >= 128), ragged edges and split K
          (128, 128, 16), (129, 300, 97), (300, 129, 1000), (257, 140, 5000), (1000, 520, 33)]


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("batch", [1, 3])
def test_gemm(dev, m, n, k, ta, tb, batch):
    import torch
    rng = np.random.default_rng(m * 7 + n * 13 + k + 100 * ta + 10 * tb + batch)
    A = rng.standard_normal((batch, k, m) if ta else (batch, m, k))
    B = rng.standard_normal((batch, n, k) if tb else (batch, k, n))
    C0 = rng.standard_normal((batch, m, n))
    tA, tB, tC = (torch.from_numpy(x).to(dev) for x in (A, B, C0))
    P.gemm(tA, tB, tC, ta=bool(ta), tb=bool(tb), alpha=0.7, beta=-1.3)
    torch.cuda.synchronize()
    opA = np.swapaxes(A, 1, 2) if ta else A
    opB = np.swapaxes(B, 1, 2) if tb else B
    ref = 0.7 * opA @ opB - 1.3 * C0
    err = np.max(np.abs(tC.cpu().numpy() - ref))
    assert err <= 1e-13 * max(1.0, np.sqrt(k)) * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("k", [9, 300])
def test_gemm_batch_beyond_one_grid(dev, k):
    """More matrices than one launch's grid z extent (65535) go in several
    launches; every matrix of the batch is right (k = 300 also splits K)."""
    import torch
    batch, m, n = 70001, 2, 3
    rng = np.random.default_rng(k)
    A = rng.standard_normal((batch, m, k))
    B = rng.standard_normal((batch, k, n))
    tA, tB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    tC = torch.zeros((batch, m, n), dtype=torch.float64, device=dev)
    P.gemm(tA, tB, tC)
    torch.cuda.synchronize()
    ref = A @ B
    err = np.max(np.abs(tC.cpu().numpy() - ref))
    assert err <= 1e-13 * np.sqrt(k) * np.max(np.abs(ref))


def test_gemm_beta_zero_ignores_nan(dev):
    import torch
    A = torch.ones((1, 4, 3), dtype=torch.float64, device=dev)
    B = torch.ones((1, 3, 5), dtype=torch.float64, device=dev)
    Cm = torch.full((1, 4, 5), float("nan"), dtype=torch.float64, device=dev)
    P.gemm(A, B, Cm, beta=0.0)
    torch.cuda.synchronize()
    assert torch.all(Cm == 3.0)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 30, 45, 64])
@pytest.mark.parametrize("kind", ["spd", "rankdef", "indef"])
def test_syevj(dev, n, kind):
    import torch
    rng = np.random.default_rng(n + len(kind))
    batch = 3
    if kind == "spd":
        X = rng.standard_normal((batch, n, n + 5))
        A = X @ np.swapaxes(X, 1, 2)
    elif kind == "rankdef":
        r = max(1, n // 3)
        X = rng.standard_normal((batch, n, r))
        A = X @ np.swapaxes(X, 1, 2)
    else:
        X = rng.standard_normal((batch, n, n))
        A = X + np.swapaxes(X, 1, 2)
    W, V = P.syevj(torch.from_numpy(A).to(dev))
    torch.cuda.synchronize()
    W, V = W.cpu().numpy(), V.cpu().numpy()
    for b in range(batch):
        ref = np.sort(np.linalg.eigvalsh(A[b]))[::-1]
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(W[b] - ref)) <= 1e-13 * scale * n
        assert np.all(np.diff(W[b]) <= 1e-12 * scale)
        # A V = V diag(W), V orthonormal
        assert np.max(np.abs(A[b] @ V[b] - V[b] * W[b][None, :])) <= 1e-12 * scale * n
        assert np.max(np.abs(V[b].T @ V[b] - np.eye(n))) <= 1e-12 * n


def _graded_gram(rng, n, rank, decades):
    Y = rng.standard_normal((3 * n + 8, rank)) * np.logspace(0, -decades, rank)
    Y = Y @ rng.standard_normal((rank, n))
    return Y.T @ Y


@pytest.mark.parametrize("n,rank,c", [(1, 1, 1), (2, 2, 1), (5, 3, 4), (26, 26, 16), (26, 10, 16),
                                      (40, 40, 30), (64, 64, 54), (64, 20, 40),
                                      # sketch sizes above 64 (rank caps up to 118)
                                      (65, 65, 60), (90, 90, 80), (96, 50, 80), (97, 97, 87), (128, 128, 118),
                                      (128, 70, 100)])
@pytest.mark.parametrize("decades", [2, 7])
def test_gram_cut_subspace(dev, n, rank, c, decades):
    """Kept eigenvectors of a PSD Gram matrix: orthonormal, eigen-relation,
    and the captured energy equals the top-c eigenvalue sum (Eckart-Young)."""
    import torch
    rng = np.random.default_rng(7 * n + rank + decades)
    G = np.stack([_graded_gram(rng, n, rank, decades) for _ in range(3)])
    S, kept, sweeps = P.gram_cut(torch.from_numpy(G).to(dev), c)
    torch.cuda.synchronize()
    S, kept, sweeps = S.cpu().numpy(), kept.cpu().numpy(), sweeps.cpu().numpy()
    for b in range(3):
        lam = np.sort(np.linalg.eigvalsh(G[b]))[::-1]
        k = int(kept[b])
        # exact rank <= c: every direction above the Cholesky threshold is kept
        assert k <= min(c, n)
        assert k >= min(c, rank) - (1 if decades > 6 else 0)
        Sk = S[b][:, :k]
        assert np.all(S[b][:, k:] == 0.0)
        assert np.max(np.abs(Sk.T @ Sk - np.eye(k))) <= 1e-13 * max(n, 4)
        GS = G[b] @ Sk
        mu = np.sum(Sk * GS, axis=0)
        assert np.all(np.diff(mu) <= 1e-13 * lam[0])
        assert np.max(np.abs(GS - Sk * mu[None, :])) <= 1e-12 * lam[0]
        captured = np.sum(mu)
        assert captured >= np.sum(lam[:k]) - 1e-13 * n * lam[0]
        assert sweeps[b] <= 12


@pytest.mark.parametrize("n", [12, 26, 40, 64, 90, 128])
def test_gram_cut_scale_invariant(dev, n):
    """G scaled by 2^600 or 2^-600 (entries far outside FP32's range, squared
    norms near FP64's limits): the cut works on G divided by a power of two
    near its largest diagonal entry, so the basis and the kept count come
    out bit for bit the same as for G itself."""
    import torch
    rng = np.random.default_rng(11 * n)
    G = np.stack([_graded_gram(rng, n, n, 7) for _ in range(2)])
    outs = []
    for e in (0, 600, -600):
        S, kept, _ = P.gram_cut(torch.from_numpy(np.ldexp(G, e)).to(dev), max(1, n - 6), tol=1e-4)
        torch.cuda.synchronize()
        outs.append((S.cpu().numpy(), kept.cpu().numpy()))
    S0, k0 = outs[0]
    assert np.all(k0 > 0)
    lam = np.sort(np.linalg.eigvalsh(G[0]))[::-1]
    assert np.max(np.abs(S0[0][:, :k0[0]].T @ G[0] @ S0[0][:, :k0[0]] - np.diag(lam[:k0[0]]))) <= 1e-12 * lam[0]
    for S, kept in outs[1:]:
        assert np.array_equal(kept, k0)
        assert np.array_equal(S, S0)


def test_gram_cut_tolerance_and_zero(dev):
    import torch
    rng = np.random.default_rng(3)
    n = 30
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = 10.0 ** -np.arange(n, dtype=np.float64)
    G = (Q * lam) @ Q.T
    G = np.stack([G, np.zeros((n, n))])
    tol = 3e-3
    S, kept, _ = P.gram_cut(torch.from_numpy(G).to(dev), 20, tol=tol)
    torch.cuda.synchronize()
    kept = kept.cpu().numpy()
    tail = np.cumsum(lam[::-1])[::-1]          # tail[k] = sum_{j >= k} lam_j
    want = int(np.argmax(tail <= tol * tol * np.sum(lam)))
    assert kept[0] == want
    assert kept[1] == 0 and float(torch.max(torch.abs(S[1]))) == 0.0


def _round_f32(x):
    return x.astype(np.float32).astype(np.float64)


def _round_bf16(x):
    """FP64 -> FP32 (nearest) -> BF16 (nearest even), as the kernel stages it."""
    u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _split_bf16(x):
    """The kernel's two-term split: x32 = FP32(x), hi = BF16(x32),
    lo = BF16(x32 - hi) (the difference is exact in FP32)."""
    x32 = x.astype(np.float32).astype(np.float64)
    hi = _round_bf16(x32)
    lo = _round_bf16(x32 - hi)
    return hi, lo


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (64, 64, 32), (65, 63, 33), (100, 30, 4050), (2430, 30, 180),
                                   (30, 30, 24300), (7, 200, 1)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_gemm_mixed(dev, m, n, k, ta, tb, prec):
    """Reduced-precision MFMA GEMM against numpy on operands rounded the same
    way (FP32; BF16 as the hi + lo split of the FP32 value, three products);
    the FP32 accumulation error bound is (terms) u32 sum|a||b| (u32 = 2^-24)."""
    import torch
    rng = np.random.default_rng(m + 3 * n + 7 * k + 11 * ta + 13 * tb + len(prec))
    batch = 2
    A = rng.standard_normal((batch, k, m) if ta else (batch, m, k))
    B = rng.standard_normal((batch, n, k) if tb else (batch, k, n))
    C0 = rng.standard_normal((batch, m, n))
    tA, tB, tC = (torch.from_numpy(x).to(dev) for x in (A, B, C0))
    P.gemm(tA, tB, tC, ta=bool(ta), tb=bool(tb), alpha=0.5, beta=2.0, precision=prec)
    torch.cuda.synchronize()
    A_ = np.swapaxes(A, 1, 2) if ta else A
    B_ = np.swapaxes(B, 1, 2) if tb else B
    if prec == "fp32":
        opA, opB = _round_f32(A_), _round_f32(B_)
        ref = 0.5 * opA @ opB + 2.0 * C0
        mag = np.abs(opA) @ np.abs(opB)
        nterm = k
    else:
        # hi*hi + hi*lo + lo*hi of the split operands
        (ah, al), (bh, bl) = _split_bf16(A_), _split_bf16(B_)
        ref = 0.5 * (ah @ bh + ah @ bl + al @ bh) + 2.0 * C0
        mag = np.abs(ah) @ np.abs(bh) + np.abs(ah) @ np.abs(bl) + np.abs(al) @ np.abs(bh)
        nterm = 3 * k
    bound = 0.5 * (nterm + 2) * 2.0 ** -24 * mag + 1e-15 * np.abs(ref)
    assert np.all(np.abs(tC.cpu().numpy() - ref) <= bound)
    # and the rounding really happened (BF16 differs from FP64 visibly)
    if prec == "bf16" and k >= 32:
        exact = 0.5 * (np.swapaxes(A, 1, 2) if ta else A) @ (np.swapaxes(B, 1, 2) if tb else B) + 2.0 * C0
        assert np.max(np.abs(tC.cpu().numpy() - exact)) > 1e-6
