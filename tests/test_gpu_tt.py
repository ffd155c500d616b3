"""TT rounding (randomised sketch + SVD cut) on the GPU against the oracle's
SVD-based truncation and exact reconstructions."""
import numpy as np
import pytest

import paper_1902_07455_amd as P
import workloads as W
from oracle import lowrank as L

pytestmark = pytest.mark.gpu


def _dev(cores_list, dev):
    """list over systems of cores -> batched torch cores (nE, r0, N, r1)."""
    import torch
    d = len(cores_list[0])
    return [torch.from_numpy(np.stack([c[j] for c in cores_list])).to(dev) for j in range(d)]


def _host(outs, e):
    return [G[e].cpu().numpy() for G in outs]


@pytest.mark.parametrize("Ns,ranks,cap", [((9, 11, 13), (1, 3, 4, 1), 5), ((15, 15, 15), (1, 6, 6, 1), 20),
                                          ((45, 27, 35), (1, 8, 5, 1), 8), ((135, 135, 135), (1, 9, 9, 1), 20),
                                          ((45, 45, 45), (1, 30, 28, 1), 40),   # sketch 44 > 32
                                          ((90, 90, 90), (1, 40, 45, 1), 80),   # sketches 80, 84 > 64
                                          ((81, 81, 81), (1, 55, 50, 1), 110)])  # sketches 81, 81
def test_exact_low_rank_is_reproduced(dev, Ns, ranks, cap):
    """A sum of two trains whose true ranks fit the cap is reproduced to
    rounding level (the randomised sketch spans the exact range)."""
    systems = []
    fulls = []
    for e in range(2):
        X = W.random_tt(Ns, list(ranks), 10 + e)
        Y = L.tt_scale(X, 0.25 + e)
        systems.append(L.tt_add(X, Y))          # ranks doubled, exact ranks unchanged
        fulls.append((1.25 + e) * L.tt_full(X))
    outs, kept = P.tt_round(_dev(systems, dev), cap=cap, tol=0.0, oversample=4, seed=3)
    for e in range(2):
        got = L.tt_full(_host(outs, e))
        assert np.max(np.abs(got - fulls[e])) <= 1e-11 * np.max(np.abs(fulls[e]))
        assert list(kept[:, e]) == [ranks[1], ranks[2]]


@pytest.mark.parametrize("e2", [-300, 300])
def test_exact_low_rank_any_scale(dev, e2):
    """The same exact-rank case with the train scaled by 2^e2: Gram entries
    far outside FP32's range must not change the ranks found, and the result
    is the scaled reconstruction."""
    Ns, ranks = (15, 17, 13), (1, 5, 4, 1)
    X = W.random_tt(Ns, list(ranks), 21)
    Xs = [np.ldexp(X[0], e2)] + [c.copy() for c in X[1:]]
    outs, kept = P.tt_round(_dev([L.tt_add(Xs, Xs)], dev), cap=8, tol=0.0, oversample=4, seed=5)
    want = np.ldexp(2.0 * L.tt_full(X), e2)
    got = L.tt_full(_host(outs, 0))
    assert list(kept[:, 0]) == [ranks[1], ranks[2]]
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


@pytest.mark.parametrize("d", [2, 3])
def test_truncation_error_near_optimal(dev, d):
    Ns = (30, 40) if d == 2 else (12, 14, 16)
    rng = np.random.default_rng(5)
    if d == 2:
        X = rng.standard_normal((Ns[0], 25)) @ np.diag(0.6 ** np.arange(25)) @ rng.standard_normal((25, Ns[1]))
        cores = L.tt_svd(X)
    else:
        X = L.tt_full(W.random_tt(Ns, [1, 12, 12, 1], 6))
        X = X + 0.01 * L.tt_full(W.random_tt(Ns, [1, 10, 10, 1], 7))
        cores = L.tt_svd(X)
    cap = 6
    best = L.tt_round(cores, rank_cap=cap)
    err_best = np.linalg.norm(L.tt_full(best) - X)
    outs, _ = P.tt_round(_dev([cores], dev), cap=cap, oversample=10, seed=1)
    err = np.linalg.norm(L.tt_full(_host(outs, 0)) - X)
    assert err <= 1.5 * err_best + 1e-12 * np.linalg.norm(X)
    if d == 2:
        s = np.linalg.svd(X, compute_uv=False)
        assert err_best == pytest.approx(np.sqrt(np.sum(s[cap:] ** 2)), rel=1e-8)


def test_tolerance_cut(dev):
    """With a tolerance, the kept rank is the smallest whose dropped tail is
    within tol^2 ||X||^2/(d-1), and the error respects the bound."""
    Ns = (20, 20, 20)
    parts = [L.tt_scale(W.random_tt(Ns, [1, 1, 1, 1], 20 + i), 10.0 ** (-i)) for i in range(6)]
    X = parts[0]
    for p in parts[1:]:
        X = L.tt_add(X, p)
    full = L.tt_full(X)
    tol = 2e-3
    outs, kept = P.tt_round(_dev([X], dev), cap=20, tol=tol, oversample=4, seed=2)
    got = L.tt_full(_host(outs, 0))
    assert np.linalg.norm(got - full) <= tol * np.linalg.norm(full) * (1 + 1e-6)
    assert kept[0, 0] < 6 and kept[1, 0] < 6


def test_zero_train(dev):
    import torch
    cores = [torch.zeros((1, 1, 9, 4), dtype=torch.float64, device=dev),
             torch.zeros((1, 4, 9, 4), dtype=torch.float64, device=dev),
             torch.zeros((1, 4, 9, 1), dtype=torch.float64, device=dev)]
    outs, kept = P.tt_round(cores, cap=3)
    assert all(float(torch.max(torch.abs(G))) == 0.0 for G in outs)
    assert list(kept[:, 0]) == [0, 0]


def test_compress_exact_low_rank(dev):
    """The smooth coefficient (CP rank 9, so TT ranks <= 9) compressed from
    its full field at cap 20, tol 0: reproduced to rounding, kept ranks equal
    the numerical ranks of the unfoldings."""
    import torch
    import workloads as W
    from oracle import lowrank as LR
    N = 45
    a = W.smooth_cp(N, W.smooth_params(0)).full()
    cores, kept = P.compress_tt(torch.from_numpy(a).to(dev), cap=20, tol=0.0, seed=1)
    torch.cuda.synchronize()
    got = LR.tt_full([G.cpu().numpy() for G in cores])
    assert np.max(np.abs(got - a)) <= 1e-11 * np.max(np.abs(a))
    ref_ranks = LR.tt_ranks(LR.tt_svd(a, tol=1e-13))[1:3]
    assert kept == ref_ranks


@pytest.mark.parametrize("cap,tol", [(12, 0.0), (16, 0.0), (40, 1e-3)])
def test_compress_ball_near_optimal(dev, cap, tol):
    """Ball inclusion (not separable; TT ranks grow with N): the compressed
    train is within 1.5x the error of the oracle's deterministic TT-SVD at the
    same kept ranks, and respects the tolerance when the cap is not binding."""
    import torch
    import workloads as W
    from oracle import lowrank as LR
    N = 63
    a = W.ball_coeff(N)
    cores, kept = P.compress_tt(torch.from_numpy(a).to(dev), cap=cap, tol=tol, seed=2)
    torch.cuda.synchronize()
    got = LR.tt_full([G.cpu().numpy() for G in cores])
    err = np.linalg.norm(got - a)
    # the oracle's TT-SVD at the same rank (the ball is symmetric: equal kept ranks)
    assert kept[0] == kept[1]
    err_opt = np.linalg.norm(LR.tt_full(LR.tt_svd(a, rank_cap=kept[0])) - a)
    assert err <= 1.5 * err_opt + 1e-12 * np.linalg.norm(a)
    if tol > 0 and max(kept) < cap:
        assert err <= tol * np.linalg.norm(a) * (1 + 1e-6)
