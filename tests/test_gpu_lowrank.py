"""Low-rank (TT, and CP = TT for d = 2) solve on the GPU against the CPU
oracle: untruncated equals the full solve; truncated is an energy upper
bound; closed forms."""
import numpy as np
import pytest

import paper_1902_07455_amd as P
import workloads as W
from oracle import fg

pytestmark = pytest.mark.gpu


def _rel(A, B):
    return np.max(np.abs(A - B)) / np.max(np.abs(B))


def _cp_args(cp):
    return (cp.weights, cp.factors)


@pytest.mark.parametrize("solver", ["pcg", "mr"])
def test_laminate_rank_one(dev, solver):
    N = 15
    prof = np.random.default_rng(1).uniform(0.5, 4.0, N)
    ones = np.ones(N)
    cp = W.CPCoeff(np.array([1.0]), [prof[None, :], ones[None, :], ones[None, :]])
    s = P.Solver(d=3, N=(N, N, N), format="tt", rank_cap=4, solver=solver, solver_tol=1e-12,
                 max_iter=200, coeff_rank=1)
    r = s.solve(cp=_cp_args(cp))
    H = 1.0 / np.mean(1.0 / prof)
    M = np.mean(prof)
    assert _rel(r.A_H, np.diag([H, M, M])) <= 1e-10
    # the corrector of E = e1 is a rank-1 train u(x1); the others vanish
    assert list(r.ranks[0]) == [1, 1, 1, 1]
    assert np.all(r.ranks[1:, 1:3] == 0)


@pytest.mark.parametrize("d,N", [(2, 45), (3, 15)])
def test_untruncated_equals_full_square(dev, d, N):
    """Rank cap at the grid size: no truncation, so the TT solve is the
    full solve (the square inclusion of the 2D workload, the cube in 3D)."""
    cp = W.square_cp(N, d)
    a = cp.full()
    s = P.Solver(d=d, N=(N,) * d, format="tt", rank_cap=N, solver_tol=1e-12, max_iter=300,
                 coeff_rank=2)
    r = s.solve(cp=_cp_args(cp))
    o = fg.solve(a, tol=1e-12)
    assert _rel(r.A_H, o.A_H) <= 1e-10


def _wide_tt_coeff(N, r, seed):
    """TT cores of a = 3 + 0.9 p / max|p| with p a random train of ranks r:
    ranks r + 1 (the constant is a rank-one train beside p), positive
    (a >= 2.1 everywhere); also the full field."""
    rng = np.random.default_rng(seed)
    R = [rng.standard_normal((1, N, r)), rng.standard_normal((r, N, r)), rng.standard_normal((r, N, 1))]
    p = np.einsum("aib,bjc,ckd->ijk", *R)
    sc = 0.9 / np.max(np.abs(p))
    one = np.ones(N)
    G1 = np.concatenate([3.0 * one[None, :, None], sc * R[0]], axis=2)
    G2 = np.zeros((r + 1, N, r + 1))
    G2[0, :, 0] = one
    G2[1:, :, 1:] = R[1]
    G3 = np.concatenate([one[None, :, None], R[2]], axis=0)
    a = np.einsum("aib,bjc,ckd->ijk", G1, G2, G3)
    return [G1, G2, G3], a


def test_untruncated_equals_full_wide_coefficient(dev):
    """A coefficient train of ranks 21 (above the 16 the register paths of
    the material contractions take: the mapped products per grid index and
    the regrouped energy form) with the rank cap at the grid size, so no
    truncation: the TT solve is the full solve."""
    import torch
    N = 21
    cores, a = _wide_tt_coeff(N, 20, 5)
    assert np.min(a) >= 2.0
    s = P.Solver(d=3, N=(N,) * 3, format="tt", rank_cap=N, solver_tol=1e-12, max_iter=300, coeff_rank=21)
    r = s.solve(tt=[torch.from_numpy(c).to(dev) for c in cores])
    o = fg.solve(a, tol=1e-12)
    assert _rel(r.A_H, o.A_H) <= 1e-10


def test_cp_format_2d_config(dev):
    """2D square (N = 45) in the CP format = the d = 2 train."""
    cp = W.square_cp(45, 2)
    s = P.Solver(d=2, N=(45, 45), format="cp", rank_cap=45, solver_tol=1e-12, max_iter=300,
                 coeff_rank=2)
    r = s.solve(cp=_cp_args(cp))
    o = fg.solve(cp.full(), tol=1e-12)
    assert _rel(r.A_H, o.A_H) <= 1e-10


@pytest.mark.parametrize("cap", [3, 6])
def test_truncated_is_upper_bound(dev, cap):
    """Truncated correctors give A_H,r >= A_H (Sec. 4.3 energy identity),
    and a larger rank is no worse."""
    N = 21
    cp = W.square_cp(N, 3, inside=10.0)
    o = fg.solve(cp.full(), tol=1e-12)
    s = P.Solver(d=3, N=(N,) * 3, format="tt", rank_cap=cap, solver_tol=1e-10, max_iter=100,
                 coeff_rank=2)
    r = s.solve(cp=_cp_args(cp))
    D = r.A_H - o.A_H
    assert np.min(np.linalg.eigvalsh(0.5 * (D + D.T))) >= -1e-9 * o.A_H[0, 0]
    assert _rel(r.A_H, o.A_H) < 0.2


@pytest.mark.parametrize("fmt", ["tt", "tucker"])
@pytest.mark.parametrize("e2", [-150, 150])
def test_scaled_coefficient(dev, fmt, e2):
    """A_H is linear in the coefficient: the coefficient times 2^e2 (every
    Gram matrix of the truncations then far outside FP32's range) gives
    2^e2 times the unscaled result."""
    N = 21
    cp = W.square_cp(N, 3, inside=10.0)
    kw = dict(d=3, N=(N,) * 3, format=fmt, rank_cap=6, solver_tol=1e-10, max_iter=100, coeff_rank=2)
    r0 = P.Solver(**kw).solve(cp=_cp_args(cp))
    r1 = P.Solver(**kw).solve(cp=(np.ldexp(cp.weights, e2), cp.factors))
    assert np.all(np.asarray(r1.ranks) == np.asarray(r0.ranks))
    assert _rel(np.ldexp(r1.A_H, -e2), r0.A_H) <= 1e-9


def test_smooth_135_rank20(dev):
    """The benchmark workload: 135^3 smooth coefficient (CP rank 9), TT
    rank cap 20; error against the oracle reported and bounded."""
    p = W.smooth_params(0)
    cp = W.smooth_cp(135, p)
    s = P.Solver(d=3, N=(135,) * 3, format="tt", rank_cap=20, trunc_tol=1e-8, solver_tol=1e-8,
                 max_iter=60, coeff_rank=9)
    r = s.solve(cp=_cp_args(cp))
    a, _ = W.smooth_coeff(135, p)
    o = fg.solve(a, tol=1e-10)
    err = _rel(r.A_H, o.A_H)
    print("TT 135^3 cap 20: A_H rel err", err, "iters", r.iters, "ranks", r.ranks)
    assert err <= 1e-6
    D = r.A_H - o.A_H
    assert np.min(np.linalg.eigvalsh(0.5 * (D + D.T))) >= -1e-9


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_precision_refinement(dev, prec):
    """Mixed-precision TT solve (FP32 / BF16 contractions, FP64 refinement)
    of the smooth 3D workload at N = 45, cap 16: the A_H error per entry
    against the FP64 oracle is within 1e-6 of max|A_H| (the config-4 bar).
    The FP64 residual of the truncated operator has a floor set by the rank
    cap; the refinement runs at least one outer step and its best residual
    is below the first one's."""
    N = 45
    cp = W.smooth_cp(N, W.smooth_params(0))
    o = fg.solve(cp.full(), tol=1e-12, max_iter=500)
    s = P.Solver(d=3, N=(N,) * 3, format="tt", rank_cap=16, solver_tol=1e-5, max_iter=60, coeff_rank=9,
                 precision=prec)
    r = s.solve(cp=_cp_args(cp))
    err = np.abs(r.A_H - o.A_H) / np.max(np.abs(o.A_H))
    assert np.max(err) <= 1e-6, err
    for e in range(3):
        hist = r.res_hist[e][r.res_hist[e] > 0]
        assert hist.size >= 1 and np.min(hist) <= hist[0]
    # and agrees with the FP64 solve of the same problem to the same bar
    r64 = P.Solver(d=3, N=(N,) * 3, format="tt", rank_cap=16, solver_tol=1e-5, max_iter=60,
                   coeff_rank=9).solve(cp=_cp_args(cp))
    assert _rel(r.A_H, r64.A_H) <= 1e-6


def test_mixed_precision_untruncated_exact(dev):
    """Without truncation the refined solve reaches the FP64 oracle's A_H to
    1e-10 even with BF16 contractions inside (the 2D N = 45 square)."""
    N = 45
    cp = W.square_cp(N, 2)
    o = fg.solve(cp.full(), tol=1e-12, max_iter=500)
    s = P.Solver(d=2, N=(N, N), format="tt", rank_cap=N, solver_tol=1e-11, max_iter=200, coeff_rank=2,
                 precision="bf16")
    r = s.solve(cp=_cp_args(cp))
    assert _rel(r.A_H, o.A_H) <= 1e-10
    assert r.rc == 0


def test_ball_compressed_coefficient_solve(dev):
    """Config-3 style: the ball (contrast 100) compressed from its full field
    into a TT (exact at N = 45: ranks 14), then the TT solve at cap 20 against
    the oracle's full solve of the same field: the truncated A_H is an upper
    bound (energy identity) and close; the full-grid GPU solve of the
    compressed coefficient matches the oracle to 1e-10."""
    import torch
    N = 45
    a = W.ball_coeff(N)
    cores, kept = P.compress_tt(torch.from_numpy(a).to(dev), cap=20, tol=1e-12, seed=3)
    o = fg.solve(a, tol=1e-12, max_iter=2000)
    sf = P.Solver(d=3, N=(N,) * 3, format="full", solver_tol=1e-12, max_iter=2000)
    rf = sf.solve(tt=cores)
    assert _rel(rf.A_H, o.A_H) <= 1e-10
    s = P.Solver(d=3, N=(N,) * 3, format="tt", rank_cap=20, solver_tol=1e-8, max_iter=300, coeff_rank=20)
    r = s.solve(tt=cores)
    d = np.diag(r.A_H) - np.diag(o.A_H)
    assert np.all(d >= -1e-9 * np.max(np.diag(o.A_H)))
    assert _rel(r.A_H, o.A_H) <= 5e-2


def _spike_cp(Ns, where, depth):
    """CP coefficient 1 - depth e_where (rank 2): positive except at one grid
    point when depth > 1."""
    d = len(Ns)
    w = np.array([1.0, -float(depth)])
    fac = []
    for j in range(d):
        f = np.zeros((2, Ns[j]))
        f[0] = 1.0
        f[1, where[j]] = 1.0
        fac.append(f)
    return w, fac


def _cp_to_tt(w, fac):
    """TT cores [r_{j-1}][N_j][r_j] of a CP coefficient (d = 3)."""
    R = len(w)
    G1 = (w[:, None] * fac[0]).T[None]                    # 1 x N x R
    G2 = np.zeros((R, fac[1].shape[1], R))
    for t in range(R):
        G2[t, :, t] = fac[1][t]
    G3 = fac[2][:, :, None]                                # R x N x 1
    return [G1, G2, G3]


@pytest.mark.parametrize("fmt", ["tt-cp", "tt-cores", "cp2d", "tucker", "full"])
def test_negative_coefficient_rejected(dev, fmt):
    """A coefficient that is negative at one grid point (1 - 2 e_x0) makes
    the operator indefinite: every path rejects it with ECOEFF before
    solving; the same construction with depth 0.5 (positive) solves."""
    Ns = (15, 15) if fmt == "cp2d" else (15, 15, 15)
    d = len(Ns)
    where = (3, 11, 7)[:d]
    for depth, ok in ((2.0, False), (0.5, True)):
        w, fac = _spike_cp(Ns, where, depth)
        if fmt == "full":
            s = P.Solver(d=d, N=Ns, format="full", solver_tol=1e-8, max_iter=200)
        else:
            s = P.Solver(d=d, N=Ns, format="tucker" if fmt == "tucker" else ("cp" if fmt == "cp2d" else "tt"),
                         rank_cap=6, solver_tol=1e-8, max_iter=200, coeff_rank=2)
        kw = dict(tt=_cp_to_tt(w, fac)) if fmt == "tt-cores" else dict(cp=(w, fac))
        if ok:
            r = s.solve(**kw)
            assert np.all(np.isfinite(r.A_H))
        else:
            with pytest.raises(P.LrfgError) as ei:
                s.solve(**kw)
            assert ei.value.status == -2
            assert "admissible" in str(ei.value) or "positive" in str(ei.value)
