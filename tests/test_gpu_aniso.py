"""Anisotropic materials a(x) I + B (paper Sec. 4.4) on the GPU against the
matrix-valued CPU oracle: full grid and TT/CP, untruncated parity, the
truncated energy bound, batching and bilinearity in E."""
import numpy as np
import pytest

import paper_1902_07455_amd as P
import workloads as W
from oracle import fg_tensor as FT

pytestmark = pytest.mark.gpu


def _rel(A, B):
    return np.max(np.abs(A - B)) / np.max(np.abs(B))


def _oracle(a, B, tol=1e-12, E=None):
    return FT.solve(FT.isotropic_plus_constant(a, B), Es=E, tol=tol, max_iter=2000)


def test_full_2d_square_paper_B(dev):
    """The 2D square (N = 45, contrast 10) with the paper's 2D B."""
    a = W.square_coeff(45, 2)
    B = W.anisotropy(2)
    s = P.Solver(d=2, N=(45, 45), format="full", solver_tol=1e-12, max_iter=2000, aniso=B)
    r = s.solve(full=a)
    o = _oracle(a, B)
    assert r.rc == 0
    assert _rel(r.A_H, o.A_H) <= 1e-10
    assert abs(r.A_H[0, 1]) > 1.0            # B couples the axes
    assert abs(r.iters[0] - o.iters[0]) <= 1


@pytest.mark.parametrize("N,seed", [((15, 15, 15), 0), ((9, 15, 21), 1), ((27, 25, 45), 2), ((21, 9, 5), 3)])
def test_full_3d_random_paper_B(dev, N, seed):
    a = np.random.default_rng(40 + seed).uniform(0.2, 8.0, N)
    B = W.anisotropy(3)
    s = P.Solver(d=3, N=N, format="full", solver_tol=1e-12, max_iter=2000, aniso=B)
    r = s.solve(full=a)
    o = _oracle(a, B)
    assert r.rc == 0
    assert _rel(r.A_H, o.A_H) <= 1e-10
    assert np.allclose(r.A_H, r.A_H.T, atol=1e-12 * np.max(np.abs(r.A_H)))


def test_full_general_E_is_bilinear(dev):
    a = W.ball_coeff(21, inside=10.0)
    B = W.anisotropy(3)
    E = np.array([[0.3, -1.2, 0.5], [1.0, 2.0, -0.7]])
    s = P.Solver(d=3, N=(21,) * 3, format="full", solver_tol=1e-12, max_iter=2000, aniso=B, max_nE=3)
    A = s.solve(full=a).A_H
    G = s.solve(full=a, E=E).A_H
    assert _rel(G, E @ A @ E.T) <= 1e-10


def test_full_constant_coefficient_is_exact(dev):
    """a constant: the right-hand side vanishes, A_H = a I + B, no iteration."""
    B = W.anisotropy(3)
    s = P.Solver(d=3, N=(9, 9, 9), format="full", solver_tol=1e-10, max_iter=50, aniso=B)
    r = s.solve(full=np.full((9, 9, 9), 2.5))
    assert np.allclose(r.A_H, 2.5 * np.eye(3) + B, rtol=0, atol=1e-13)
    assert list(r.iters) == [0, 0, 0]


@pytest.mark.parametrize("d,N", [(2, 45), (3, 9), (3, 11), (3, 13), (3, 15)])
def test_tt_untruncated_equals_oracle(dev, d, N):
    """Rank cap at the grid size: no truncation, so the TT solve of
    a I + B is the full solve.  The axis coupling of B gives the 3D
    correctors the full bond rank N (smallest singular values 1e-5 .. 1e-3
    of the largest), so every rounding runs with sketches as wide as the
    bond space (identity sketches: a square Gaussian one shrinks directions
    below the orthonormalisation's threshold and costs 1e-9 .. 1e-8)."""
    bound = 1e-10
    cp = W.square_cp(N, d)
    B = W.anisotropy(d)
    s = P.Solver(d=d, N=(N,) * d, format="tt", rank_cap=N, solver_tol=1e-12, max_iter=300, coeff_rank=2,
                 aniso=B)
    r = s.solve(cp=(cp.weights, cp.factors))
    o = _oracle(cp.full(), B)
    assert _rel(r.A_H, o.A_H) <= bound


def test_cp_untruncated_equals_oracle_2d(dev):
    cp = W.square_cp(45, 2)
    B = W.anisotropy(2)
    s = P.Solver(d=2, N=(45, 45), format="cp", rank_cap=45, solver_tol=1e-12, max_iter=300, coeff_rank=2,
                 aniso=B)
    r = s.solve(cp=(cp.weights, cp.factors))
    assert _rel(r.A_H, _oracle(cp.full(), B).A_H) <= 1e-10


def test_tt_untruncated_mr(dev):
    """The minimal-residual solver with B, untruncated (3D, N = 9)."""
    N = 9
    cp = W.square_cp(N, 3)
    B = W.anisotropy(3)
    s = P.Solver(d=3, N=(N,) * 3, format="tt", rank_cap=N, solver="mr", solver_tol=1e-12, max_iter=600,
                 coeff_rank=2, aniso=B)
    r = s.solve(cp=(cp.weights, cp.factors))
    assert _rel(r.A_H, _oracle(cp.full(), B).A_H) <= 1e-10


@pytest.mark.parametrize("cap", [4, 8])
def test_tt_truncated_is_upper_bound(dev, cap):
    """Truncated correctors give A_H,r - A_H positive semi-definite (the
    energy identity of Sec. 4.3 holds for any SPD coefficient)."""
    N = 21
    cp = W.square_cp(N, 3, inside=10.0)
    B = W.anisotropy(3)
    o = _oracle(cp.full(), B)
    s = P.Solver(d=3, N=(N,) * 3, format="tt", rank_cap=cap, solver_tol=1e-10, max_iter=100, coeff_rank=2,
                 aniso=B)
    r = s.solve(cp=(cp.weights, cp.factors))
    D = r.A_H - o.A_H
    assert np.min(np.linalg.eigvalsh(0.5 * (D + D.T))) >= -1e-9 * np.max(np.abs(o.A_H))
    assert _rel(r.A_H, o.A_H) < 0.2


def test_tt_batch_equals_solo(dev):
    """Two microstructures in one batched solve equal their solo solves."""
    N = 15
    B = W.anisotropy(3)
    cps = [W.square_cp(N, 3, inside=10.0), W.square_cp(N, 3, inside=4.0)]
    kw = dict(d=3, N=(N,) * 3, format="tt", rank_cap=6, solver_tol=1e-8, max_iter=100, coeff_rank=2, aniso=B)
    solo = [P.Solver(**kw).solve(cp=(c.weights, c.factors)).A_H for c in cps]
    sb = P.Solver(max_nE=6, **kw)
    both = sb.solve_batch([dict(cp=(c.weights, c.factors)) for c in cps])
    for r, s in zip(both, solo):
        assert np.array_equal(r.A_H, s)


def test_zero_B_is_the_isotropic_solve(dev):
    """B = 0 takes the isotropic path: bit-identical results."""
    N = 15
    cp = W.square_cp(N, 3, inside=10.0)
    kw = dict(d=3, N=(N,) * 3, format="tt", rank_cap=6, solver_tol=1e-8, max_iter=100, coeff_rank=2)
    r0 = P.Solver(**kw).solve(cp=(cp.weights, cp.factors)).A_H
    r1 = P.Solver(aniso=np.zeros((3, 3)), **kw).solve(cp=(cp.weights, cp.factors)).A_H
    assert np.array_equal(r0, r1)
