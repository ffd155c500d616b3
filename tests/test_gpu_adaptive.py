"""Rank-adaptive TT solve (Sec. 4.2: start at a low solution rank and raise
it during the iterations) against the CPU oracle and the fixed-rank solve."""
import numpy as np
import pytest

import paper_1902_07455_amd as P
import workloads as W
from oracle import fg
from oracle import fg_tensor as FT

pytestmark = pytest.mark.gpu


def _rel(A, B):
    return np.max(np.abs(A - B)) / np.max(np.abs(B))


@pytest.mark.parametrize("d,N,start", [(3, 15, 3), (3, 15, 10), (2, 45, 4)])
def test_adaptive_untruncated_equals_oracle(dev, d, N, start):
    """Stages up to a cap at the grid size: the last stage is untruncated,
    so the solve is the full solve whatever the earlier stages left.  Every
    later stage starts from a true residual T(b - K x), whose rounding floor
    lies near 1e-8 of ||P^-1 b|| (the Gram-based truncation), so the
    tolerance sits above it; A_H's error is quadratic in the residual."""
    cp = W.square_cp(N, d, inside=10.0)
    s = P.Solver(d=d, N=(N,) * d, format="tt", rank_cap=N, rank_start=start, solver_tol=1e-7, max_iter=300,
                 coeff_rank=2)
    r = s.solve(cp=(cp.weights, cp.factors))
    o = fg.solve(cp.full(), tol=1e-12)
    assert list(r.status) == [0] * d
    assert _rel(r.A_H, o.A_H) <= 1e-10


def test_adaptive_anisotropic_untruncated(dev):
    N = 9
    cp = W.square_cp(N, 3)
    B = W.anisotropy(3)
    s = P.Solver(d=3, N=(N,) * 3, format="tt", rank_cap=N, rank_start=2, solver_tol=1e-7, max_iter=300,
                 coeff_rank=2, aniso=B)
    r = s.solve(cp=(cp.weights, cp.factors))
    o = FT.solve(FT.isotropic_plus_constant(cp.full(), B), tol=1e-12, max_iter=2000)
    assert _rel(r.A_H, o.A_H) <= 1e-10


def test_start_at_cap_is_the_fixed_solve(dev):
    """rank_start >= rank_cap: one solve at the cap, bit-identical."""
    N = 21
    cp = W.square_cp(N, 3, inside=10.0)
    kw = dict(d=3, N=(N,) * 3, format="tt", rank_cap=6, solver_tol=1e-10, max_iter=100, coeff_rank=2)
    r0 = P.Solver(**kw).solve(cp=(cp.weights, cp.factors))
    r1 = P.Solver(rank_start=6, **kw).solve(cp=(cp.weights, cp.factors))
    assert np.array_equal(r0.A_H, r1.A_H)
    assert np.array_equal(r0.iters, r1.iters)


@pytest.mark.parametrize("start", [2, 4])
def test_adaptive_truncated_upper_bound(dev, start):
    """A truncated adaptive solve: A_H,r - A_H positive semi-definite (the
    energy identity, Sec. 4.3), and about as accurate as the fixed solve at
    its final cap (within a factor 4 on the error: the last stage restarts
    the Krylov iteration from the previous stage's corrector)."""
    N = 21
    cp = W.square_cp(N, 3, inside=10.0)
    o = fg.solve(cp.full(), tol=1e-12)
    kw = dict(d=3, N=(N,) * 3, format="tt", rank_cap=8, solver_tol=1e-10, max_iter=100, coeff_rank=2)
    fixed = P.Solver(**kw).solve(cp=(cp.weights, cp.factors))
    r = P.Solver(rank_start=start, **kw).solve(cp=(cp.weights, cp.factors))
    D = r.A_H - o.A_H
    assert np.min(np.linalg.eigvalsh(0.5 * (D + D.T))) >= -1e-9 * o.A_H[0, 0]
    assert _rel(r.A_H, o.A_H) <= 4.0 * _rel(fixed.A_H, o.A_H) + 1e-9
    assert np.all(r.iters > 0)
    assert list(r.ranks[0]) == [1, 8, 8, 1] or max(r.ranks[0]) <= 8


def test_adaptive_batch_equals_solo(dev):
    N = 15
    cps = [W.square_cp(N, 3, inside=10.0), W.square_cp(N, 3, inside=3.0)]
    kw = dict(d=3, N=(N,) * 3, format="tt", rank_cap=8, rank_start=3, solver_tol=1e-9, max_iter=100,
              coeff_rank=2)
    solo = [P.Solver(**kw).solve(cp=(c.weights, c.factors)) for c in cps]
    both = P.Solver(max_nE=6, **kw).solve_batch([dict(cp=(c.weights, c.factors)) for c in cps])
    for r, s in zip(both, solo):
        assert np.array_equal(r.A_H, s.A_H)
        assert np.array_equal(r.iters, s.iters)
