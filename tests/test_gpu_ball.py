"""The 243^3 ball inclusion of contrast 100 (radius 0.3, a = 100 inside, 1
outside): full-grid solve against the oracle's stored value, compression
of the coefficient into an admissible tensor train, and the truncated TT
solve against the full-grid solve of the same field."""
import os

import numpy as np
import pytest

import paper_1902_07455_amd as P
import workloads as W

pytestmark = pytest.mark.gpu

N = 243
HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    with open(os.path.join(HERE, "golden", "ball3d_N243_c100_AH.txt")) as f:
        return float([ln for ln in f if not ln.startswith("#")][0])


@pytest.fixture(scope="module")
def ball(dev):
    import torch
    return torch.from_numpy(W.ball_coeff(N)).to(dev)


def _trim(cores, kept):
    k1, k2 = kept
    return [cores[0][:, :, :k1].contiguous(), cores[1][:k1, :, :k2].contiguous(), cores[2][:k2].contiguous()]


def _tt_full(cores):
    import torch
    return torch.einsum("ia,ajb,bk->ijk", cores[0][0], cores[1], cores[2][:, :, 0])


def test_full_grid_against_oracle(ball):
    """a_H of the full-grid GPU solve (E = e1) against the oracle's PCG at
    1e-10 (stored by tests/golden/make_golden.py): the parity bar 1e-10; the
    ball is symmetric under axis permutations, so A_H = a_H I."""
    s = P.Solver(d=3, N=(N,) * 3, format="full", solver_tol=1e-10, max_iter=2000)
    r = s.solve(full=ball)
    g = _golden()
    assert abs(r.A_H[0, 0] - g) <= 1e-10 * g
    assert np.max(np.abs(np.diag(r.A_H) - g)) <= 1e-10 * g
    assert np.max(np.abs(r.A_H - np.diag(np.diag(r.A_H)))) <= 1e-10 * g


def test_compressed_ball_is_exact_and_admissible(ball):
    """The ball's TT ranks at N = 243 are 73 (one unfolding row per distinct
    |x_1| inside plus the constant): cap 80 at tol 1e-6 keeps 73 and
    reproduces the field, which stays positive; every cap below leaves the
    truncated indicator undershooting at the sphere (negative values), and
    the solver rejects such a coefficient."""
    import torch
    cores, kept = P.compress_tt(ball, cap=80, tol=1e-6, seed=1)
    assert kept == [73, 73]
    tc = _trim(cores, kept)
    f = _tt_full(tc)
    assert float(torch.linalg.norm(f - ball) / torch.linalg.norm(ball)) <= 1e-6
    assert float(f.min()) > 0.99
    cores72, kept72 = P.compress_tt(ball, cap=72, tol=1e-6, seed=1)
    f72 = _tt_full(_trim(cores72, kept72))
    assert float(f72.min()) < 0.0
    s = P.Solver(d=3, N=(N,) * 3, format="tt", rank_cap=20, solver_tol=1e-4, max_iter=5, coeff_rank=72)
    with pytest.raises(P.LrfgError) as ei:
        s.solve(tt=_trim(cores72, kept72), E=[[1.0, 0.0, 0.0]])
    assert ei.value.status == -2


@pytest.mark.parametrize("cap,over,bound", [(90, 38, 1e-6), (80, 48, 5e-6)])
def test_tt_solve_ball_c100(ball, cap, over, bound):
    """Truncated TT PCG on the compressed ball (coefficient ranks 73, product
    ranks 73 c) at rank cap 90 and 80: A_H within `bound` of the full-grid
    value and above it (the energy identity of Sec. 4.3: the truncated
    corrector's A_H E.E exceeds the exact one by its squared energy error).
    Sketches of 128 columns and 16 exponential-sum terms; the iterate is
    kept by its energy once the residual stops decreasing."""
    cores, kept = P.compress_tt(ball, cap=80, tol=1e-6, seed=1)
    tc = _trim(cores, kept)
    g = _golden()
    s = P.Solver(d=3, N=(N,) * 3, format="tt", rank_cap=cap, trunc_tol=0.0, solver_tol=1e-6, max_iter=100,
                 coeff_rank=73, oversample=over, precond_terms=16, max_nE=1)
    r = s.solve(tt=tc, E=[[1.0, 0.0, 0.0]])
    err = (r.A_H[0, 0] - g) / g
    print(f"TT cap {cap}: a_H {r.A_H[0, 0]:.12f} rel err {err:.3e} iters {r.iters} ranks {r.ranks.tolist()}")
    assert err >= -1e-10
    assert err <= bound
    assert max(r.ranks[0][1:3]) <= cap
