"""Full-grid GaNi PCG on the GPU against the FP64 CPU oracle."""
import os

import numpy as np
import pytest

import paper_1902_07455_amd as P
import workloads as W
from oracle import fg

pytestmark = pytest.mark.gpu


def _half(x):
    H = (x.shape[-1] + 1) // 2
    return np.ascontiguousarray(x[..., :H])


def _rel(A, B):
    return np.max(np.abs(A - B)) / np.max(np.abs(B))


@pytest.mark.parametrize("N", [(5, 5, 5), (9, 15, 21), (27, 25, 45), (45, 45, 45)])
def test_operator_K_and_Pinv(dev, N):
    import torch
    rng = np.random.default_rng(sum(N))
    a = rng.uniform(0.5, 3.0, N)
    u = rng.standard_normal(N)
    uh = fg.fwd(u)
    ref = fg.apply_K(a, uh)
    ta = torch.from_numpy(a).to(dev)
    tu = torch.from_numpy(_half(uh)).to(dev)
    out = torch.zeros_like(tu)
    P.full_op(0, N, ta, tu, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.max(np.abs(got - _half(ref))) <= 1e-12 * np.max(np.abs(ref))
    P.full_op(1, N, None, tu, out)
    torch.cuda.synchronize()
    refp = fg.precond_diag(N) * uh
    assert np.max(np.abs(out.cpu().numpy() - _half(refp))) <= 1e-15 * np.max(np.abs(refp)) + 1e-300


def _solve(a, d, tol=1e-12, E=None, cp=None, max_iter=2000):
    N = a.shape if a is not None else None
    s = P.Solver(d=d, N=N, format="full", solver_tol=tol, max_iter=max_iter,
                 max_nE=(len(E) if E is not None else d))
    if cp is not None:
        return s.solve(cp=cp, E=E)
    return s.solve(full=a, E=E)


def test_square_2d_config(dev):
    """2D, N = 45, square inclusion (contrast 10, fraction 0.3), tol 1e-10."""
    a = W.square_coeff(45, 2)
    r = _solve(a, 2, tol=1e-10)
    o = fg.solve(a, tol=1e-10)
    assert r.rc == 0
    assert _rel(r.A_H, o.A_H) <= 1e-10
    g = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "square2d_N45_AH.txt"))
    assert _rel(r.A_H, g) <= 1e-10
    assert abs(r.iters[0] - o.iters[0]) <= 1
    h = r.res_hist[0, :r.iters[0]]
    assert np.allclose(h, o.res_hist[0][:len(h)], rtol=1e-6)


@pytest.mark.parametrize("N,seed", [((15, 15, 15), 0), ((9, 15, 21), 1), ((21, 9, 5), 2)])
def test_random_3d(dev, N, seed):
    a = np.random.default_rng(seed).uniform(0.2, 8.0, N)
    r = _solve(a, 3)
    o = fg.solve(a, tol=1e-12)
    assert _rel(r.A_H, o.A_H) <= 1e-10


@pytest.mark.parametrize("N", [(13, 29), (45, 27)])
def test_random_2d_nonsquare(dev, N):
    a = np.random.default_rng(5).uniform(0.3, 5.0, N)
    r = _solve(a, 2)
    o = fg.solve(a, tol=1e-12)
    assert _rel(r.A_H, o.A_H) <= 1e-10


@pytest.mark.parametrize("N", [(625, 3, 675), (729, 625, 3), (3, 675, 405)])
def test_register_pass_lengths_against_oracle(dev, N):
    """The lengths with register passes above 243 (405, 625, 675, 729; the
    benchmark's and the Ga double grids') on each of the three internal
    axes: axis 1 (gradient / divergence passes), axis 2 (line passes) and
    axis 3 (the coefficient pass), the other axes short."""
    a = np.random.default_rng(sum(N)).uniform(0.5, 2.0, N)
    r = _solve(a, 3, tol=1e-11)
    o = fg.solve(a, tol=1e-11)
    assert r.rc == 0
    assert _rel(r.A_H, o.A_H) <= 1e-10
    assert abs(int(r.iters.max()) - max(o.iters)) <= 1


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate_closed_form(dev, axis):
    N = 27
    prof = np.random.default_rng(axis).uniform(0.5, 6.0, N)
    a = W.laminate_coeff(N, 3, prof, axis=axis)
    r = _solve(a, 3)
    H = 1.0 / np.mean(1.0 / prof)
    M = np.mean(prof)
    expect = M * np.eye(3)
    expect[axis, axis] = H
    assert _rel(r.A_H, expect) <= 1e-11


def test_constant_and_general_E(dev):
    a = W.constant_coeff(9, 3, 2.5)
    r = _solve(a, 3)
    assert np.allclose(r.A_H, 2.5 * np.eye(3), atol=1e-14)
    assert list(r.iters) == [0, 0, 0]
    a = np.random.default_rng(9).uniform(0.5, 3.0, (11, 11, 11))
    E = np.array([[0.3, -1.0, 2.0]])
    r = _solve(a, 3, E=E)
    o = fg.solve(a, E, tol=1e-12)
    assert r.A_H.shape == (1, 1)
    assert _rel(r.A_H, o.A_H) <= 1e-10


def test_smooth_cp_input_135(dev):
    """3D smooth coefficient at 135^3 (the benchmark grid), given as CP
    factors and expanded on the device; oracle at the same size."""
    p = W.smooth_params(0)
    cp = W.smooth_cp(135, p)
    a, clipped = W.smooth_coeff(135, p)
    assert not clipped
    s = P.Solver(d=3, N=(135, 135, 135), format="full", solver_tol=1e-10, max_iter=200)
    r = s.solve(cp=(cp.weights, cp.factors))
    o = fg.solve(a, tol=1e-10)
    assert r.rc == 0
    assert _rel(r.A_H, o.A_H) <= 1e-10
    assert np.allclose(r.A_H, r.A_H.T, atol=1e-14)


def test_ball_243_properties(dev):
    """Ball of contrast 100 at 243^3: symmetric, isotropic, inside the
    Voigt/Reuss bounds (no oracle solve at this size)."""
    a = W.ball_coeff(243)
    r = _solve(a, 3, tol=1e-8, max_iter=1000)
    assert r.rc == 0
    A = r.A_H
    assert np.max(np.abs(A - A.T)) <= 1e-12 * A[0, 0]
    assert np.max(np.abs(A - np.diag(np.diag(A)))) <= 1e-8 * A[0, 0]
    assert np.ptp(np.diag(A)) <= 1e-8 * A[0, 0]
    reuss = 1.0 / np.mean(1.0 / a)
    voigt = np.mean(a)
    assert reuss < A[0, 0] < voigt
