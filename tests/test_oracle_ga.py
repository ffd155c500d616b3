"""Pins of the Ga (exact integration, double grid) oracle, Sec. 2.2.3.

The closed-form Fourier integrals against quadrature, the double-grid solve
against a dense Galerkin system assembled from the Fourier integrals alone
(no double grid, no FFT), nested-space monotonicity, the Voigt bound, the
constant coefficient and the symmetric geometries."""
import itertools

import numpy as np
import pytest
from scipy import integrate

from oracle import fg_ga as G


@pytest.mark.parametrize("m", [0, 1, 2, 5, 13])
def test_square_fourier_integral_by_quadrature(m):
    h = 0.3
    val, _ = integrate.quad(lambda x: np.cos(2 * np.pi * m * x), -h, h, epsabs=1e-14, epsrel=1e-14)
    assert abs(G.square_hat_1d(np.array([m]), h)[0] - val) < 1e-13


@pytest.mark.parametrize("rho", [0.0, 0.7, 1.0, np.sqrt(3.0), 5.0, 11.2])
def test_ball_fourier_integral_by_quadrature(rho):
    """Radial form of the ball's Fourier integral: int_0^R 4 pi r^2 sinc(2 rho r) dr."""
    R = 0.3
    f = lambda r: 4 * np.pi * r * r * np.sinc(2 * rho * r)
    val, _ = integrate.quad(f, 0.0, R, epsabs=1e-14, epsrel=1e-13, limit=200)
    assert abs(G.ball_hat(np.array([rho]), R)[0] - val) < 1e-12


def _dense_galerkin(inc, N, d):
    """Galerkin on T_N with exact integrals: K[l, k] = 4 pi^2 (k.l) A^(l - k),
    f[l] = 2 pi i (l.E) A^(l); A_H[i][j] = A^(0) E_i.E_j + sum_k u_j[k] 2 pi i
    (k.E_i) A^(-k) (Galerkin orthogonality)."""
    half = (N - 1) // 2
    ks = [np.array(k) for k in itertools.product(range(-half, half + 1), repeat=d) if any(k)]
    n = len(ks)
    K = np.zeros((n, n), dtype=complex)
    hat = lambda m: inc.hat([np.array([[mm]]).reshape([1] * d) for mm in m]).reshape(-1)[0]
    for a, l in enumerate(ks):
        for b, k in enumerate(ks):
            K[a, b] = 4 * np.pi ** 2 * np.dot(k, l) * hat(l - k)
    A = np.zeros((d, d))
    us = []
    for i in range(d):
        E = np.eye(d)[i]
        f = np.array([2j * np.pi * np.dot(l, E) * hat(l) for l in ks])
        us.append(np.linalg.solve(K, f))
    for i in range(d):
        Ei = np.eye(d)[i]
        for j in range(d):
            Ej = np.eye(d)[j]
            s = hat(np.zeros(d, dtype=int)) * np.dot(Ei, Ej)
            s += sum(us[j][b] * 2j * np.pi * np.dot(k, Ei) * hat(-k) for b, k in enumerate(ks))
            A[i, j] = s.real
    return A


@pytest.mark.parametrize("shape,d,N", [("square", 2, 5), ("square", 2, 7), ("square", 3, 3), ("ball", 3, 3),
                                       ("ball", 3, 5)])
def test_double_grid_equals_dense_galerkin(shape, d, N):
    inc = G.Inclusion(shape, 0.3, 10.0, 1.0)
    A1 = G.solve(inc, [N] * d, tol=1e-15, max_iter=2000).A_H
    A2 = _dense_galerkin(inc, N, d)
    assert np.max(np.abs(A1 - A2)) <= 1e-12 * np.max(np.abs(A2))


@pytest.mark.parametrize("shape,d,N,M", [("square", 2, 5, 15), ("square", 2, 7, 25), ("ball", 3, 3, 9),
                                         ("square", 3, 5, 15)])
def test_larger_double_grid_is_the_same_galerkin_system(shape, d, N, M):
    """Any odd double grid of at least 2N - 1 points integrates the products
    of T_N's gradients exactly, so the solve on M (here the smallest odd
    3^a 5^b >= 2N - 1, as the GPU path takes it, and 3^a 5^b above that)
    is the dense Galerkin solve."""
    inc = G.Inclusion(shape, 0.3, 10.0, 1.0)
    A1 = G.solve(inc, [N] * d, tol=1e-15, max_iter=2000, M=[M] * d).A_H
    A2 = _dense_galerkin(inc, N, d)
    assert np.max(np.abs(A1 - A2)) <= 1e-12 * np.max(np.abs(A2))


def test_double_grid_below_2n_minus_1_rejected():
    with pytest.raises(ValueError):
        G.coefficient_on_double_grid(G.Inclusion("square", 0.3, 10.0, 1.0), [5, 5], [7, 9])


def test_nested_spaces_decrease_the_energy():
    """T_N is contained in T_{N+2}: the Galerkin energy minimum can only fall."""
    inc = G.Inclusion("square", 0.3, 10.0, 1.0)
    prev = None
    for N in (5, 7, 9, 15, 25):
        A = G.solve(inc, [N, N], tol=1e-13).A_H
        if prev is not None:
            assert np.linalg.eigvalsh(prev - A).min() >= -1e-12
        prev = A


@pytest.mark.parametrize("shape,d", [("square", 2), ("square", 3), ("ball", 3)])
def test_voigt_bound_and_symmetry(shape, d):
    inc = G.Inclusion(shape, 0.3, 10.0, 1.0)
    A = G.solve(inc, [11] * d, tol=1e-13).A_H
    mean = inc.hat([np.zeros([1] * d, dtype=int)] * d).reshape(-1)[0]
    assert np.linalg.eigvalsh(mean * np.eye(d) - A).min() > 0
    assert np.max(np.abs(A - np.diag(np.diag(A)))) < 1e-12
    assert np.ptp(np.diag(A)) < 1e-11


def test_constant_coefficient_is_exact():
    inc = G.Inclusion("ball", 0.3, 2.5, 2.5)
    r = G.solve(inc, [7, 7, 7])
    assert np.allclose(r.A_H, 2.5 * np.eye(3), rtol=0, atol=1e-14)
    assert max(r.iters) == 0
