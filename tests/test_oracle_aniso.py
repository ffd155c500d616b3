"""Pins of the matrix-valued oracle (the anisotropic materials of Sec. 4.4).

Each test names the fact it checks: closed forms of the discrete problem
(constant and laminated tensors), an independent dense assembly, the
Voigt/Reuss bounds, 2D duality and reflection covariance.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import brute, fg
from oracle import fg_tensor as FT

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kv(name):
    out = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


def _random_spd(d, rng, lo=0.3, hi=6.0):
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    return Q @ np.diag(rng.uniform(lo, hi, d)) @ Q.T


def test_paper_B_matrices_have_the_stated_eigenvalues():
    g = _kv("aniso_B.txt")
    s2 = math.sqrt(2.0)
    B2 = np.array([[g["B2_00"], g["B2_01"]], [g["B2_01"], g["B2_11"]]])
    B3 = np.array([[g["B3_00"], g["B3_01"], g["B3_02_over_s2"] * s2],
                   [g["B3_01"], g["B3_11"], g["B3_12_over_s2"] * s2],
                   [g["B3_02_over_s2"] * s2, g["B3_12_over_s2"] * s2, g["B3_22"]]])
    assert np.allclose(np.linalg.eigvalsh(B2), [g["B2_eig0"], g["B2_eig1"]], atol=1e-13)
    assert np.allclose(np.linalg.eigvalsh(B3), [g["B3_eig0"], g["B3_eig1"], g["B3_eig2"]], atol=1e-13)
    assert np.array_equal(W.anisotropy(2), B2)
    assert np.allclose(W.anisotropy(3), B3, rtol=0, atol=1e-15)


@pytest.mark.parametrize("d,N", [(2, 9), (3, 7)])
def test_constant_tensor_is_exact(d, N):
    """A constant matrix coefficient: zero right-hand side, A_H = A."""
    A0 = 2.0 * np.eye(d) + W.anisotropy(d)
    A = FT.isotropic_plus_constant(W.constant_coeff(N, d, 2.0), W.anisotropy(d))
    r = FT.solve(A)
    assert np.allclose(r.A_H, A0, rtol=0, atol=1e-13)
    assert max(r.iters) == 0


def _laminate_closed_form(layers, axis, d):
    """Tensor laminate normal to e_axis: the corrector gradient is c_E(x) e_axis
    with A_aa c_E + (A E)_a constant and c_E of zero mean, so
    c_E = (lam_E - (A E)_a)/A_aa with lam_E = mean((A E)_a/A_aa)/mean(1/A_aa)."""
    N = len(layers)
    out = np.zeros((d, d))
    fields = []
    for i in range(d):
        E = np.eye(d)[i]
        AE = np.array([L @ E for L in layers])            # (N, d)
        Aaa = np.array([L[axis, axis] for L in layers])
        lam = np.mean(AE[:, axis] / Aaa) / np.mean(1.0 / Aaa)
        c = (lam - AE[:, axis]) / Aaa
        F = np.tile(E, (N, 1))
        F[:, axis] += c
        fields.append(F)
    for i in range(d):
        for j in range(d):
            out[i, j] = np.mean([fields[j][n] @ layers[n] @ fields[i][n] for n in range(N)])
    return out


@pytest.mark.parametrize("d,N,axis", [(2, 11, 0), (2, 9, 1), (3, 9, 2), (3, 7, 0)])
def test_tensor_laminate_closed_form(d, N, axis):
    """Layers of arbitrary SPD matrices normal to x_axis: the discrete
    minimiser is invariant along the layers (as for the scalar laminate),
    which gives A_H in closed form, off-diagonal entries included."""
    rng = np.random.default_rng(20 + 3 * d + axis)
    layers = [_random_spd(d, rng) for _ in range(N)]
    A = np.empty((d, d) + (N,) * d)
    sh = [1] * d
    sh[axis] = N
    for al in range(d):
        for be in range(d):
            prof = np.array([L[al, be] for L in layers]).reshape(sh)
            A[al, be] = np.broadcast_to(prof, (N,) * d)
    r = FT.solve(A, tol=1e-14, max_iter=400)
    expect = _laminate_closed_form(layers, axis, d)
    assert np.allclose(r.A_H, expect, rtol=0, atol=1e-12 * np.max(np.abs(expect)))
    assert np.max(np.abs(expect - expect.T)) < 1e-13


@pytest.mark.parametrize("d,N", [(2, 3), (2, 5), (2, 7), (3, 3), (3, 5)])
def test_tensor_brute_force_dense_assembly(d, N):
    rng = np.random.default_rng(40 + 5 * N + d)
    a = W.random_positive_coeff(N, d, seed=50 + N + d, lo=0.3, hi=9.0)
    A = FT.isotropic_plus_constant(a, _random_spd(d, rng, 0.1, 3.0))
    A1 = FT.solve(A, tol=1e-15, max_iter=2000).A_H
    A2 = brute.solve_tensor(A)
    assert np.max(np.abs(A1 - A2)) <= 1e-12 * np.max(np.abs(A2))


@pytest.mark.parametrize("d,N", [(2, 15), (3, 9)])
def test_tensor_voigt_reuss(d, N):
    """mean(A^-1)^-1 <= A_H <= mean(A) in the PSD sense."""
    a = W.random_positive_coeff(N, d, seed=60 + d, lo=0.2, hi=20.0)
    A = FT.isotropic_plus_constant(a, W.anisotropy(d))
    AH = FT.solve(A, tol=1e-13).A_H
    voigt = np.mean(A.reshape(d, d, -1), axis=2)
    inv = np.linalg.inv(np.moveaxis(A.reshape(d, d, -1), 2, 0))
    reuss = np.linalg.inv(np.mean(inv, axis=0))
    assert np.linalg.eigvalsh(voigt - AH).min() > -1e-11
    assert np.linalg.eigvalsh(AH - reuss).min() > -1e-11


@pytest.mark.parametrize("N,seed", [(9, 0), (15, 1)])
def test_tensor_duality_2d(N, seed):
    """2D: the effective matrix of R A(x)^-1 R^T is R A_H^-1 R^T (R = 90 deg
    rotation), exact for odd-N GaNi: R maps gradient fields onto the
    divergence-free ones."""
    a = W.random_positive_coeff(N, 2, seed, 0.2, 10.0)
    A = FT.isotropic_plus_constant(a, W.anisotropy(2))
    R = np.array([[0.0, -1.0], [1.0, 0.0]])
    Ainv = np.linalg.inv(np.moveaxis(A.reshape(2, 2, -1), 2, 0))   # (n, 2, 2)
    dual = np.moveaxis(R @ Ainv @ R.T, 0, 2).reshape(A.shape)
    AH = FT.solve(A, tol=1e-14, max_iter=1000).A_H
    DH = FT.solve(dual, tol=1e-14, max_iter=1000).A_H
    assert np.allclose(DH, R @ np.linalg.inv(AH) @ R.T, atol=1e-11)


def test_reflection_covariance():
    """Reflecting x_1 -> -x_1 (a symmetric ball) maps B to S B S and A_H to
    S A_H S with S = diag(-1, 1, 1): the signs of the off-diagonal entries
    in row and column 1 flip, the rest is unchanged."""
    a = W.ball_coeff(9, inside=10.0)
    B = W.anisotropy(3)
    S = np.diag([-1.0, 1.0, 1.0])
    A1 = FT.solve(FT.isotropic_plus_constant(a, B), tol=1e-13).A_H
    A2 = FT.solve(FT.isotropic_plus_constant(a, S @ B @ S), tol=1e-13).A_H
    assert np.allclose(A2, S @ A1 @ S, atol=1e-11)
    assert abs(A1[0, 1]) > 1.0     # the anisotropy really couples the axes


def test_zero_B_reduces_to_the_scalar_oracle():
    a = W.random_positive_coeff(9, 3, 7)
    A = FT.isotropic_plus_constant(a, np.zeros((3, 3)))
    assert np.allclose(FT.solve(A, tol=1e-13).A_H, fg.solve(a, tol=1e-13).A_H, atol=1e-12)


# ---------------------------------------------------------------- material S
@pytest.mark.parametrize("d,n,k2", [(2, 20, {1, 2, 4, 5}), (3, 26, {1, 2, 3})])
def test_material_s_modes(d, n, k2):
    """Sec. 4.1: 20 modes in 2D and 26 in 3D, the lowest frequencies (cos and
    sin of one k per pair +-k), coefficients in [-0.5, 0.5]."""
    p = W.material_s_params(d, seed=3)
    assert len(p.c) == n and np.all(np.abs(p.c) <= 0.5)
    assert {int(k @ k) for k in p.ks} == k2
    pairs = {(tuple(k), int(t)) for k, t in zip(p.ks, p.kinds)}
    assert len(pairs) == n                                   # no mode twice
    assert all(tuple(-k) not in {tuple(q) for q in p.ks} for k in p.ks)


def test_material_s_range_and_periodicity():
    a = W.material_s(27, 3, seed=0)
    assert np.isclose(a.min(), 1.0) and np.isclose(a.max(), 10.0)
    # the exponent is a trigonometric polynomial of degree 1 per axis and
    # |k|^2 <= 3: log a has no Fourier content beyond it
    la = np.log(a)
    spec = np.fft.fftn(la) / la.size
    k = np.fft.fftfreq(27, d=1 / 27)
    K2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    assert np.max(np.abs(spec[K2 > 3])) < 1e-12
