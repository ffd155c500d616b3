"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the fact it checks; none re-types the oracle's formulas.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import brute, expsum, fg
from oracle import lowrank as L

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_kv(name):
    out = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


# ---------------------------------------------------------------- P1 constant
@pytest.mark.parametrize("d,N", [(2, 9), (3, 7)])
def test_constant_coefficient_is_exact(d, N):
    """GaNi is exact for constant coefficients (Sec. 2.2.2): A_H = a I and
    the right-hand side vanishes up to rounding."""
    a = W.constant_coeff(N, d, 3.25)
    r = fg.solve(a)
    assert np.allclose(r.A_H, 3.25 * np.eye(d), rtol=0, atol=1e-14)
    assert np.max(np.abs(fg.rhs(a, np.eye(d)[0]))) < 1e-14
    assert max(r.iters) <= 1


# ---------------------------------------------------------------- P2 laminate
@pytest.mark.parametrize("d,N,axis", [(2, 11, 0), (3, 9, 1), (3, 15, 2)])
def test_laminate_harmonic_and_arithmetic_means(d, N, axis):
    """Layers normal to x_axis: harmonic mean across, arithmetic mean along
    (exact for the discrete problem at any odd N)."""
    prof = np.random.default_rng(7).uniform(0.3, 8.0, N)
    a = W.laminate_coeff(N, d, prof, axis=axis)
    r = fg.solve(a, tol=1e-14, max_iter=500)
    H = 1.0 / np.mean(1.0 / prof)
    M = np.mean(prof)
    expect = np.eye(d) * M
    expect[axis, axis] = H
    assert np.allclose(r.A_H, expect, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- P3 bounds
def test_square_bounds_golden():
    g = _read_kv("square2d_N45_bounds.txt")
    a = W.square_coeff(45, d=2)
    x = W.grid_points(45)
    assert int(np.sum(np.abs(x) < 0.5 * np.sqrt(0.3))) == g["inside_points_per_axis"]
    assert np.isclose(np.mean(a), g["voigt"], rtol=1e-15)
    assert np.isclose(1.0 / np.mean(1.0 / a), g["reuss"], rtol=1e-15)
    r = fg.solve(a, tol=1e-12)
    ev = np.linalg.eigvalsh(r.A_H)
    assert g["reuss"] < ev.min() and ev.max() < g["voigt"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_voigt_reuss_random(seed):
    a = W.random_positive_coeff(9, 3, seed, 0.2, 20.0)
    r = fg.solve(a, tol=1e-12)
    ev = np.linalg.eigvalsh(0.5 * (r.A_H + r.A_H.T))
    assert 1.0 / np.mean(1.0 / a) <= ev.min() + 1e-12
    assert ev.max() <= np.mean(a) + 1e-12


# ---------------------------------------------------------------- P4 symmetry
def test_symmetric_geometries_are_isotropic():
    for a in (W.square_coeff(21, 2), W.square_coeff(15, 3), W.ball_coeff(15)):
        A = fg.solve(a, tol=1e-12).A_H
        d = a.ndim
        assert np.allclose(A, A.T, atol=1e-14)
        assert np.max(np.abs(A - np.diag(np.diag(A)))) < 1e-10
        assert np.ptp(np.diag(A)) < 1e-9


def test_energy_and_flux_forms_agree():
    a = W.random_positive_coeff(9, 3, 3)
    r = fg.solve(a, tol=1e-13)
    assert np.allclose(r.A_H, r.flux, atol=1e-11)


# ---------------------------------------------------------------- P5 duality
@pytest.mark.parametrize("N,seed", [(9, 0), (15, 1)])
def test_keller_duality_2d(N, seed):
    """2D: A_H[a] R A_H[1/a] R^T = I (R = 90 deg rotation), exact for odd-N
    GaNi because R maps gradient fields onto divergence-free ones."""
    a = W.random_positive_coeff(N, 2, seed, 0.2, 10.0)
    A = fg.solve(a, tol=1e-14, max_iter=1000).A_H
    B = fg.solve(1.0 / a, tol=1e-14, max_iter=1000).A_H
    R = np.array([[0.0, -1.0], [1.0, 0.0]])
    assert np.allclose(A @ R @ B @ R.T, np.eye(2), atol=1e-11)


def test_keller_duality_square_config():
    a_in = fg.solve(W.square_coeff(45, 2, inside=10.0), tol=1e-13).A_H[0, 0]
    a_out = fg.solve(W.square_coeff(45, 2, inside=0.1), tol=1e-13).A_H[0, 0]
    assert abs(a_in * a_out - 1.0) < 1e-11


# ---------------------------------------------------------------- P6 brute force
@pytest.mark.parametrize("d,N", [(2, 3), (2, 5), (2, 7), (3, 3), (3, 5)])
def test_brute_force_dense_assembly(d, N):
    a = W.random_positive_coeff(N, d, seed=10 + N + d, lo=0.3, hi=9.0)
    A1 = fg.solve(a, tol=1e-15, max_iter=2000).A_H
    A2 = brute.solve(a)
    assert np.max(np.abs(A1 - A2)) <= 1e-12 * np.max(np.abs(A2))


def test_nonbasis_E():
    """A_H E.E' is bilinear in E (checks the right-hand side's E scaling)."""
    a = W.random_positive_coeff(7, 3, 4)
    A = fg.solve(a, tol=1e-14).A_H
    E = [np.array([0.3, -1.2, 0.5]), np.array([1.0, 2.0, -0.7])]
    G = fg.solve(a, E, tol=1e-14).A_H
    assert np.allclose(G, np.array(E) @ A @ np.array(E).T, atol=1e-12)


# ---------------------------------------------------------------- P7 energy identity
def test_energy_identity_upper_bound():
    """A_{H,r} - A_H = ||u - u_r||_A^2 >= 0 for any approximate corrector
    (Sec. 4.3)."""
    a = W.random_positive_coeff(9, 3, 5)
    r = fg.solve(a, tol=1e-14)
    rng = np.random.default_rng(0)
    E = [np.eye(3)[0]]
    uh = r.u_hat[0]
    pert = fg.fwd(rng.standard_normal(a.shape)) * 0.01
    Ar = fg.energy_matrix(a, E, [uh + pert])[0, 0]
    gap = Ar - r.A_H[0, 0]
    assert gap > 0
    assert np.isclose(gap, fg.energy_norm_sq(a, pert), rtol=1e-9)


# ---------------------------------------------------------------- P11 spectrum
def test_preconditioned_spectrum_and_richardson():
    """spec(P^-1 K) on zero-mean fields lies in [min a, max a] (Sec. 3.3),
    so Richardson with omega = 2/(min a + max a) converges."""
    N, d = 5, 2
    a = W.random_positive_coeff(N, d, 11, 0.5, 4.0)
    n = a.size
    cols = []
    for i in range(n):             # operator on real nodal values
        e = np.zeros(n)
        e[i] = 1.0
        ch = fg.precond_diag(a.shape) * fg.apply_K(a, fg.fwd(e.reshape(a.shape)))
        cols.append(fg.inv(ch).reshape(-1))
    C = np.array(cols).T
    ev = np.linalg.eigvals(C).real
    ev = np.sort(ev)[1:]          # drop the constant-mode zero
    assert ev.min() >= a.min() - 1e-12 and ev.max() <= a.max() + 1e-12
    omega = 2.0 / (a.min() + a.max())
    bh = fg.rhs(a, [1.0, 0.0])
    Pinv = fg.precond_diag(a.shape)
    u = np.zeros_like(bh)
    d0 = np.linalg.norm(Pinv * bh)
    for _ in range(200):
        u = u + omega * Pinv * (bh - fg.apply_K(a, u))
    assert np.linalg.norm(Pinv * (bh - fg.apply_K(a, u))) < 1e-8 * d0


# ---------------------------------------------------------------- PCG history
def test_residual_history_monotone_end():
    a = W.square_coeff(45, 2)
    r = fg.solve(a, tol=1e-10)
    h = r.res_hist[0]
    assert h[-1] <= 1e-10 < h[-2]
    g = np.loadtxt(os.path.join(GOLD, "square2d_N45_AH.txt"))
    assert np.allclose(r.A_H, g, rtol=0, atol=1e-10)


# ---------------------------------------------------------------- low-rank pins
def test_square_rank_two_all_formats():
    """The square/cube coefficient has rank 2 in CP, Tucker and TT (Sec. 4.1)."""
    a2 = W.square_coeff(27, 2)
    s = np.linalg.svd(a2, compute_uv=False)
    assert np.sum(s > 1e-12 * s[0]) == 2
    a3 = W.square_coeff(15, 3)
    assert L.tt_ranks(L.tt_svd(a3, tol=1e-13)) == [1, 2, 2, 1]
    assert L.hosvd(a3, tol=1e-13).ranks == (2, 2, 2)
    cp = W.square_cp(15, 3)
    assert np.allclose(cp.full(), a3)


def test_laminate_rank_one_and_smooth_rank():
    prof = np.linspace(1, 3, 11)
    a = W.laminate_coeff(11, 3, prof)
    assert L.tt_ranks(L.tt_svd(a, tol=1e-13)) == [1, 1, 1, 1]
    p = W.smooth_params(0)
    a, clipped = W.smooth_coeff(21, p)
    assert not clipped
    rk = L.tt_ranks(L.tt_svd(a, tol=1e-13))
    assert max(rk) <= 9


@pytest.mark.parametrize("fmt", ["tt", "tucker", "cp"])
def test_hadamard_ranks_multiply(fmt):
    Ns = (5, 6, 7)
    x = W.random_cp(Ns, 3, 1)
    y = W.random_cp(Ns, 2, 2)
    X, Y = x.full(), y.full()
    if fmt == "cp":
        z = L.cp_hadamard(L.CP(x.weights, x.factors), L.CP(y.weights, y.factors))
        assert z.rank == 6
        assert np.allclose(z.full(), X * Y)
    elif fmt == "tt":
        a = L.tt_from_cp(L.CP(x.weights, x.factors))
        b = L.tt_from_cp(L.CP(y.weights, y.factors))
        z = L.tt_hadamard(a, b)
        assert L.tt_ranks(z) == [1, 6, 6, 1]
        assert np.allclose(L.tt_full(z), X * Y)
        s = L.tt_add(a, b)
        assert L.tt_ranks(s) == [1, 5, 5, 1]
        assert np.allclose(L.tt_full(s), X + Y)
    else:
        a = L.hosvd(X)
        b = L.hosvd(Y)
        z = L.tucker_hadamard(a, b)
        assert z.ranks == tuple(p * q for p, q in zip(a.ranks, b.ranks))
        assert np.allclose(z.full(), X * Y)
        s = L.tucker_add(a, b)
        assert np.allclose(s.full(), X + Y)


def test_dft_of_carriages_is_the_full_dft():
    """d-dim DFT = 1-D DFTs of the carriages; rank unchanged (Appendix A)."""
    cores = W.random_tt((5, 7, 9), [1, 3, 4, 1], 3)
    F = L.tt_dft(cores)
    assert L.tt_ranks(F) == [1, 3, 4, 1]
    X = L.tt_full(cores)
    assert np.allclose(L.tt_full(F), np.fft.fftn(X) / X.size)
    assert np.allclose(L.tt_full(L.tt_dft(F, inverse=True)), X)


def test_tt_round_error_bound_and_exactness():
    cores = W.random_tt((8, 9, 10), [1, 4, 5, 1], 4)
    big = L.tt_add(cores, L.tt_scale(cores, 0.5))      # rank 8, 10 but exact rank 4, 5
    r = L.tt_round(big, tol=1e-13)
    assert L.tt_ranks(r) == [1, 4, 5, 1]
    assert np.allclose(L.tt_full(r), 1.5 * L.tt_full(cores))
    X = L.tt_full(L.tt_add(cores, W.random_tt((8, 9, 10), [1, 4, 5, 1], 5)))
    full_cores = L.tt_svd(X)
    for tol in (1e-1, 3e-2):
        t = L.tt_round(full_cores, tol=tol)
        err = np.linalg.norm(L.tt_full(t) - X)
        assert err <= tol * np.linalg.norm(X) * (1 + 1e-12)


def test_cp2d_truncation_is_eckart_young():
    x = W.random_cp((30, 40), 12, 6)
    X = x.full()
    t = L.cp_truncate_2d(L.CP(x.weights, x.factors), 5)
    s = np.linalg.svd(X, compute_uv=False)
    assert np.isclose(np.linalg.norm(t.full() - X), np.sqrt(np.sum(s[5:] ** 2)), rtol=1e-10)


def test_tucker_truncation_bound():
    X = L.tt_full(W.random_tt((8, 9, 10), [1, 6, 6, 1], 8))
    h = L.hosvd(X)
    t = L.tucker_truncate(L.tucker_add(h, h), ranks=(4, 4, 4))
    err = np.linalg.norm(t.full() - 2 * X)
    c = L.hosvd(2 * X).c
    bound2 = 0.0
    for j in range(3):
        sl = np.sqrt(np.sum(np.moveaxis(c, j, 0).reshape(c.shape[j], -1) ** 2, axis=1))
        bound2 += np.sum(sl[4:] ** 2)
    assert err <= np.sqrt(bound2) * (1 + 1e-10)


def test_untruncated_lowrank_reproduces_full_solve():
    """Low-rank MR without truncation equals the full solve (TT, d = 3)."""
    a = W.square_coeff(9, 3, fraction=0.3)
    op = L.LowRankOperator(L.tt_svd(a, tol=1e-14), L.lowrank_precond_tt(a.shape),
                           rank_cap=1000, tol=1e-14)
    E = [1.0, 0.0, 0.0]
    u, hist = L.minimal_residual(op, E, max_iter=80, tol=1e-12)
    A_lr = L.energy_from_tt(a, [E], [u])[0, 0]
    A_f = fg.solve(a, [E], tol=1e-13).A_H[0, 0]
    assert abs(A_lr - A_f) <= 1e-10 * A_f


def test_truncated_lowrank_dominates_full():
    """Truncated solutions are energy upper bounds (Sec. 4.3)."""
    a = W.ball_coeff(11, inside=10.0)
    A_f = fg.solve(a, [[1, 0, 0]], tol=1e-13).A_H[0, 0]
    op = L.LowRankOperator(L.tt_svd(a, tol=1e-12), L.lowrank_precond_tt(a.shape),
                           rank_cap=2, tol=0.0)
    u, _ = L.minimal_residual(op, [1.0, 0.0, 0.0], max_iter=60)
    A_r = L.energy_from_tt(a, [[1, 0, 0]], [u])[0, 0]
    assert A_r >= A_f - 1e-12


# ---------------------------------------------------------------- exponential sums
@pytest.mark.parametrize("R,M,band", [(13467.0, 8, 0.12), (13467.0, 12, 0.02), (200.0, 6, 0.12), (200.0, 8, 0.03)])
def test_expsum_approximates_reciprocal(R, M, band):
    t, w = expsum.expsum_nodes(R, M)
    assert np.all(t > 0) and np.all(w > 0)
    y = np.exp(np.linspace(0.0, np.log(R), 4000))
    rel = expsum.expsum_eval(y, t, w) * y
    assert rel.min() > 1 - band and rel.max() < 1 + band


# ---------------------------------------------------------------- remaining format operations
def test_cp_add_expands_to_the_sum():
    """CP addition (Table 1: ranks add) expands to the sum of the expansions."""
    x = W.random_cp((6, 7, 8), 3, 11)
    y = W.random_cp((6, 7, 8), 4, 12)
    s = L.cp_add(L.CP(x.weights, x.factors), L.CP(y.weights, y.factors))
    assert s.rank == 7
    assert np.allclose(s.full(), x.full() + y.full(), rtol=0, atol=1e-12 * np.abs(x.full()).max())


@pytest.mark.parametrize("j", [0, 1, 2])
def test_tt_mode_apply_is_the_mode_product(j):
    """A matrix applied along the mode index of carriage j (rank unchanged)
    is numpy's mode-j product of the full tensor; with the spectral
    derivative F^-1 diag(2 pi i k) F as the matrix it is numpy's FFT
    derivative along axis j (Sec. 2.2.1, Appendix A.3)."""
    Ns = (5, 7, 9)
    cores = W.random_tt(Ns, [1, 3, 4, 1], 21)
    X = L.tt_full(cores)
    M = np.random.default_rng(j).standard_normal((Ns[j], Ns[j]))
    Y = L.tt_full(L.tt_mode_apply(cores, j, M))
    assert L.tt_ranks(L.tt_mode_apply(cores, j, M)) == [1, 3, 4, 1]
    assert np.allclose(Y, np.moveaxis(np.tensordot(M, X, axes=(1, j)), 0, j), atol=1e-12)
    n = Ns[j]
    k = np.fft.fftfreq(n, d=1.0 / n)
    D = np.real(np.fft.ifft(2j * np.pi * k[:, None] * np.fft.fft(np.eye(n), axis=0), axis=0))
    sh = [1, 1, 1]
    sh[j] = n
    want = np.real(np.fft.ifft(2j * np.pi * k.reshape(sh) * np.fft.fft(X, axis=j), axis=j))
    assert np.allclose(L.tt_full(L.tt_mode_apply(cores, j, D)), want, atol=1e-11)


@pytest.mark.parametrize("shape", [(15, 17, 19), (45, 45)])
def test_precond_symbol_approximates_inverse_laplacian(shape):
    """The separable preconditioner symbol is within the exponential sum's
    band of 1/(4 pi^2 |k|^2) at every nonzero frequency of the grid, and
    positive (Sec. 2.3, eq. Pls_GaNi_fourier)."""
    sym = expsum.precond_symbol(shape)
    d = len(shape)
    kk = 0.0
    for al, n in enumerate(shape):
        sh = [1] * d
        sh[al] = n
        kk = kk + (np.fft.fftfreq(n, d=1.0 / n) ** 2).reshape(sh)
    nz = kk > 0
    ratio = sym[nz] * (4 * np.pi ** 2) * kk[nz]
    assert np.all(sym > 0)
    assert ratio.min() > 0.88 and ratio.max() < 1.12
