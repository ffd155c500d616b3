"""Full-grid GaNi Fourier-Galerkin solve, FP64, CPU -- oracle (test infrastructure).

Follows the paper, Sec. 2 (model problem and Fourier-Galerkin method):

* discretisation with trigonometric polynomials on an odd grid N^d
  (Sec. 2.2.1), DFT matrices with the 1/|N| factor on the forward transform;
* GaNi (rectangle-rule) bilinear form (Sec. 2.2.2); the quadrature weight
  1/|N| is taken as a grid mean so that a constant coefficient A gives
  A_H = A exactly;
* the linear system in Fourier space, eq. (ls_GaNi_fourier):
      grad*^ F A F^-1 grad^ u^ = - grad*^ F A E,
  with grad^ = 2 pi i k and grad*^ = sum_alpha -2 pi i k_alpha;
* the Laplacian preconditioner of Sec. 2.3, eq. (Pls_GaNi_fourier): the
  pseudo-inverse of diag(k.k), zero at k = 0.  The 4 pi^2 factor is
  included (it rescales the preconditioned spectrum onto [min a, max a] and
  leaves every CG iterate unchanged);
* preconditioned conjugate gradients (Sec. 3.3 and Sec. 4: the full system
  is solved by CG), stopped when the Euclidean norm of the preconditioned
  residual's Fourier coefficients (Sec. 4.2) falls below tol times its
  initial value;
* A_H from eq. (homog): A_H E.E' = mean_x a (E + grad u_E).(E' + grad u_E').

Storage: nodal values are indexed j in [0, N) along each axis; numpy's FFT
over that index differs from the paper's centred-index DFT by a phase per
frequency which cancels between F and F^-1, so the solution's nodal values
and A_H are those of the paper's system.

Scalar isotropic coefficients A = a(x) I only.
"""
from __future__ import annotations

import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np
import scipy.fft as sfft

# FFTs on every host core (pocketfft threads); the results are those of the
# single-threaded transform up to rounding.
FFT_WORKERS = os.cpu_count() or 1


def frequencies(N: int) -> np.ndarray:
    """Integer frequencies k of an odd-N axis in FFT storage order."""
    return np.fft.fftfreq(N, d=1.0 / N).round().astype(np.float64)


def _kgrid(shape: Sequence[int]) -> List[np.ndarray]:
    d = len(shape)
    out = []
    for alpha, n in enumerate(shape):
        sh = [1] * d
        sh[alpha] = n
        out.append(frequencies(n).reshape(sh))
    return out


def fwd(v: np.ndarray) -> np.ndarray:
    """F_N: forward DFT with the 1/|N| factor."""
    return sfft.fftn(v, workers=FFT_WORKERS) / v.size


def inv(vh: np.ndarray) -> np.ndarray:
    """F_N^-1: unnormalised inverse DFT; fields here are real."""
    return sfft.ifftn(vh, workers=FFT_WORKERS).real * vh.size


def grad_hat(uh: np.ndarray) -> List[np.ndarray]:
    """grad^ u^ = 2 pi i k_alpha u^ for each alpha."""
    return [2j * np.pi * k * uh for k in _kgrid(uh.shape)]


def div_hat(wh: Sequence[np.ndarray]) -> np.ndarray:
    """grad*^ w^ = sum_alpha -2 pi i k_alpha w^_alpha."""
    ks = _kgrid(wh[0].shape)
    return sum(-2j * np.pi * k * w for k, w in zip(ks, wh))


def apply_K(a: np.ndarray, uh: np.ndarray) -> np.ndarray:
    """K u^ = grad*^ F (a F^-1 grad^ u^)   (left side of eq. ls_GaNi_fourier)."""
    return div_hat([fwd(a * inv(g)) for g in grad_hat(uh)])


def rhs(a: np.ndarray, E: Sequence[float]) -> np.ndarray:
    """b^ = - grad*^ F (a E)   (right side of eq. ls_GaNi_fourier)."""
    return -div_hat([fwd(a * float(e)) for e in E])


def precond_diag(shape: Sequence[int]) -> np.ndarray:
    """Pseudo-inverse of the Fourier Laplacian 4 pi^2 k.k, zero at k = 0."""
    ks = _kgrid(shape)
    kk = sum(k * k for k in ks) * (4.0 * np.pi ** 2)
    out = np.zeros(shape)
    nz = kk != 0
    out[nz] = 1.0 / kk[nz]
    return out


def dot(x: np.ndarray, y: np.ndarray) -> float:
    """Real part of sum conj(x) y over all Fourier coefficients."""
    return float(np.real(np.vdot(x, y)))


@dataclasses.dataclass
class FGResult:
    A_H: np.ndarray              # (nE, nE) energy Gram matrix A_H E_i.E_j
    iters: List[int]
    res_hist: List[List[float]]  # relative preconditioned residual norms
    u_hat: List[np.ndarray]      # Fourier coefficients of each corrector
    flux: np.ndarray             # (nE, d) mean of a (E + grad u), consistency only


ROUNDING_FLOOR = 1e-14


def pcg(a: np.ndarray, bh: np.ndarray, tol: float, max_iter: int,
        scale: float = 1.0):
    """Preconditioned CG on K u^ = b^ with the Laplacian pseudo-inverse.

    A right-hand side whose preconditioned norm is below
    ROUNDING_FLOOR * scale (scale = rms(a) |E|) is zero up to rounding (for
    instance E along the layers of a laminate): the corrector is zero and no
    iteration runs.  The same floor ends the iteration if the residual
    reaches it before the relative tolerance."""
    Pinv = precond_diag(a.shape)
    x = np.zeros_like(bh)
    r = bh.copy()
    z = Pinv * r
    z0 = np.sqrt(dot(z, z))
    hist = []
    floor = ROUNDING_FLOOR * scale
    if z0 <= floor:
        return x, 0, hist
    p = z.copy()
    rho = dot(r, z)
    it = 0
    while it < max_iter:
        q = apply_K(a, p)
        alpha = rho / dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        z = Pinv * r
        it += 1
        zn = np.sqrt(dot(z, z))
        rel = zn / z0
        hist.append(rel)
        if rel <= tol or zn <= floor:
            break
        rho_new = dot(r, z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, it, hist


def gradient_field(uh: np.ndarray) -> List[np.ndarray]:
    """Nodal values of grad u from its Fourier coefficients (eq. grad_trig)."""
    return [inv(g) for g in grad_hat(uh)]


def energy_matrix(a: np.ndarray, Es: Sequence[Sequence[float]],
                  uhs: Sequence[np.ndarray]) -> np.ndarray:
    """A_H E_i.E_j = mean_x a (E_i + grad u_i).(E_j + grad u_j)  (eq. homog)."""
    fields = []
    for E, uh in zip(Es, uhs):
        g = gradient_field(uh)
        fields.append([float(E[al]) + g[al] for al in range(a.ndim)])
    nE = len(Es)
    A = np.zeros((nE, nE))
    for i in range(nE):
        for j in range(nE):
            A[i, j] = np.mean(a * sum(fields[i][al] * fields[j][al]
                                      for al in range(a.ndim)))
    return A


def solve(a: np.ndarray, Es: Optional[Sequence[Sequence[float]]] = None,
          tol: float = 1e-10, max_iter: int = 1000) -> FGResult:
    """Homogenised matrix of a scalar coefficient field a (nodal values)."""
    a = np.asarray(a, dtype=np.float64)
    d = a.ndim
    if any(n % 2 == 0 for n in a.shape):
        raise ValueError("odd grid sizes only (Sec. 2.2.1)")
    if Es is None:
        Es = [np.eye(d)[i] for i in range(d)]
    uhs, iters, hists = [], [], []
    rms = float(np.sqrt(np.mean(a * a)))
    for E in Es:
        bh = rhs(a, E)
        scale = rms * float(np.linalg.norm(np.asarray(E, dtype=np.float64)))
        uh, it, hist = pcg(a, bh, tol, max_iter, scale)
        uhs.append(uh)
        iters.append(it)
        hists.append(hist)
    A = energy_matrix(a, Es, uhs)
    flux = np.zeros((len(Es), d))
    for i, (E, uh) in enumerate(zip(Es, uhs)):
        g = gradient_field(uh)
        for al in range(d):
            flux[i, al] = np.mean(a * (float(E[al]) + g[al]))
    return FGResult(A, iters, hists, uhs, flux)


def energy_norm_sq(a: np.ndarray, uh: np.ndarray) -> float:
    """a(grad u, grad u) as a grid mean (energy semi-norm squared)."""
    g = gradient_field(uh)
    return float(np.mean(a * sum(gi * gi for gi in g)))
