"""Full-grid GaNi solve with a matrix-valued coefficient, FP64, CPU -- oracle
(test infrastructure).

Sec. 4.4 of the paper turns the isotropic materials a(x) I into anisotropic
ones by adding a spatially constant symmetric positive definite matrix B:
A~(x) = a(x) I + B.  The homogenisation problem (Sec. 2.1, eq. homog) and
its GaNi discretisation (Sec. 2.2.2, eq. ls_GaNi_fourier) are unchanged
except that the material law multiplies the gradient by the d x d matrix
A(x) at every grid point:

    K u^ = grad*^ F A F^-1 grad^ u^ ,   b^ = - grad*^ F (A E),
    A_H E.E' = mean_x A (E + grad u_E).(E' + grad u_E').

This module takes the coefficient as d x d nodal fields A[alpha][beta]
(any symmetric positive definite field, not only a I + B), so the pins can
use general tensor laminates.  The Fourier transforms, the gradient and
divergence symbols and the Laplacian preconditioner are those of
`oracle.fg` (Sec. 2.2-2.3); the CG iteration is the same preconditioned CG,
written here over an operator argument.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence

import numpy as np

from . import fg


def isotropic_plus_constant(a: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Nodal fields of A~(x) = a(x) I + B (Sec. 4.4), shape (d, d, *a.shape)."""
    a = np.asarray(a, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    d = a.ndim
    A = np.empty((d, d) + a.shape)
    for al in range(d):
        for be in range(d):
            A[al, be] = B[al, be] + (a if al == be else 0.0)
    return A


def material_law(A: np.ndarray, g: Sequence[np.ndarray]) -> List[np.ndarray]:
    """h_alpha = sum_beta A[alpha][beta] g_beta at every grid point."""
    d = A.shape[0]
    return [sum(A[al, be] * g[be] for be in range(d)) for al in range(d)]


def apply_K(A: np.ndarray, uh: np.ndarray) -> np.ndarray:
    """K u^ = grad*^ F (A F^-1 grad^ u^)."""
    g = [fg.inv(gh) for gh in fg.grad_hat(uh)]
    return fg.div_hat([fg.fwd(h) for h in material_law(A, g)])


def rhs(A: np.ndarray, E: Sequence[float]) -> np.ndarray:
    """b^ = - grad*^ F (A E)."""
    d = A.shape[0]
    shape = A.shape[2:]
    const = [np.full(shape, float(E[be])) for be in range(d)]
    return -fg.div_hat([fg.fwd(h) for h in material_law(A, const)])


def pcg(op: Callable[[np.ndarray], np.ndarray], bh: np.ndarray, tol: float,
        max_iter: int, floor: float):
    """Preconditioned CG on op(u^) = b^ with the Laplacian pseudo-inverse,
    stopped on the relative norm of the preconditioned residual (Sec. 4.2);
    a preconditioned right-hand side below `floor` is zero up to rounding."""
    Pinv = fg.precond_diag(bh.shape)
    x = np.zeros_like(bh)
    r = bh.copy()
    z = Pinv * r
    z0 = np.sqrt(fg.dot(z, z))
    hist: List[float] = []
    if z0 <= floor:
        return x, 0, hist
    p = z.copy()
    rho = fg.dot(r, z)
    it = 0
    while it < max_iter:
        q = op(p)
        alpha = rho / fg.dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        z = Pinv * r
        it += 1
        zn = np.sqrt(fg.dot(z, z))
        hist.append(zn / z0)
        if zn / z0 <= tol or zn <= floor:
            break
        rho_new = fg.dot(r, z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, it, hist


def energy_matrix(A: np.ndarray, Es: Sequence[Sequence[float]],
                  uhs: Sequence[np.ndarray]) -> np.ndarray:
    """A_H E_i.E_j = mean_x A (E_i + grad u_i).(E_j + grad u_j)  (eq. homog)."""
    d = A.shape[0]
    fields = []
    for E, uh in zip(Es, uhs):
        g = fg.gradient_field(uh)
        fields.append([float(E[al]) + g[al] for al in range(d)])
    nE = len(Es)
    out = np.zeros((nE, nE))
    for i in range(nE):
        flux = material_law(A, fields[i])
        for j in range(nE):
            out[i, j] = np.mean(sum(flux[al] * fields[j][al] for al in range(d)))
    return out


@dataclasses.dataclass
class TensorResult:
    A_H: np.ndarray
    iters: List[int]
    res_hist: List[List[float]]
    u_hat: List[np.ndarray]


def solve(A: np.ndarray, Es: Optional[Sequence[Sequence[float]]] = None,
          tol: float = 1e-10, max_iter: int = 1000) -> TensorResult:
    """Homogenised matrix of a matrix-valued coefficient A (shape (d, d, N..))."""
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[0]
    shape = A.shape[2:]
    if A.shape[1] != d or len(shape) != d:
        raise ValueError("coefficient must have shape (d, d, N_1, .., N_d)")
    if any(n % 2 == 0 for n in shape):
        raise ValueError("odd grid sizes only (Sec. 2.2.1)")
    if Es is None:
        Es = [np.eye(d)[i] for i in range(d)]
    rms = float(np.sqrt(np.mean(np.sum(A * A, axis=(0, 1)))))
    uhs, iters, hists = [], [], []
    for E in Es:
        bh = rhs(A, E)
        floor = fg.ROUNDING_FLOOR * rms * float(np.linalg.norm(np.asarray(E, dtype=np.float64)))
        uh, it, hist = pcg(lambda v: apply_K(A, v), bh, tol, max_iter, floor)
        uhs.append(uh)
        iters.append(it)
        hists.append(hist)
    return TensorResult(energy_matrix(A, Es, uhs), iters, hists, uhs)
