"""Full-grid Fourier-Galerkin solve with exact integration (Ga), FP64, CPU --
oracle (test infrastructure).

Sec. 2.2.3 of the paper: the Galerkin approximation on the trigonometric
polynomials T_N with the bilinear form integrated exactly, made sparse by
double-grid integration with projection (DoGIP):

    grad*^_N I* F_M  A_M  F_M^-1 I grad^_N u^ = - grad*^_N I* F_M A_M E,

with M = 2N - 1 per axis, I the zero-padding injection of N-frequencies into
M-frequencies and I* its adjoint (restriction), and A_M the nodal values on
the M grid of the coefficient's Fourier series truncated to |m_alpha| <= N - 1
(the coefficients A[k] = integral of A against the double grid's
fundamental trigonometric polynomials).  The product of two gradients of T_N
lies in T_M, whose grid mean is its exact integral, so the bilinear form and
the energy form of eq. (homog) are exact.  Preconditioner: the Laplacian
pseudo-inverse of Sec. 2.3 on the N-frequencies (eq. Pls_Ga_fourier).

Coefficients are inclusions with closed-form Fourier integrals: the centred
square (2D) or cube (3D) |x_alpha| < h and the centred ball |x| < R (3D), with
value `inside` in the inclusion and `outside` elsewhere.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import fg, fg_tensor


def square_hat_1d(m: np.ndarray, half: float) -> np.ndarray:
    """Integral over (-1/2, 1/2) of the indicator of |x| < half times
    exp(-2 pi i m x): 2 half at m = 0, sin(2 pi m half) / (pi m) otherwise."""
    m = np.asarray(m, dtype=np.float64)
    out = np.empty_like(m)
    z = m == 0
    out[z] = 2.0 * half
    out[~z] = np.sin(2.0 * np.pi * m[~z] * half) / (np.pi * m[~z])
    return out


def ball_hat(rho: np.ndarray, radius: float) -> np.ndarray:
    """Fourier integral of the indicator of |x| < R in 3D at frequency
    vectors of length rho: (sin z - z cos z) / (2 pi^2 rho^3), z = 2 pi R rho;
    4 pi R^3 / 3 at rho = 0 (the ball lies inside the cell for R < 1/2)."""
    rho = np.asarray(rho, dtype=np.float64)
    out = np.empty_like(rho)
    z0 = rho == 0
    out[z0] = 4.0 * np.pi * radius ** 3 / 3.0
    r = rho[~z0]
    z = 2.0 * np.pi * radius * r
    out[~z0] = (np.sin(z) - z * np.cos(z)) / (2.0 * np.pi ** 2 * r ** 3)
    return out


@dataclasses.dataclass
class Inclusion:
    shape: str          # "square" (2D square / 3D cube) or "ball" (3D)
    size: float         # half side or radius
    inside: float
    outside: float

    def hat(self, ms: Sequence[np.ndarray]) -> np.ndarray:
        """Exact Fourier coefficients A^(m) on the broadcast frequency grids ms."""
        d = len(ms)
        shape = np.broadcast(*ms).shape
        if self.shape == "square":
            chi = np.ones(shape)
            for m in ms:
                chi = chi * square_hat_1d(np.broadcast_to(m, shape), self.size)
        elif self.shape == "ball":
            if d != 3:
                raise ValueError("the ball is a 3D inclusion")
            rho = np.sqrt(sum(np.broadcast_to(np.asarray(m, dtype=np.float64), shape) ** 2 for m in ms))
            chi = ball_hat(rho, self.size)
        else:
            raise ValueError(self.shape)
        out = (self.inside - self.outside) * chi
        at_zero = np.ones(shape, dtype=bool)
        for m in ms:
            at_zero &= np.broadcast_to(m, shape) == 0
        out[at_zero] += self.outside          # the constant: A^(0) only
        return out


def double_grid(N: Sequence[int]) -> List[int]:
    """The paper's double grid 2N - 1: the smallest odd grid whose mean
    integrates T_{2N-1} (the products of two gradients of T_N) exactly.  Any
    odd M >= 2N - 1 does as well and gives the same system; `solve` takes
    such an M as an option."""
    return [2 * n - 1 for n in N]


def coefficient_on_double_grid(inc: Inclusion, N: Sequence[int],
                               M: Optional[Sequence[int]] = None) -> np.ndarray:
    """A_M: values at the M-grid points x_j = -1/2 + (j + 1/2)/M of the
    Fourier series of the coefficient truncated to |m_alpha| <= N_alpha - 1
    (M odd, at least 2N - 1; default 2N - 1)."""
    M = double_grid(N) if M is None else list(M)
    d = len(N)
    for n, mm in zip(N, M):
        if mm % 2 == 0 or mm < 2 * n - 1:
            raise ValueError("the double grid must be odd and at least 2N - 1")
    ms = []
    for a, mm in enumerate(M):
        sh = [1] * d
        sh[a] = mm
        ms.append(np.arange(-(mm // 2), mm // 2 + 1).reshape(sh))  # centred order
    Ahat = inc.hat(ms)
    keep = np.ones(Ahat.shape, dtype=bool)
    for m, n in zip(ms, N):
        keep &= np.abs(np.broadcast_to(m, Ahat.shape)) <= n - 1
    Ahat = np.where(keep, Ahat, 0.0)
    # sum_m A^(m) exp(2 pi i m x_j) over centred m and centred x: an inverse
    # DFT between centred orders (ifftshift / fftshift around numpy's ifftn)
    vals = np.fft.fftshift(np.fft.ifftn(np.fft.ifftshift(Ahat))) * float(np.prod(M))
    return vals.real


def pad(vh: np.ndarray, M: Sequence[int]) -> np.ndarray:
    """I: N-frequencies (FFT storage order) into M-frequencies, zeros elsewhere."""
    out = np.zeros(tuple(M), dtype=complex)
    idx = []
    for n, mm in zip(vh.shape, M):
        f = fg.frequencies(n).astype(int)
        idx.append(np.mod(f, mm))
    out[np.ix_(*idx)] = vh
    return out


def restrict(vh: np.ndarray, N: Sequence[int]) -> np.ndarray:
    """I*: keep the N-frequencies of an M-spectrum (FFT storage order)."""
    idx = []
    for n, mm in zip(N, vh.shape):
        f = fg.frequencies(n).astype(int)
        idx.append(np.mod(f, mm))
    return vh[np.ix_(*idx)]


def apply_K(AM: np.ndarray, uh: np.ndarray) -> np.ndarray:
    """grad*^ I* F_M A_M F_M^-1 I grad^ u^  (left side of eq. ls_Ga_fourier)."""
    M = AM.shape
    out = []
    for g in fg.grad_hat(uh):
        out.append(restrict(fg.fwd(AM * fg.inv(pad(g, M))), uh.shape))
    return fg.div_hat(out)


def rhs(AM: np.ndarray, N: Sequence[int], E: Sequence[float]) -> np.ndarray:
    """- grad*^ I* F_M (A_M E)."""
    return -fg.div_hat([restrict(fg.fwd(AM * float(e)), N) for e in E])


def energy_matrix(AM: np.ndarray, Es, uhs) -> np.ndarray:
    """A_H E_i.E_j = integral of A (E_i + grad u_i).(E_j + grad u_j), as the
    M-grid mean with A_M (exact for gradients in T_N)."""
    M = AM.shape
    d = AM.ndim
    fields = []
    for E, uh in zip(Es, uhs):
        g = [fg.inv(pad(gh, M)) for gh in fg.grad_hat(uh)]
        fields.append([float(E[a]) + g[a] for a in range(d)])
    nE = len(Es)
    out = np.zeros((nE, nE))
    for i in range(nE):
        for j in range(nE):
            out[i, j] = np.mean(AM * sum(fields[i][a] * fields[j][a] for a in range(d)))
    return out


@dataclasses.dataclass
class GaResult:
    A_H: np.ndarray
    iters: List[int]
    res_hist: List[List[float]]
    u_hat: List[np.ndarray]


def solve(inc: Inclusion, N: Sequence[int], Es: Optional[Sequence[Sequence[float]]] = None,
          tol: float = 1e-10, max_iter: int = 1000, M: Optional[Sequence[int]] = None) -> GaResult:
    """Homogenised matrix of an inclusion coefficient by Ga (DoGIP) on the
    double grid M (default 2N - 1)."""
    N = list(N)
    d = len(N)
    if any(n % 2 == 0 for n in N):
        raise ValueError("odd grid sizes only (Sec. 2.2.1)")
    if Es is None:
        Es = [np.eye(d)[i] for i in range(d)]
    AM = coefficient_on_double_grid(inc, N, M)
    scale = float(np.sqrt(np.mean(AM * AM)))
    uhs, iters, hists = [], [], []
    for E in Es:
        bh = rhs(AM, N, E)
        floor = fg.ROUNDING_FLOOR * scale * float(np.linalg.norm(np.asarray(E, dtype=np.float64)))
        uh, it, hist = fg_tensor.pcg(lambda v: apply_K(AM, v), bh, tol, max_iter, floor)
        uhs.append(uh)
        iters.append(it)
        hists.append(hist)
    return GaResult(energy_matrix(AM, Es, uhs), iters, hists, uhs)
