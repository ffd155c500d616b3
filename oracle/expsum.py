"""Exponential-sum preconditioner for the low-rank path -- oracle (test infrastructure).

The paper applies the preconditioner to low-rank tensors as an element-wise
product that raises the rank (Sec. 3.2, Table 1) but gives no separable form
of diag(1/(4 pi^2 k.k)).  The reading used here: approximate 1/y on
[1, R] by a positive exponential sum obtained from the trapezoidal (sinc)
quadrature of the integral identity

    1/y = integral over s in R of exp(s - e^s y) ds,

    1/y ~ sum_{m=0}^{M-1} w_m exp(-t_m y),  t_m = exp(s_m),  w_m = h exp(s_m),
    s_m = s_lo + m h,  s_lo = ln(eps / R),  s_hi = ln(ln(1/eps)),
    h = (s_hi - s_lo) / (M - 1),  eps = 1e-2.

With y = k.k (x = 4 pi^2 y), exp(-t y) = prod_alpha exp(-t k_alpha^2) is a
rank-1 tensor, so the preconditioner becomes a rank-M Kronecker sum.  Every
weight is positive, so the approximate preconditioner stays SPD and the
discrete solution is unchanged; only the convergence rate depends on M.
"""
from __future__ import annotations

import math

import numpy as np

EPS_TAIL = 1e-2


def expsum_nodes(R: float, M: int):
    """Exponents t_m and weights w_m for 1/y on [1, R] (see module doc)."""
    if M < 2:
        raise ValueError("M >= 2")
    s_lo = math.log(EPS_TAIL / R)
    s_hi = math.log(math.log(1.0 / EPS_TAIL))
    h = (s_hi - s_lo) / (M - 1)
    s = s_lo + h * np.arange(M)
    return np.exp(s), h * np.exp(s)


def expsum_eval(y: np.ndarray, t: np.ndarray, w: np.ndarray) -> np.ndarray:
    return np.sum(w[:, None] * np.exp(-np.outer(t, np.ravel(y))), axis=0).reshape(np.shape(y))


def default_terms(R: float) -> int:
    """M such that the node spacing h is at most 2."""
    s_lo = math.log(EPS_TAIL / R)
    s_hi = math.log(math.log(1.0 / EPS_TAIL))
    return int(math.ceil((s_hi - s_lo) / 2.0)) + 1


def precond_symbol(shape, M: int = 0) -> np.ndarray:
    """Full-grid symbol (1/(4 pi^2)) sum_m w_m exp(-t_m k.k) in FFT order."""
    d = len(shape)
    R = float(sum(((n - 1) // 2) ** 2 for n in shape))
    if M == 0:
        M = default_terms(R)
    t, w = expsum_nodes(R, M)
    kk = 0
    for al, n in enumerate(shape):
        sh = [1] * d
        sh[al] = n
        kk = kk + (np.fft.fftfreq(n, d=1.0 / n).round() ** 2).reshape(sh)
    return expsum_eval(kk, t, w) / (4 * np.pi ** 2)
