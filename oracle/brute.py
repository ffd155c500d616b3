"""Dense brute force of the GaNi cell problem on tiny grids -- oracle (test infrastructure).

An independent route to the same discrete minimiser as `oracle.fg`: the
paper's eq. (homog) restricted to trigonometric polynomials T_N (Sec. 2.2.1)
with the rectangle rule (Sec. 2.2.2) is

    A_H E.E = min_{v in T_N, mean 0}  mean_x a(x) |E + grad v(x)|^2,

and on nodal values grad v = D v with the real matrices
D_alpha = F^-1 diag(2 pi i k_alpha) F (eq. grad_trig).  Here F is built as
an explicit DFT matrix from cos/sin of the centred indices (no FFT), the
normal equations D^T A D v = -D^T A E are solved with a pseudo-inverse
(the constant mode is the null space), and A_H is formed from the
minimiser.  Real-space, dense, direct: it shares nothing with the FFT/CG
oracle except the definitions.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np


def dft_matrix_1d(N: int) -> np.ndarray:
    """F_N[m, k] = (1/N) exp(-2 pi i m k / N) on centred indices m, k."""
    c = np.arange(N) - (N - 1) // 2
    ang = -2.0 * np.pi * np.outer(c, c) / N
    return (np.cos(ang) + 1j * np.sin(ang)) / N


def derivative_matrix_1d(N: int) -> np.ndarray:
    """Real N x N matrix of the spectral derivative on nodal values."""
    c = np.arange(N) - (N - 1) // 2
    F = dft_matrix_1d(N)
    Finv = np.conj(F.T) * N          # unnormalised inverse
    D = Finv @ np.diag(2j * np.pi * c) @ F
    assert np.max(np.abs(D.imag)) < 1e-9 * max(1.0, np.max(np.abs(D.real)))
    return D.real


def solve(a: np.ndarray, Es: Optional[Sequence[Sequence[float]]] = None) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    d = a.ndim
    shape = a.shape
    n = a.size
    if Es is None:
        Es = [np.eye(d)[i] for i in range(d)]
    Ds = []
    for alpha in range(d):
        mats = [np.eye(s) for s in shape]
        mats[alpha] = derivative_matrix_1d(shape[alpha])
        M = mats[0]
        for m in mats[1:]:
            M = np.kron(M, m)
        Ds.append(M)
    D = np.vstack(Ds)                       # (d n) x n
    W = np.tile(a.reshape(-1), d) / n       # grid-mean quadrature of a
    K = D.T @ (W[:, None] * D)
    Kp = np.linalg.pinv(K, rcond=1e-13, hermitian=True)
    fields = []
    for E in Es:
        eE = np.concatenate([np.full(n, float(E[al])) for al in range(d)])
        rhs = -D.T @ (W * eE)
        v = Kp @ rhs
        fields.append(eE + D @ v)
    nE = len(Es)
    A = np.zeros((nE, nE))
    for i in range(nE):
        for j in range(nE):
            A[i, j] = float(np.sum(W * fields[i] * fields[j]))
    return A


def solve_tensor(A: np.ndarray, Es: Optional[Sequence[Sequence[float]]] = None) -> np.ndarray:
    """The same dense minimisation for a matrix-valued coefficient A (shape
    (d, d, N..)): mean_x A(x)(E + D v).(E + D v), with the quadrature weight
    now a d x d block per grid point (Sec. 4.4's a I + B is one case)."""
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[0]
    shape = A.shape[2:]
    n = int(np.prod(shape))
    if Es is None:
        Es = [np.eye(d)[i] for i in range(d)]
    Ds = []
    for alpha in range(d):
        mats = [np.eye(s) for s in shape]
        mats[alpha] = derivative_matrix_1d(shape[alpha])
        M = mats[0]
        for m in mats[1:]:
            M = np.kron(M, m)
        Ds.append(M)
    D = np.vstack(Ds)                       # (d n) x n
    W = np.zeros((d * n, d * n))            # block (alpha, beta) = diag(A_ab)/n
    for al in range(d):
        for be in range(d):
            W[al * n:(al + 1) * n, be * n:(be + 1) * n] = np.diag(A[al, be].reshape(-1)) / n
    K = D.T @ W @ D
    Kp = np.linalg.pinv(K, rcond=1e-13, hermitian=True)
    fields = []
    for E in Es:
        eE = np.concatenate([np.full(n, float(E[al])) for al in range(d)])
        v = Kp @ (-D.T @ (W @ eE))
        fields.append(eE + D @ v)
    nE = len(Es)
    out = np.zeros((nE, nE))
    for i in range(nE):
        for j in range(nE):
            out[i, j] = float(fields[j] @ (W @ fields[i]))
    return out
