"""Low-rank tensor formats on small NumPy arrays -- oracle (test infrastructure).

Written from the paper's Sec. 3.1 (overview of CP, Tucker and TT formats and
rank truncation), Sec. 3.2 (low-rank application of the operator,
eq. Pls_lowrank, Table 1) and Appendix A (element-wise products, Fourier
transforms and truncation in each format).  FP64 throughout; complex cores
are allowed (the low-rank solve of Sec. 3.2 runs in Fourier space).

Layouts follow the paper's indexing:
  CP      weights c (r,), factors b[j] of shape (r, N_j)        (eq. cano)
  Tucker  core c (r_1, ..., r_d), frames b[j] of shape (r_j, N_j) (eq. tucker)
  TT      cores b[j] of shape (r_{j-1}, N_j, r_j), r_0 = r_d = 1  (eq. TT)
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np


# ==========================================================================
# CP (paper Sec. 3.1.1, Appendix A.1)
# ==========================================================================

@dataclasses.dataclass
class CP:
    c: np.ndarray
    b: List[np.ndarray]

    @property
    def rank(self):
        return self.c.shape[0]

    def full(self):
        d = len(self.b)
        out = 0
        for i in range(self.rank):
            t = self.c[i]
            for j in range(d):
                sh = [1] * d
                sh[j] = self.b[j].shape[1]
                t = t * self.b[j][i].reshape(sh)
            out = out + t
        return np.asarray(out)


def cp_add(v: CP, w: CP) -> CP:
    """Sum: concatenation of the terms (rank r + s)."""
    return CP(np.concatenate([v.c, w.c]),
              [np.concatenate([x, y]) for x, y in zip(v.b, w.b)])


def cp_hadamard(v: CP, w: CP) -> CP:
    """Element-wise product: all pairs of terms, rank r*s (Appendix A.1)."""
    c = np.einsum("i,k->ik", v.c, w.c).reshape(-1)
    b = [np.einsum("in,kn->ikn", x, y).reshape(-1, x.shape[1])
         for x, y in zip(v.b, w.b)]
    return CP(c, b)


def cp_truncate_2d(v: CP, rank: int) -> CP:
    """d = 2 truncation: QR of both factor matrices, SVD of R1 diag(c) R2^T,
    keep `rank` leading singular triplets (Appendix A.1)."""
    B1 = v.b[0].T            # N1 x r
    B2 = v.b[1].T
    Q1, R1 = np.linalg.qr(B1)
    Q2, R2 = np.linalg.qr(B2)
    U, s, Vh = np.linalg.svd(R1 @ np.diag(v.c) @ R2.T)
    k = min(rank, s.shape[0])
    return CP(s[:k].copy(), [(Q1 @ U[:, :k]).T.copy(), (Q2 @ Vh[:k].T).T.copy()])


# ==========================================================================
# Tucker (paper Sec. 3.1.2, Appendix A.2)
# ==========================================================================

@dataclasses.dataclass
class Tucker:
    c: np.ndarray
    b: List[np.ndarray]

    @property
    def ranks(self):
        return tuple(self.c.shape)

    def full(self):
        out = self.c
        for j, B in enumerate(self.b):
            out = np.moveaxis(np.tensordot(out, B, axes=([j], [0])), -1, j)
        return out


def tucker_add(v: Tucker, w: Tucker) -> Tucker:
    """Sum: frames concatenated, block-diagonal core."""
    shape = tuple(x + y for x, y in zip(v.c.shape, w.c.shape))
    c = np.zeros(shape, dtype=np.result_type(v.c, w.c))
    c[tuple(slice(0, s) for s in v.c.shape)] = v.c
    c[tuple(slice(s, None) for s in v.c.shape)] = w.c
    return Tucker(c, [np.concatenate([x, y]) for x, y in zip(v.b, w.b)])


def tucker_hadamard(v: Tucker, w: Tucker) -> Tucker:
    """Element-wise product: Khatri-Rao frames and Kronecker core.

    The combined index of frame j is l = i*s_j + k (0-based) for the
    v-index i and the w-index k, the same order as np.kron.
    """
    c = np.kron(v.c, w.c)
    b = [np.einsum("in,kn->ikn", x, y).reshape(-1, x.shape[1])
         for x, y in zip(v.b, w.b)]
    return Tucker(c, b)


def hosvd(t: np.ndarray, ranks: Optional[Sequence[int]] = None,
          tol: float = 0.0) -> Tucker:
    """Truncated HOSVD of a full tensor (or of a core): frame j from the
    left singular vectors of the mode-j unfolding.  With `tol`, the ranks
    are the smallest whose discarded mode-wise singular values satisfy the
    error bound of Appendix A.2 with budget tol*||t|| split evenly over
    the d modes."""
    d = t.ndim
    nrm = np.linalg.norm(t)
    frames = []
    for j in range(d):
        M = np.moveaxis(t, j, 0).reshape(t.shape[j], -1)
        U, s, _ = np.linalg.svd(M, full_matrices=False)
        k = U.shape[1] if ranks is None else min(ranks[j], U.shape[1])
        if tol > 0:
            tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]   # tail[i] = ||s[i:]||
            budget = tol * nrm / np.sqrt(d)
            kk = next((i for i in range(len(s)) if tail[i] <= budget), len(s))
            k = min(k, max(kk, 1))
        frames.append(U[:, :k])
    c = t
    for j, U in enumerate(frames):
        c = np.moveaxis(np.tensordot(c, U.conj(), axes=([j], [0])), -1, j)
    return Tucker(c, [U.T.copy() for U in frames])


def tucker_truncate(v: Tucker, ranks: Optional[Sequence[int]] = None,
                    tol: float = 0.0) -> Tucker:
    """Re-orthogonalise the frames by QR, then HOSVD of the updated core
    (Appendix A.2)."""
    c = v.c
    Qs = []
    for j, B in enumerate(v.b):
        Q, R = np.linalg.qr(B.T)            # N_j x r_j = Q R
        Qs.append(Q)
        c = np.moveaxis(np.tensordot(c, R, axes=([j], [1])), -1, j)
    h = hosvd(c, ranks, tol)
    return Tucker(h.c, [(Q @ U.T).T.copy() for Q, U in zip(Qs, h.b)])


# ==========================================================================
# Tensor train (paper Sec. 3.1.3, Appendix A.3)
# ==========================================================================

def tt_full(cores: Sequence[np.ndarray]) -> np.ndarray:
    out = cores[0]                              # (1, N1, r1)
    for G in cores[1:]:
        out = np.tensordot(out, G, axes=([-1], [0]))
    return out.reshape(out.shape[1:-1])


def tt_ranks(cores) -> List[int]:
    return [cores[0].shape[0]] + [G.shape[2] for G in cores]


def tt_svd(t: np.ndarray, rank_cap: int = 10 ** 9, tol: float = 0.0) -> List[np.ndarray]:
    """TT decomposition of a full tensor by d-1 sequential SVDs (TT-SVD).
    Each SVD drops at most tol*||t||/sqrt(d-1) in Frobenius norm, so the
    total error is below tol*||t|| (Appendix A.3 bound)."""
    d = t.ndim
    Ns = t.shape
    delta = tol * np.linalg.norm(t) / np.sqrt(max(d - 1, 1))
    cores = []
    r = 1
    M = t.reshape(1, -1)
    for j in range(d - 1):
        M = M.reshape(r * Ns[j], -1)
        U, s, Vh = np.linalg.svd(M, full_matrices=False)
        k = _cut(s, delta, rank_cap)
        cores.append(U[:, :k].reshape(r, Ns[j], k))
        M = s[:k, None] * Vh[:k]
        r = k
    cores.append(M.reshape(r, Ns[-1], 1))
    return cores


def _cut(s: np.ndarray, delta: float, cap: int) -> int:
    """Smallest k <= cap with ||s[k:]|| <= delta (at least 1)."""
    tail = np.sqrt(np.cumsum((np.abs(s) ** 2)[::-1]))[::-1]
    k = len(s)
    for i in range(len(s)):
        if tail[i] <= delta:
            k = i
            break
    return int(max(1, min(k, cap)))


def tt_add(v, w) -> List[np.ndarray]:
    """Sum of two TTs: first cores side by side, middle cores block-diagonal,
    last cores stacked (ranks add)."""
    d = len(v)
    out = []
    for j, (A, B) in enumerate(zip(v, w)):
        dt = np.result_type(A, B)
        if d == 1:
            out.append(A + B)
        elif j == 0:
            out.append(np.concatenate([A, B], axis=2).astype(dt))
        elif j == d - 1:
            out.append(np.concatenate([A, B], axis=0).astype(dt))
        else:
            C = np.zeros((A.shape[0] + B.shape[0], A.shape[1],
                          A.shape[2] + B.shape[2]), dtype=dt)
            C[:A.shape[0], :, :A.shape[2]] = A
            C[A.shape[0]:, :, A.shape[2]:] = B
            out.append(C)
    return out


def tt_scale(v, s) -> List[np.ndarray]:
    out = [G.copy() for G in v]
    out[0] = out[0] * s
    return out


def tt_hadamard(v, w) -> List[np.ndarray]:
    """Element-wise product: slice-wise Kronecker (Khatri-Rao over the mode
    index) of the carriages; ranks multiply (Appendix A.3)."""
    out = []
    for A, B in zip(v, w):
        C = np.einsum("anb,cnd->acnbd", A, B)
        out.append(C.reshape(A.shape[0] * B.shape[0], A.shape[1],
                             A.shape[2] * B.shape[2]))
    return out


def tt_mode_apply(v, j: int, M: np.ndarray) -> List[np.ndarray]:
    """Apply an N_j x N_j matrix along the mode index of carriage j."""
    out = [G.copy() for G in v]
    out[j] = np.einsum("mn,anb->amb", M, v[j])
    return out


def tt_mode_scale(v, j: int, s: np.ndarray) -> List[np.ndarray]:
    """Multiply carriage j by a vector along its mode index (rank-1 operator)."""
    out = [G.copy() for G in v]
    out[j] = v[j] * s[None, :, None]
    return out


def tt_dft(v, inverse: bool = False) -> List[np.ndarray]:
    """d-dimensional DFT as 1-D DFTs of every carriage along its mode
    index (Appendix A.3); F carries 1/N_j, F^-1 is unnormalised."""
    out = []
    for G in v:
        if inverse:
            out.append(np.fft.ifft(G, axis=1) * G.shape[1])
        else:
            out.append(np.fft.fft(G, axis=1) / G.shape[1])
    return out


def tt_dot(v, w) -> complex:
    """<v, w> = sum conj(v) w, contracted carriage by carriage."""
    M = np.ones((1, 1))
    for A, B in zip(v, w):
        M = np.einsum("ac,anb,cnd->bd", M, A.conj(), B)
    return complex(M[0, 0])


def tt_round(v, rank_cap: int = 10 ** 9, tol: float = 0.0) -> List[np.ndarray]:
    """TT truncation (rounding): right-to-left re-orthogonalisation by QR,
    then d-1 left-to-right SVDs of the unfolded carriages, each cut at the
    smallest rank whose dropped singular values have norm <= tol*||v||/sqrt(d-1),
    capped at rank_cap (Appendix A.3)."""
    d = len(v)
    cores = [G.copy() for G in v]
    for j in range(d - 1, 0, -1):
        G = cores[j]
        r0, n, r1 = G.shape
        Q, R = np.linalg.qr(G.reshape(r0, n * r1).T)      # (n r1) x k
        k = Q.shape[1]
        cores[j] = Q.T.reshape(k, n, r1)
        cores[j - 1] = np.tensordot(cores[j - 1], R.T, axes=([2], [0]))
    nrm = np.linalg.norm(cores[0])
    delta = tol * nrm / np.sqrt(max(d - 1, 1))
    for j in range(d - 1):
        G = cores[j]
        r0, n, r1 = G.shape
        U, s, Vh = np.linalg.svd(G.reshape(r0 * n, r1), full_matrices=False)
        k = _cut(s, delta, rank_cap)
        cores[j] = U[:, :k].reshape(r0, n, k)
        cores[j + 1] = np.tensordot(s[:k, None] * Vh[:k], cores[j + 1], axes=([1], [0]))
    return cores


def tt_from_cp(v: CP) -> List[np.ndarray]:
    """CP -> TT with diagonal middle carriages."""
    d = len(v.b)
    r = v.rank
    cores = []
    for j, B in enumerate(v.b):
        n = B.shape[1]
        if j == 0:
            cores.append((B.T * v.c[None, :]).reshape(1, n, r))
        elif j == d - 1:
            cores.append(B.reshape(r, n, 1))
        else:
            C = np.zeros((r, n, r), dtype=B.dtype)
            for i in range(r):
                C[i, :, i] = B[i]
            cores.append(C)
    return cores


# ==========================================================================
# Low-rank operator of Sec. 3.2 and truncated minimal residual, Sec. 3.3
# ==========================================================================

def _freq(N):
    return np.fft.fftfreq(N, d=1.0 / N).round()


def lowrank_precond_tt(shape, tol: float = 1e-13) -> List[np.ndarray]:
    """TT of the Fourier-space preconditioner diag 1/(4 pi^2 k.k) (0 at
    k = 0) obtained by TT-SVD of the full array (small grids only)."""
    d = len(shape)
    kk = 0
    for al, n in enumerate(shape):
        sh = [1] * d
        sh[al] = n
        kk = kk + (_freq(n) ** 2).reshape(sh)
    P = np.zeros(shape)
    P[kk != 0] = 1.0 / (4 * np.pi ** 2 * kk[kk != 0])
    return tt_svd(P, tol=tol)


@dataclasses.dataclass
class LowRankOperator:
    """C v ~ T P^-1 T div^ F T A F^-1 grad^ v  (eq. Pls_lowrank, GaNi)."""
    a_tt: List[np.ndarray]                  # coefficient, real space
    p_tt: List[np.ndarray]                  # preconditioner, Fourier space
    rank_cap: int
    tol: float

    def T(self, v):
        return tt_round(v, self.rank_cap, self.tol)

    def grad(self, vh, alpha):
        n = vh[alpha].shape[1]
        return tt_mode_scale(vh, alpha, 2j * np.pi * _freq(n))

    def div_sum(self, wh):
        acc = None
        for alpha, w in enumerate(wh):
            n = w[alpha].shape[1]
            t = tt_mode_scale(w, alpha, -2j * np.pi * _freq(n))
            acc = t if acc is None else tt_add(acc, t)
        return acc

    def K(self, vh):
        d = len(vh)
        hs = []
        for alpha in range(d):
            g = tt_dft(self.grad(vh, alpha), inverse=True)
            h = self.T(tt_hadamard(self.a_tt, g))
            hs.append(tt_dft(h))
        return self.T(self.div_sum(hs))

    def Pinv(self, vh):
        return self.T(tt_hadamard(self.p_tt, vh))

    def C(self, vh):
        return self.Pinv(self.K(vh))

    def rhs(self, E):
        d = len(self.a_tt)
        hs = []
        for alpha in range(d):
            hs.append(tt_dft(tt_scale(self.a_tt, float(E[alpha]))))
        b = self.div_sum(hs)
        return self.T(tt_hadamard(self.p_tt, tt_scale(b, -1.0)))


def tt_norm(v) -> float:
    return float(np.sqrt(max(tt_dot(v, v).real, 0.0)))


def minimal_residual(op: LowRankOperator, E, max_iter: int = 200,
                     tol: float = 1e-10):
    """Truncated minimal-residual iteration (Sec. 3.3):
        r_i = d - C u_i,  omega_i = (C r_i, r_i)/||C r_i||^2,
        u_{i+1} = T[u_i + omega_i r_i],
    stopped when the residual fails to decrease (Sec. 4.3) or drops below
    tol relative to ||d||; the best iterate is returned."""
    dvec = op.rhs(E)
    d0 = tt_norm(dvec)
    u = [np.zeros((1 if j == 0 else 1, G.shape[1], 1), dtype=complex)
         for j, G in enumerate(dvec)]
    hist = []
    best, best_res = u, np.inf
    if d0 == 0.0:
        return u, hist
    for _ in range(max_iter):
        r = op.T(tt_add(dvec, tt_scale(op.C(u), -1.0)))
        res = tt_norm(r) / d0
        hist.append(res)
        if res >= best_res:
            break
        best, best_res = u, res
        if res <= tol:
            break
        Cr = op.C(r)
        omega = tt_dot(Cr, r).real / tt_dot(Cr, Cr).real
        u = op.T(tt_add(u, tt_scale(r, omega)))
    return best, hist


def energy_from_tt(a: np.ndarray, Es, uhs_tt) -> np.ndarray:
    """A_H E_i.E_j from Fourier-space TT correctors, evaluated on the full
    grid (small grids only; eq. homog with the GaNi mean)."""
    d = a.ndim
    fields = []
    for E, uh in zip(Es, uhs_tt):
        U = tt_full(uh)
        g = []
        for al in range(d):
            sh = [1] * d
            sh[al] = a.shape[al]
            gh = 2j * np.pi * _freq(a.shape[al]).reshape(sh) * U
            g.append(np.fft.ifftn(gh).real * a.size + float(E[al]))
        fields.append(g)
    nE = len(Es)
    A = np.zeros((nE, nE))
    for i in range(nE):
        for j in range(nE):
            A[i, j] = np.mean(a * sum(fields[i][al] * fields[j][al] for al in range(d)))
    return A
