"""Seeded synthetic inputs for the periodic cell problem.

This module is shared by the HIP path, the CPU oracle, the tests and the
benchmark.  It holds only input definitions: coefficient fields sampled at
the grid points, their separable (CP) factors where a closed form exists,
and request streams for the serving loop.  None of the homogenisation
arithmetic (FFTs, operators, solvers, truncation) lives here.

Grid convention (paper Sec. 2.2.1, the regular grid x_k = k/N for centred
k in Z_N, odd N): along each axis the point with storage index j in [0, N)
sits at x_j = -1/2 + (j + 1/2)/N, i.e. the cell centres of Y = (-1/2, 1/2)^d.
Arrays are C-ordered, axis 0 = x_1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "grid_points", "CPCoeff", "square_coeff", "cube_coeff", "ball_coeff",
    "laminate_coeff", "constant_coeff", "smooth_params", "smooth_cp",
    "smooth_coeff", "random_positive_coeff", "random_cp", "random_tt",
    "ServingRequest", "serving_requests", "anisotropy", "MaterialS", "material_s_params", "material_s",
]


def grid_points(N: int) -> np.ndarray:
    """Cell-centre grid points of one axis (odd N), float64."""
    if N < 1 or N % 2 == 0:
        raise ValueError("N must be odd and positive")
    return -0.5 + (np.arange(N, dtype=np.float64) + 0.5) / N


@dataclasses.dataclass
class CPCoeff:
    """A coefficient given as a sum of separable terms.

    a(x) = sum_t weights[t] * prod_i factors[i][t, j_i]   (factors[i]: (R, N_i)).
    This is the CP form of the paper's appendix (eq. cano); it is the natural
    way to hand a separable coefficient to the low-rank path.
    """
    weights: np.ndarray          # (R,)
    factors: List[np.ndarray]    # d arrays of shape (R, N_i)

    @property
    def rank(self) -> int:
        return int(self.weights.shape[0])

    def full(self) -> np.ndarray:
        """Dense nodal values (small grids only)."""
        d = len(self.factors)
        shape = tuple(f.shape[1] for f in self.factors)
        out = np.zeros(shape)
        for t in range(self.rank):
            term = np.asarray(self.weights[t], dtype=np.float64)
            for i in range(d):
                sh = [1] * d
                sh[i] = shape[i]
                term = term * self.factors[i][t].reshape(sh)
            out = out + term
        return out


# --------------------------------------------------------------------------
# Inclusions (paper Sec. 4.1, eq. Adef / shape_fun; ball of the 3D workload)
# --------------------------------------------------------------------------

def square_coeff(N: int, d: int = 2, fraction: float = 0.3,
                 inside: float = 10.0, outside: float = 1.0) -> np.ndarray:
    """Centred square (d=2) or cube (d=3) of volume fraction `fraction`.

    Side s = fraction**(1/d); a = inside where |x_i| < s/2 for all i.
    """
    half = 0.5 * fraction ** (1.0 / d)
    x = grid_points(N)
    ind = (np.abs(x) < half).astype(np.float64)
    chi = ind
    for _ in range(d - 1):
        chi = np.multiply.outer(chi, ind)
    return outside + (inside - outside) * chi


def square_cp(N: int, d: int = 2, fraction: float = 0.3,
              inside: float = 10.0, outside: float = 1.0) -> CPCoeff:
    """The same square/cube as two separable terms: outside*1 + (in-out)*chi."""
    half = 0.5 * fraction ** (1.0 / d)
    x = grid_points(N)
    ind = (np.abs(x) < half).astype(np.float64)
    ones = np.ones(N)
    factors = [np.stack([ones, ind]) for _ in range(d)]
    return CPCoeff(np.array([outside, inside - outside]), factors)


def cube_coeff(N: int, half_side: float = 0.3, inside: float = 11.0,
               outside: float = 1.0, d: int = 3) -> np.ndarray:
    """The paper's cube: a = inside where |x_i| < half_side for every i.

    With rho = 10 the paper's A = I(1 + rho*chi) gives inside = 11.
    """
    x = grid_points(N)
    ind = (np.abs(x) < half_side).astype(np.float64)
    chi = ind
    for _ in range(d - 1):
        chi = np.multiply.outer(chi, ind)
    return outside + (inside - outside) * chi


def ball_coeff(N: int, radius: float = 0.3, inside: float = 100.0,
               outside: float = 1.0, d: int = 3) -> np.ndarray:
    """Centred ball |x| < radius (no odd-N grid point lies on the sphere
    for radius 0.3 at the sizes used here; ties resolve to 'outside')."""
    x = grid_points(N)
    r2 = np.zeros((N,) * d)
    for i in range(d):
        sh = [1] * d
        sh[i] = N
        r2 = r2 + (x ** 2).reshape(sh)
    return np.where(r2 < radius * radius, inside, outside).astype(np.float64)


def laminate_coeff(N: int, d: int, profile: np.ndarray, axis: int = 0) -> np.ndarray:
    """a(x) = profile[j_axis]: layers normal to `axis`."""
    profile = np.asarray(profile, dtype=np.float64)
    assert profile.shape == (N,)
    sh = [1] * d
    sh[axis] = N
    return np.broadcast_to(profile.reshape(sh), (N,) * d).copy()


def constant_coeff(N: int, d: int, value: float) -> np.ndarray:
    return np.full((N,) * d, float(value))


@dataclasses.dataclass
class MaterialS:
    """Parameters of one sample of the paper's stochastic material S."""
    ks: np.ndarray       # (n, d) integer frequency of each real mode
    kinds: np.ndarray    # (n,) 0: cos(2 pi k.x), 1: sin(2 pi k.x)
    c: np.ndarray        # (n,) coefficients ~ U(-0.5, 0.5)


def material_s_params(d: int, seed: int = 0) -> MaterialS:
    """Sec. 4.1, eq. shape_fun2: the leading modes of a Karhunen-Loeve
    expansion of a squared-exponential covariance on the periodic cell are
    the real Fourier modes of the lowest frequencies; 20 modes in 2D and 26
    in 3D are exactly cos and sin of one k of each pair +-k with |k|^2 <= 5
    (2D) or |k|^2 <= 3 (3D).  Modes in order of |k|^2, then k
    lexicographically (first nonzero component positive), cos before sin;
    default_rng(seed) draws the n coefficients c ~ U(-0.5, 0.5) in that
    order."""
    kmax2 = {2: 5, 3: 3}[d]
    r = int(math.isqrt(kmax2))
    ks = []
    for k in np.ndindex(*(2 * r + 1,) * d):
        k = np.array(k) - r
        nz = k[np.nonzero(k)[0]]
        if nz.size == 0 or nz[0] < 0 or int(k @ k) > kmax2:
            continue
        ks.append(k)
    ks.sort(key=lambda k: (int(k @ k), tuple(k)))
    ks = np.array([k for k in ks for _ in (0, 1)])
    kinds = np.tile([0, 1], len(ks) // 2)
    c = np.random.default_rng(seed).uniform(-0.5, 0.5, len(ks))
    return MaterialS(ks, kinds, c)


def material_s(N: int, d: int, seed: int = 0, amin: float = 1.0, amax: float = 10.0) -> np.ndarray:
    """Nodal values of a(x) = exp(C + D sum_k c[k] phi_k(x)) (eq. shape_fun2),
    C and D chosen so that the grid samples span [amin, amax] (the paper
    scales the sample to [1, 10])."""
    p = material_s_params(d, seed)
    x = grid_points(N)
    grids = np.meshgrid(*([x] * d), indexing="ij")
    s = np.zeros((N,) * d)
    for k, kind, c in zip(p.ks, p.kinds, p.c):
        ph = 2.0 * np.pi * sum(int(k[a]) * grids[a] for a in range(d))
        s += c * (np.cos(ph) if kind == 0 else np.sin(ph))
    D = math.log(amax / amin) / (s.max() - s.min())
    C = math.log(amin) - D * s.min()
    return np.exp(C + D * s)


def anisotropy(d: int) -> np.ndarray:
    """The constant matrix B that Sec. 4.4 adds to an isotropic material
    (A~ = a I + B); the paper gives its eigenvalues as (1, 10) in 2D and
    (1, 5, 10) in 3D."""
    if d == 2:
        return np.array([[5.5, -4.5], [-4.5, 5.5]])
    if d == 3:
        q = 1.25 * math.sqrt(2.0)
        return np.array([[4.25, -3.25, -q], [-3.25, 4.25, q], [-q, q, 7.5]])
    raise ValueError("d must be 2 or 3")


# --------------------------------------------------------------------------
# Smooth coefficient:  a = 1 + 0.5 sum_j c_j prod_i cos(2 pi k_ji x_i + phi_ji)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class SmoothParams:
    c: np.ndarray        # (J,)
    k: np.ndarray        # (J, d) integers
    phi: np.ndarray      # (J, d)
    amp: float = 0.5
    clip: tuple = (0.1, 10.0)


def smooth_params(seed: int = 0, J: int = 8, d: int = 3, c_max: float = 0.3,
                  k_max: int = 4) -> SmoothParams:
    """Draw order: c (J values, U(-c_max, c_max)), then k (J x d, U{1..k_max}),
    then phi (J x d, U(0, 2 pi)); one numpy default_rng(seed) stream."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-c_max, c_max, J)
    k = rng.integers(1, k_max + 1, size=(J, d))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=(J, d))
    return SmoothParams(c=c, k=k, phi=phi)


def smooth_cp(N: int, p: SmoothParams) -> CPCoeff:
    """Unclipped smooth coefficient as J+1 separable terms (rank <= J+1)."""
    x = grid_points(N)
    J, d = p.k.shape
    weights = np.concatenate([[1.0], p.amp * p.c])
    factors = []
    for i in range(d):
        rows = [np.ones(N)]
        for j in range(J):
            rows.append(np.cos(2.0 * np.pi * p.k[j, i] * x + p.phi[j, i]))
        factors.append(np.stack(rows))
    return CPCoeff(weights, factors)


def smooth_coeff(N: int, p: SmoothParams, clip: bool = True):
    """Dense smooth coefficient; returns (a, clipped_flag)."""
    a = smooth_cp(N, p).full()
    lo, hi = p.clip
    clipped = bool(clip and (a.min() < lo or a.max() > hi))
    if clip:
        a = np.clip(a, lo, hi)
    return a, clipped


def rescale_contrast(a: np.ndarray, contrast: float) -> np.ndarray:
    """Affine map of a field onto [1, contrast] using its grid min and max."""
    lo, hi = float(a.min()), float(a.max())
    if hi - lo <= 0:
        return np.ones_like(a)
    return 1.0 + (contrast - 1.0) * (a - lo) / (hi - lo)


def rescale_contrast_cp(cp: CPCoeff, contrast: float) -> CPCoeff:
    """rescale_contrast for a CP coefficient whose first term is a constant
    (weights[0] times all-ones factors, as smooth_cp builds it): the affine
    map only changes the weights, so the rank is kept.  The grid min and max
    are taken slab by slab."""
    d = len(cp.factors)
    lo, hi = np.inf, -np.inf
    for n0 in range(cp.factors[0].shape[1]):
        sub = CPCoeff(cp.weights * cp.factors[0][:, n0], list(cp.factors[1:])) if d > 1 else None
        v = sub.full() if sub is not None else cp.weights @ cp.factors[0][:, n0:n0 + 1]
        lo, hi = min(lo, float(np.min(v))), max(hi, float(np.max(v)))
    if hi - lo <= 0:
        return CPCoeff(np.concatenate([[1.0], np.zeros(cp.rank - 1)]), [f.copy() for f in cp.factors])
    beta = (contrast - 1.0) / (hi - lo)
    w = beta * cp.weights
    w[0] += 1.0 - beta * lo
    return CPCoeff(w, [f.copy() for f in cp.factors])


def cube_cp(N: int, contrast: float, half_side: float = 0.3, d: int = 3) -> CPCoeff:
    """Centred cube |x_i| < half_side with a = contrast inside, 1 outside, as
    the two separable terms 1 + (contrast - 1) chi."""
    x = grid_points(N)
    ind = (np.abs(x) < half_side).astype(np.float64)
    ones = np.ones(N)
    return CPCoeff(np.array([1.0, contrast - 1.0]), [np.stack([ones, ind]) for _ in range(d)])


def request_ball(req: "ServingRequest") -> np.ndarray:
    """Nodal values of a ball request: the centred ball of radius 0.3 with
    a = contrast inside and 1 outside."""
    return ball_coeff(req.N, radius=0.3, inside=req.contrast, outside=1.0)


def request_coeff(req: "ServingRequest") -> CPCoeff:
    """The CP coefficient of a serving request: the contrast-rescaled smooth
    family (seed = request id), or for kind "ball" its separable stand-in,
    the centred cube of half side 0.3 at the same contrast (the ball itself
    is not separable and would need a compressed TT)."""
    if req.kind == "smooth":
        return rescale_contrast_cp(smooth_cp(req.N, smooth_params(req.rid)), req.contrast)
    return cube_cp(req.N, req.contrast)


# --------------------------------------------------------------------------
# Random inputs for tests
# --------------------------------------------------------------------------

def random_positive_coeff(N: int, d: int, seed: int, lo: float = 0.5,
                          hi: float = 5.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(N,) * d)


def random_cp(Ns: Sequence[int], R: int, seed: int, positive: bool = False) -> CPCoeff:
    rng = np.random.default_rng(seed)
    if positive:
        w = rng.uniform(0.2, 1.0, R)
        f = [rng.uniform(0.5, 1.5, size=(R, n)) for n in Ns]
    else:
        w = rng.standard_normal(R)
        f = [rng.standard_normal((R, n)) for n in Ns]
    return CPCoeff(w, f)


def random_tt(Ns: Sequence[int], ranks: Sequence[int], seed: int) -> List[np.ndarray]:
    """Random TT cores [r_{j-1}][N_j][r_j] with r_0 = r_d = 1."""
    rng = np.random.default_rng(seed)
    d = len(Ns)
    assert len(ranks) == d + 1 and ranks[0] == 1 and ranks[-1] == 1
    return [rng.standard_normal((ranks[j], Ns[j], ranks[j + 1])) for j in range(d)]


# --------------------------------------------------------------------------
# Serving request stream
# --------------------------------------------------------------------------

@dataclasses.dataclass
class ServingRequest:
    rid: int
    N: int
    kind: str            # "ball" or "smooth"
    contrast: float
    rank_cap: int
    arrival_s: float


def serving_requests(n: int, rate_per_s: float, seed: int = 0,
                     N_lo: int = 45, N_hi: int = 405,
                     cap_lo: int = 10, cap_hi: int = 60) -> List[ServingRequest]:
    """Request i uses default_rng(seed + i): N odd uniform in [N_lo, N_hi],
    kind ball/smooth with probability 1/2, contrast log-uniform in [2, 100],
    rank cap uniform in {cap_lo..cap_hi}.  Arrivals: Poisson process with
    the given rate, drawn from default_rng(seed) (exponential gaps)."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps)
    out = []
    odd = np.arange(N_lo | 1, N_hi + 1, 2)
    for i in range(n):
        r = np.random.default_rng(seed + i)
        N = int(r.choice(odd))
        kind = "ball" if r.random() < 0.5 else "smooth"
        contrast = float(math.exp(r.uniform(math.log(2.0), math.log(100.0))))
        cap = int(r.integers(cap_lo, cap_hi + 1))
        out.append(ServingRequest(i, N, kind, contrast, cap, float(t[i])))
    return out
