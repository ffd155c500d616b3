"""Fourier-Galerkin with exact integration (Ga, Sec. 2.2.3) on the GPU's
double grid against the CPU oracle (oracle.fg_ga)."""
import numpy as np
import pytest

import paper_1902_07455_amd as P
import workloads as W
from oracle import fg_ga as G

pytestmark = pytest.mark.gpu


def _rel(A, B):
    return np.max(np.abs(A - B)) / np.max(np.abs(B))


@pytest.mark.parametrize("shape,d,N,inside", [("square", 2, 15, 10.0), ("square", 2, 23, 10.0),
                                              ("square", 3, 15, 10.0), ("ball", 3, 15, 100.0),
                                              ("ball", 3, 23, 10.0), ("square", 2, 45, 0.1)])
def test_ga_equals_oracle(dev, shape, d, N, inside):
    """Double grids 45, 45 and 125 (the smallest odd 3^a 5^b >= 2N - 1)
    against the oracle on its grid 2N - 1 = 29, 45 and 89: the same Galerkin
    system."""
    size = 0.3
    s = P.Solver(d=d, N=(N,) * d, format="full", discretisation="ga", solver_tol=1e-12, max_iter=3000)
    r = s.solve(inclusion=dict(shape=shape, size=size, inside=inside, outside=1.0))
    o = G.solve(G.Inclusion(shape, size, inside, 1.0), [N] * d, tol=1e-12, max_iter=3000)
    assert r.rc == 0
    assert _rel(r.A_H, o.A_H) <= 1e-10
    assert abs(int(r.iters.max()) - max(o.iters)) <= 2


def test_ga_nonsquare_grid_and_general_E(dev):
    N = (9, 15, 11)
    inc = dict(shape="square", size=0.25, inside=5.0, outside=1.0)
    E = np.array([[1.0, -0.5, 0.3], [0.2, 1.0, 0.7]])
    s = P.Solver(d=3, N=N, format="full", discretisation="ga", solver_tol=1e-12, max_iter=3000, max_nE=3)
    A = s.solve(inclusion=inc).A_H
    G2 = s.solve(inclusion=inc, E=E).A_H
    o = G.solve(G.Inclusion("square", 0.25, 5.0, 1.0), list(N), tol=1e-12, max_iter=3000)
    assert _rel(A, o.A_H) <= 1e-10
    assert _rel(G2, E @ A @ E.T) <= 1e-10


def _ga_aniso_oracle(shape, d, N, inside, B):
    """Ga of the matrix coefficient a I + B from the oracle's double-grid
    coefficient (a constant B only adds B at the zero frequency): the
    oracle's Ga steps with the tensor material law."""
    from oracle import fg_tensor as FT
    inc = G.Inclusion(shape, 0.3, inside, 1.0)
    AM = G.coefficient_on_double_grid(inc, [N] * d)
    AT = FT.isotropic_plus_constant(AM, B)
    Es = [np.eye(d)[i] for i in range(d)]
    uhs = []
    for E in Es:
        bh = -G.fg.div_hat([G.restrict(G.fg.fwd(sum(AT[al, be] * E[be] for be in range(d))), [N] * d)
                           for al in range(d)])
        op = lambda v: G.fg.div_hat([G.restrict(G.fg.fwd(h), [N] * d) for h in FT.material_law(
            AT, [G.fg.inv(G.pad(gh, AM.shape)) for gh in G.fg.grad_hat(v)])])
        uh, _, _ = FT.pcg(op, bh, 1e-12, 3000, 0.0)
        uhs.append(uh)
    fields = []
    for E, uh in zip(Es, uhs):
        g = [G.fg.inv(G.pad(gh, AM.shape)) for gh in G.fg.grad_hat(uh)]
        fields.append([E[a] + g[a] for a in range(d)])
    return np.array([[np.mean(sum(f * e for f, e in zip(FT.material_law(AT, fields[i]), fields[j])))
                      for j in range(d)] for i in range(d)])


def test_ga_with_anisotropy(dev):
    """Ga with the constant B of Sec. 4.4: B is integrated exactly too."""
    N = 15
    B = W.anisotropy(3)
    s = P.Solver(d=3, N=(N,) * 3, format="full", discretisation="ga", solver_tol=1e-12, max_iter=3000, aniso=B)
    r = s.solve(inclusion=dict(shape="ball", size=0.3, inside=10.0, outside=1.0))
    assert _rel(r.A_H, _ga_aniso_oracle("ball", 3, N, 10.0, B)) <= 1e-10


def test_ga_upper_bound_decreasing_in_N(dev):
    """Nested trial spaces: the Ga a_H falls as N grows (Galerkin minimum)."""
    inc = dict(shape="ball", size=0.3, inside=10.0, outside=1.0)
    prev = None
    for N in (9, 15, 23):
        r = P.Solver(d=3, N=(N,) * 3, format="full", discretisation="ga", solver_tol=1e-12,
                     max_iter=3000).solve(inclusion=inc)
        a = r.A_H[0, 0]
        if prev is not None:
            assert a < prev + 1e-12
        prev = a


def test_ga_rejects_bad_inclusions(dev):
    s = P.Solver(d=2, N=(15, 15), format="full", discretisation="ga", solver_tol=1e-8, max_iter=100)
    with pytest.raises(Exception):
        s.solve(inclusion=dict(shape="ball", size=0.3, inside=10.0, outside=1.0))   # the ball is 3D
    with pytest.raises(Exception):
        s.solve(inclusion=dict(shape="square", size=0.6, inside=10.0, outside=1.0))  # size beyond 1/2
    with pytest.raises(Exception):
        s.solve(full=np.ones((15, 15)))                                              # Ga takes inclusions


# ---------------------------------------------------------------- low-rank Ga
@pytest.mark.parametrize("fmt,d,N", [("tt", 3, 9), ("tt", 3, 15), ("tt", 2, 21), ("cp", 2, 21)])
def test_lowrank_ga_untruncated_equals_oracle(dev, fmt, d, N):
    """The TT solve on the double grid, every train kept on T_N's frequencies;
    rank cap N (the dimension of T_N per axis): no truncation."""
    s = P.Solver(d=d, N=(N,) * d, format=fmt, discretisation="ga", rank_cap=N, solver_tol=1e-12, max_iter=400,
                 coeff_rank=2)
    r = s.solve(inclusion=dict(shape="square", size=0.3, inside=10.0, outside=1.0))
    o = G.solve(G.Inclusion("square", 0.3, 10.0, 1.0), [N] * d, tol=1e-12, max_iter=3000)
    assert _rel(r.A_H, o.A_H) <= 1e-10


def test_lowrank_ga_truncated_upper_bound(dev):
    """Truncated correctors in T_N: the exact Ga energy form bounds the Ga
    A_H from above (Sec. 4.3's identity holds for any Galerkin space)."""
    N = 21
    o = G.solve(G.Inclusion("square", 0.3, 10.0, 1.0), [N] * 3, tol=1e-12, max_iter=3000).A_H
    s = P.Solver(d=3, N=(N,) * 3, format="tt", discretisation="ga", rank_cap=6, solver_tol=1e-10, max_iter=150,
                 coeff_rank=2)
    r = s.solve(inclusion=dict(shape="square", size=0.3, inside=10.0, outside=1.0))
    D = r.A_H - o
    assert np.linalg.eigvalsh(0.5 * (D + D.T)).min() >= -1e-9 * np.max(np.abs(o))
    assert _rel(r.A_H, o) < 0.1


@pytest.mark.parametrize("fmt,d,N", [("tt", 3, 15), ("tt", 2, 21), ("cp", 2, 21)])
def test_lowrank_ga_with_anisotropy(dev, fmt, d, N):
    """Low-rank Ga with B, untruncated, against the oracle's Ga of a I + B
    and against the full-grid Ga with B."""
    B = W.anisotropy(d)
    inc = dict(shape="square", size=0.3, inside=10.0, outside=1.0)
    f = P.Solver(d=d, N=(N,) * d, format="full", discretisation="ga", solver_tol=1e-12, max_iter=3000,
                 aniso=B).solve(inclusion=inc)
    t = P.Solver(d=d, N=(N,) * d, format=fmt, discretisation="ga", rank_cap=N, solver_tol=1e-12, max_iter=400,
                 coeff_rank=2, aniso=B).solve(inclusion=inc)
    o = _ga_aniso_oracle("square", d, N, 10.0, B)
    assert _rel(t.A_H, o) <= 1e-10
    assert _rel(f.A_H, o) <= 1e-10


def test_lowrank_ga_ball_unsupported(dev):
    s = P.Solver(d=3, N=(9, 9, 9), format="tt", discretisation="ga", rank_cap=4, solver_tol=1e-6, max_iter=20)
    with pytest.raises(Exception):
        s.solve(inclusion=dict(shape="ball", size=0.3, inside=10.0, outside=1.0))
