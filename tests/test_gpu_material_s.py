"""The paper's stochastic material S (Sec. 4.1, eq. shape_fun2) compressed to
TT rank 10 (as the paper did): full grid and TT on the compressed field
against the CPU oracle."""
import numpy as np
import pytest

import paper_1902_07455_amd as P
import workloads as W
from oracle import fg
from oracle import fg_tensor as FT

pytestmark = pytest.mark.gpu


def _rel(A, B):
    return np.max(np.abs(A - B)) / np.max(np.abs(B))


def _compressed(N, dev):
    import torch
    a0 = torch.from_numpy(W.material_s(N, 3, seed=0)).to(dev)
    cores, (k1, k2) = P.compress_tt(a0, cap=10, tol=0.0, seed=2)
    tt = [cores[0][:, :, :k1].contiguous(), cores[1][:k1, :, :k2].contiguous(), cores[2][:k2].contiguous()]
    full = np.einsum("ia,ajb,bk->ijk", tt[0][0].cpu().numpy(), tt[1].cpu().numpy(), tt[2][:, :, 0].cpu().numpy())
    return a0.cpu().numpy(), tt, full, (k1, k2)


def test_material_s_rank10_compression(dev):
    a0, tt, full, kept = _compressed(45, dev)
    assert max(kept) <= 10
    assert np.linalg.norm(full - a0) / np.linalg.norm(a0) < 1e-2
    assert full.min() > 0.5


@pytest.mark.parametrize("aniso", [False, True])
def test_material_s_full_grid_equals_oracle(dev, aniso):
    _, _, full, _ = _compressed(45, dev)
    B = W.anisotropy(3) if aniso else None
    s = P.Solver(d=3, N=(45,) * 3, format="full", solver_tol=1e-12, max_iter=2000, aniso=B)
    r = s.solve(full=full)
    o = FT.solve(FT.isotropic_plus_constant(full, B), tol=1e-12) if aniso else fg.solve(full, tol=1e-12)
    assert _rel(r.A_H, o.A_H) <= 1e-10


def test_material_s_tt_untruncated_equals_oracle(dev):
    _, tt, full, kept = _compressed(21, dev)
    s = P.Solver(d=3, N=(21,) * 3, format="tt", rank_cap=21, solver_tol=1e-12, max_iter=300, coeff_rank=max(kept))
    r = s.solve(tt=tt)
    assert _rel(r.A_H, fg.solve(full, tol=1e-12).A_H) <= 1e-10


def test_material_s_tt_truncated_bound(dev):
    _, tt, full, kept = _compressed(45, dev)
    o = fg.solve(full, tol=1e-12).A_H
    s = P.Solver(d=3, N=(45,) * 3, format="tt", rank_cap=8, solver_tol=1e-8, max_iter=150, coeff_rank=max(kept))
    r = s.solve(tt=tt)
    D = r.A_H - o
    assert np.linalg.eigvalsh(0.5 * (D + D.T)).min() >= -1e-9 * np.max(np.abs(o))
    assert _rel(r.A_H, o) < 1e-3
