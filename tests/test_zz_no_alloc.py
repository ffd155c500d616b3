"""The allocation-free solve (lrfg_solve_noalloc, the library's own device
workspace) against lrfg_solve with a caller workspace, through the C ABI:
the same A_H, iteration counts and statuses, on two calls in a row with
the second problem smaller than the first (the shared device array keeps
the first call's contents)."""
import ctypes as C

import numpy as np
import pytest

import paper_1902_07455_amd as P
from paper_1902_07455_amd import _lib
import workloads as W

pytestmark = pytest.mark.gpu


def _plan(L, **kw):
    p = P._make_problem(**kw)
    plan = C.c_void_p()
    assert L.lrfg_plan_create(C.byref(p), C.byref(plan)) == 0, L.lrfg_last_error()
    return plan


def _call(L, plan, coeff_kw, E, d, max_iter, dev, noalloc):
    import torch
    h = P._Held(dev)
    c = _lib.Coeff()
    P._fill_coeff(c, h, **coeff_kw)
    nE = d if E is None else len(E)
    Eptr = None
    if E is not None:
        Earr = np.ascontiguousarray(np.asarray(E, dtype=np.float64))
        h.keep.append(Earr)
        Eptr = Earr.ctypes.data
    r = _lib.Result()
    bufs = P._result_buffers(r, nE, d, max_iter)
    stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    if noalloc:
        rc = L.lrfg_solve_noalloc(plan, C.byref(c), Eptr, nE, stream, C.byref(r))
    else:
        nb = C.c_size_t()
        assert L.lrfg_plan_workspace_bytes(plan, nE, C.byref(nb)) == 0
        ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        rc = L.lrfg_solve(plan, C.byref(c), Eptr, nE, C.c_void_p(ws.data_ptr()), nb.value, stream, C.byref(r))
    assert rc in (0, 1, 2), (rc, L.lrfg_last_error())
    return rc, bufs


def _same(a, b):
    rca, (A1, it1, h1, rk1, st1) = a
    rcb, (A2, it2, h2, rk2, st2) = b
    assert rca == rcb
    assert np.max(np.abs(A1 - A2)) <= 1e-12 * np.max(np.abs(A2))
    assert np.array_equal(it1, it2) and np.array_equal(st1, st2)


CASES = {
    # (problem, coefficient, E, max_iter): the first of each pair is the larger
    "tt": [(dict(d=3, N=(21, 21, 21), format="tt", rank_cap=8, solver_tol=1e-10, max_iter=80, coeff_rank=2),
            "cube21", None, 80),
           (dict(d=3, N=(15, 15, 15), format="tt", rank_cap=6, solver_tol=1e-10, max_iter=80, coeff_rank=2),
            "cube15", [[1.0, 0.0, 0.0]], 80)],
    "full": [(dict(d=2, N=(45, 45), format="full", solver_tol=1e-10, max_iter=500), "square45", None, 500),
             (dict(d=2, N=(25, 25), format="full", solver_tol=1e-10, max_iter=500), "square25",
              [[1.0, 0.5]], 500)],
}


def _coeff(name):
    if name.startswith("cube"):
        cp = W.cube_cp(int(name[4:]), 10.0)
        return dict(cp=(cp.weights, cp.factors))
    return dict(full=W.square_coeff(int(name[6:]), 2))


@pytest.mark.parametrize("fmt", ["tt", "full"])
def test_noalloc_equals_solve_twice(dev, fmt):
    L = _lib.lib()
    for prob, cname, E, mi in CASES[fmt]:
        plan = _plan(L, **prob)
        try:
            d = prob["d"]
            kw = _coeff(cname)
            got = _call(L, plan, kw, E, d, mi, dev, noalloc=True)
            want = _call(L, plan, kw, E, d, mi, dev, noalloc=False)
            _same(got, want)
        finally:
            L.lrfg_plan_destroy(plan)


def test_noalloc_rejects_oversized_plan(dev):
    """A plan whose workspace exceeds the library's array is refused with
    LRFG_EWORKSPACE before any device work."""
    L = _lib.lib()
    plan = _plan(L, d=3, N=(135, 135, 135), format="tt", rank_cap=16, solver_tol=1e-8, max_iter=10,
                 coeff_rank=9)
    try:
        cp = W.smooth_cp(135, W.smooth_params(0))
        h = P._Held(dev)
        c = _lib.Coeff()
        P._fill_coeff(c, h, cp=(cp.weights, cp.factors))
        r = _lib.Result()
        P._result_buffers(r, 3, 3, 10)
        assert L.lrfg_solve_noalloc(plan, C.byref(c), None, 3, None, C.byref(r)) == -3
        assert b"allocation-free" in L.lrfg_last_error()
    finally:
        L.lrfg_plan_destroy(plan)
