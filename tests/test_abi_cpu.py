"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/lrfg.h declares, and validates arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lrfg.h")


def _lib():
    from paper_1902_07455_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("liblrfg.so not built (run __graft_entry__.build())")
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lrfg_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    L = _lib()
    lib = C.CDLL(L.LIB_PATH)
    names = declared_functions()
    assert "lrfg_solve" in names and "lrfg_plan_create" in names
    for n in names:
        assert hasattr(lib, n), f"{n} declared in lrfg.h but not exported"
    assert set(L.EXPORTS) <= set(names)


def test_version_and_status_strings():
    L = _lib()
    lib = L.lib()
    assert lib.lrfg_abi_version() == 2
    for s in (0, 1, 2, -1, -2, -3, -4, -5):
        assert len(lib.lrfg_status_string(s)) > 0


def test_ga_double_grid():
    """The smallest odd 3^a 5^b >= 2N - 1 (2N - 1 beyond 2025); bad N rejected."""
    L = _lib()
    lib = L.lib()
    smooth = sorted(3 ** a * 5 ** b for a in range(8) for b in range(6) if 3 ** a * 5 ** b <= 2048)
    for N in (1, 3, 13, 15, 23, 63, 203, 243, 313, 609, 939, 1013):
        want = next(m for m in smooth if m >= 2 * N - 1)
        assert lib.lrfg_ga_double_grid(N) == want
    assert [lib.lrfg_ga_double_grid(N) for N in (15, 63, 203, 243, 939)] == [45, 125, 405, 625, 2025]
    assert lib.lrfg_ga_double_grid(1015) == 2029 and lib.lrfg_ga_double_grid(1023) == 2045
    for bad in (0, -3, 4, 1025):
        assert lib.lrfg_ga_double_grid(bad) == -1


def _problem(L, **kw):
    p = L.Problem()
    p.d = kw.get("d", 3)
    for i, n in enumerate(kw.get("N", (15, 15, 15))):
        p.N[i] = n
    p.format = kw.get("format", L.FORMAT_FULL)
    p.rank_cap = kw.get("rank_cap", 10)
    p.trunc_tol = kw.get("trunc_tol", 0.0)
    p.solver_tol = kw.get("solver_tol", 1e-8)
    p.max_iter = kw.get("max_iter", 100)
    p.solver = kw.get("solver", L.SOLVER_PCG)
    p.precision = kw.get("precision", L.PREC_FP64)
    p.precond_terms = kw.get("precond_terms", 0)
    p.oversample = kw.get("oversample", 0)
    p.coeff_rank = kw.get("coeff_rank", 0)
    p.seed = 0
    p.flags = kw.get("flags", 0)
    for i, v in enumerate(kw.get("aniso", ())):
        p.aniso[i] = v
    p.rank_start = kw.get("rank_start", 0)
    return p


@pytest.mark.parametrize("kw,code", [
    (dict(d=4), -1),
    (dict(N=(14, 15, 15)), -1),
    (dict(N=(1, 15, 15)), -1),
    (dict(d=3, format=1), -1),                 # CP needs d = 2
    (dict(format=3, rank_cap=0), -1),
    (dict(solver_tol=0.0), -1),
    (dict(solver_tol=float("nan")), -1),
    (dict(trunc_tol=-1.0), -1),
    (dict(max_iter=0), -1),
    (dict(flags=1), -1),
    (dict(precond_terms=1), -1),
    (dict(precision=1), -5),                   # full grid is FP64 only
    (dict(solver=1), -5),                      # full grid uses PCG
    (dict(d=2, N=(15, 15), format=2), -5),     # Tucker path is d = 3 only
    (dict(N=(131, 131, 131), format=2, rank_cap=129), -5),  # sketch sizes beyond 128
    (dict(N=(131, 131, 131), format=3, rank_cap=129), -5),
    (dict(format=3, coeff_rank=129), -5),               # coefficient ranks beyond 128
    (dict(aniso=(1, 0.5, 0, 0.4, 1, 0, 0, 0, 1)), -1),  # B not symmetric
    (dict(aniso=(1, 2, 0, 2, 1, 0, 0, 0, 1)), -1),      # B indefinite (2 x 2 minor < 0)
    (dict(aniso=(1, 0, 0, 0, -1e-3, 0, 0, 0, 1)), -1),  # negative diagonal entry
    (dict(aniso=(2, 1, 1, 1, 2, -1, 1, -1, 0.5)), -1),  # minors of order 2 fine, det < 0
    (dict(aniso=(1, 0, 0, 0, 1, 0, 0, 0, float("inf"))), -1),
    (dict(d=2, N=(15, 15), aniso=(1, 0, 0, 1, 1)), -1),  # entry past d x d
    (dict(format=2, aniso=(1, 0, 0, 0, 1, 0, 0, 0, 1)), -5),  # Tucker: isotropic only
    (dict(format=3, rank_start=-1), -1),
    (dict(format=3, rank_start=4, solver=1), -5),     # rank-adaptive: PCG only
    (dict(format=3, rank_start=4, precision=1), -5),  # rank-adaptive: FP64 only
    (dict(format=2, rank_start=4), -5),               # rank-adaptive: TT/CP only
    (dict(rank_start=4), -5),                         # not the full grid
])
def test_plan_validation(kw, code):
    L = _lib()
    lib = L.lib()
    plan = C.c_void_p()
    rc = lib.lrfg_plan_create(C.byref(_problem(L, **kw)), C.byref(plan))
    assert rc == code
    assert not plan.value
    assert len(lib.lrfg_last_error()) > 0


@pytest.mark.parametrize("d,B", [
    (2, (5.5, -4.5, -4.5, 5.5)),
    (3, (4.25, -3.25, -1.25 * 2 ** 0.5, -3.25, 4.25, 1.25 * 2 ** 0.5, -1.25 * 2 ** 0.5, 1.25 * 2 ** 0.5, 7.5)),
    (3, (1, 1, 0, 1, 1, 0, 0, 0, 0)),           # singular PSD is admissible
])
def test_plan_accepts_psd_anisotropy(d, B):
    L = _lib()
    lib = L.lib()
    for fmt in (L.FORMAT_FULL, L.FORMAT_TT):
        plan = C.c_void_p()
        N = (15,) * d + (1,) * (3 - d)
        rc = lib.lrfg_plan_create(C.byref(_problem(L, d=d, N=N, format=fmt, aniso=B)), C.byref(plan))
        assert rc == 0, lib.lrfg_last_error()
        lib.lrfg_plan_destroy(plan)


def test_plan_and_workspace_sizes():
    L = _lib()
    lib = L.lib()
    plan = C.c_void_p()
    assert lib.lrfg_plan_create(C.byref(_problem(L, N=(45, 45, 45))), C.byref(plan)) == 0
    nb = C.c_size_t()
    assert lib.lrfg_plan_workspace_bytes(plan, 3, C.byref(nb)) == 0
    S = 45 * 45 * 23 * 16
    assert nb.value >= 3 * 7 * S            # x, r, p, q and d gradients per E
    nb1 = C.c_size_t()
    assert lib.lrfg_plan_workspace_bytes(plan, 1, C.byref(nb1)) == 0
    assert nb1.value < nb.value
    assert lib.lrfg_plan_workspace_bytes(plan, 0, C.byref(nb1)) == -1
    lib.lrfg_plan_destroy(plan)
    lib.lrfg_plan_destroy(None)


def test_tucker_workspace_one_microstructure_at_a_time():
    """Tucker batches run one microstructure after another, so the workspace
    for k microstructures of 3 fields is the one for 3 fields."""
    L = _lib()
    lib = L.lib()
    plan = C.c_void_p()
    assert lib.lrfg_plan_create(C.byref(_problem(L, N=(45, 45, 45), format=2, rank_cap=8)), C.byref(plan)) == 0
    sz = []
    for n in (1, 3, 6, 12):
        nb = C.c_size_t()
        assert lib.lrfg_plan_workspace_bytes(plan, n, C.byref(nb)) == 0
        sz.append(nb.value)
    lib.lrfg_plan_destroy(plan)
    assert sz[0] < sz[1] == sz[2] == sz[3]
    # at least x, r, p, q, z and the mode frames of 3 systems
    assert sz[1] >= 3 * 5 * 3 * 45 * 8 * 8


def test_tucker_mixed_precision_workspace():
    """Mixed precision adds the refinement's b0, x and best-x Tucker tensors
    (three systems' frames and cores) on top of the FP64 workspace."""
    L = _lib()
    lib = L.lib()
    sz = {}
    for prec in (0, 1, 2):
        plan = C.c_void_p()
        pr = _problem(L, N=(45, 45, 45), format=2, rank_cap=8, precision=prec)
        assert lib.lrfg_plan_create(C.byref(pr), C.byref(plan)) == 0
        nb = C.c_size_t()
        assert lib.lrfg_plan_workspace_bytes(plan, 3, C.byref(nb)) == 0
        lib.lrfg_plan_destroy(plan)
        sz[prec] = nb.value
    extra = 3 * 3 * (3 * 45 * 8 + 8 ** 3) * 8
    assert sz[1] == sz[2] >= sz[0] + extra


def test_solve_rejects_bad_workspace_before_device():
    L = _lib()
    lib = L.lib()
    plan = C.c_void_p()
    assert lib.lrfg_plan_create(C.byref(_problem(L, d=2, N=(9, 9, 1))), C.byref(plan)) == 0
    c = L.Coeff()
    buf = (C.c_double * 81)()
    c.full = C.addressof(buf)
    r = L.Result()
    # misaligned / too small workspace: EWORKSPACE without any device call
    assert lib.lrfg_solve(plan, C.byref(c), None, 2, C.c_void_p(8), 16, None, C.byref(r)) == -3
    # nE must equal d when E is NULL
    assert lib.lrfg_solve(plan, C.byref(c), None, 1, C.c_void_p(256), 1 << 30, None, C.byref(r)) == -1
    lib.lrfg_plan_destroy(plan)


def test_server_validation_before_device():
    lib = _lib().lib()
    h = C.c_void_p()
    buf = (C.c_double * 64)()
    # slots / batch / pool checks come before any device call
    assert lib.lrfg_server_create(0, 0, 4, C.addressof(buf), 1 << 20, C.byref(h)) == -1
    assert lib.lrfg_server_create(0, 17, 4, C.addressof(buf), 1 << 20, C.byref(h)) == -1
    assert lib.lrfg_server_create(0, 2, 0, C.addressof(buf), 1 << 20, C.byref(h)) == -1
    assert lib.lrfg_server_create(0, 2, 4, None, 1 << 20, C.byref(h)) == -1
    assert lib.lrfg_server_create(0, 2, 4, C.addressof(buf) + 8, 1 << 20, C.byref(h)) == -1
    n = C.c_int()
    assert lib.lrfg_server_submit(None, None, None, None, 3, None, 0, None) == -1
    assert lib.lrfg_server_poll(None, None, 0, C.byref(n), 0) == -1
    assert lib.lrfg_server_pending(None) == 0
    lib.lrfg_server_destroy(None)


def test_solve_batch_validation_before_device():
    L = _lib()
    lib = L.lib()
    plan = C.c_void_p()
    assert lib.lrfg_plan_create(C.byref(_problem(L, d=2, N=(9, 9, 1))), C.byref(plan)) == 0
    cs = (L.Coeff * 2)()
    rs = (L.Result * 2)()
    # count < 1
    assert lib.lrfg_solve_batch(plan, cs, 0, None, 2, C.c_void_p(256), 1 << 30, None, rs) == -1
    # misaligned workspace
    assert lib.lrfg_solve_batch(plan, cs, 2, None, 2, C.c_void_p(8), 1 << 30, None, rs) == -3
    lib.lrfg_plan_destroy(plan)


def test_tucker_coefficient_validation_before_device():
    """Tucker coefficients go with the Tucker format only, need all three
    frames and ranks in [1, N]; checked before any device work (the
    workspace pointer below is never dereferenced)."""
    L = _lib()
    lib = L.lib()
    core = (C.c_double * 8)()
    frame = (C.c_double * 30)()

    def tucker_coeff(ranks=(2, 2, 2), frames=3):
        c = L.Coeff()
        c.tucker_core = C.cast(core, C.c_void_p)
        for j in range(3):
            c.tucker_ranks[j] = ranks[j]
            if j < frames:
                c.tucker_frames[j] = C.cast(frame, C.c_void_p)
        return c

    r = L.Result()
    for fmt, code in ((3, -5), (0, -5)):           # TT and full-grid plans refuse it
        plan = C.c_void_p()
        assert lib.lrfg_plan_create(C.byref(_problem(L, N=(15, 15, 15), format=fmt, rank_cap=4)), C.byref(plan)) == 0
        assert lib.lrfg_solve(plan, C.byref(tucker_coeff()), None, 3, C.c_void_p(256), 1 << 40, None,
                              C.byref(r)) == code
        lib.lrfg_plan_destroy(plan)
    plan = C.c_void_p()
    assert lib.lrfg_plan_create(C.byref(_problem(L, N=(15, 15, 15), format=2, rank_cap=4)), C.byref(plan)) == 0
    # a missing frame, a rank above N
    assert lib.lrfg_solve(plan, C.byref(tucker_coeff(frames=2)), None, 3, C.c_void_p(256), 1 << 40, None,
                          C.byref(r)) == -1
    assert lib.lrfg_solve(plan, C.byref(tucker_coeff(ranks=(2, 16, 2))), None, 3, C.c_void_p(256), 1 << 40, None,
                          C.byref(r)) == -1
    # a TT coefficient on the Tucker plan
    c = L.Coeff()
    c.tt_cores[0] = C.cast(core, C.c_void_p)
    assert lib.lrfg_solve(plan, C.byref(c), None, 3, C.c_void_p(256), 1 << 40, None, C.byref(r)) == -5
    lib.lrfg_plan_destroy(plan)


def test_gram_cut_validation_before_device():
    lib = _lib().lib()
    buf = (C.c_double * 16)()
    # n out of range, c < 1, negative / NaN tol, null pointers: EINVAL, no device call
    assert lib.lrfg_gram_cut(129, 4, C.addressof(buf), 1, 0.0, C.addressof(buf), None, None, None) == -1
    assert lib.lrfg_gram_cut(0, 4, C.addressof(buf), 1, 0.0, C.addressof(buf), None, None, None) == -1
    assert lib.lrfg_gram_cut(4, 0, C.addressof(buf), 1, 0.0, C.addressof(buf), None, None, None) == -1
    assert lib.lrfg_gram_cut(4, 2, C.addressof(buf), 1, -1.0, C.addressof(buf), None, None, None) == -1
    assert lib.lrfg_gram_cut(4, 2, C.addressof(buf), 1, float("nan"), C.addressof(buf), None, None, None) == -1
    assert lib.lrfg_gram_cut(4, 2, None, 1, 0.0, C.addressof(buf), None, None, None) == -1
    # empty batch: nothing to do
    assert lib.lrfg_gram_cut(4, 2, C.addressof(buf), 0, 0.0, C.addressof(buf), None, None, None) == 0


def test_compress_tucker_validation_before_device():
    """Bad sizes or pointers are refused before any device work; the
    workspace size grows with the grid and the cap."""
    lib = _lib().lib()
    N = (C.c_int * 3)(15, 17, 19)
    n1 = lib.lrfg_compress_tucker_workspace_bytes(N, 6, 10)
    n2 = lib.lrfg_compress_tucker_workspace_bytes(N, 12, 10)
    assert 0 < n1 < n2
    assert lib.lrfg_compress_tucker_workspace_bytes(N, 0, 10) == 0
    assert lib.lrfg_compress_tucker_workspace_bytes((C.c_int * 3)(15, 0, 19), 6, 10) == 0
    buf = (C.c_double * 16)()
    frames = (C.c_void_p * 3)(C.addressof(buf), C.addressof(buf), C.addressof(buf))
    ranks = (C.c_int * 3)()
    # null field, null outputs, negative or NaN tolerance, cap < 1
    assert lib.lrfg_compress_tucker(N, None, 6, 0.0, 10, 0, frames, C.addressof(buf), ranks, None,
                                    C.c_void_p(256), n1, None) == -1
    assert lib.lrfg_compress_tucker(N, C.addressof(buf), 6, 0.0, 10, 0, None, C.addressof(buf), ranks, None,
                                    C.c_void_p(256), n1, None) == -1
    assert lib.lrfg_compress_tucker(N, C.addressof(buf), 6, -1.0, 10, 0, frames, C.addressof(buf), ranks, None,
                                    C.c_void_p(256), n1, None) == -1
    assert lib.lrfg_compress_tucker(N, C.addressof(buf), 6, float("nan"), 10, 0, frames, C.addressof(buf), ranks,
                                    None, C.c_void_p(256), n1, None) == -1
    assert lib.lrfg_compress_tucker(N, C.addressof(buf), 0, 0.0, 10, 0, frames, C.addressof(buf), ranks, None,
                                    C.c_void_p(256), n1, None) == -1
    # workspace below the reported size
    assert lib.lrfg_compress_tucker(N, C.addressof(buf), 6, 0.0, 10, 0, frames, C.addressof(buf), ranks, None,
                                    C.c_void_p(256), n1 - 1024, None) == -3


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES") is None and not os.path.exists("/dev/kfd"),
                    reason="no ROCm device nodes")
def test_device_check_runs():
    L = _lib()
    assert L.lib().lrfg_device_check() in (0, -4)


def test_product_path_does_not_import_oracle():
    """The package never imports the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_1902_07455_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.findall(r"(?:import|from)\s+(\w+)", text), f


def test_noalloc_oversized_refused_before_device():
    """lrfg_solve_noalloc refuses a plan whose workspace exceeds the
    library's array (LRFG_EWORKSPACE) before touching a device."""
    L = _lib()
    lib = L.lib()
    plan = C.c_void_p()
    assert lib.lrfg_plan_create(C.byref(_problem(L, N=(135, 135, 135), format=3, rank_cap=16, coeff_rank=9)),
                                C.byref(plan)) == 0
    nb = C.c_size_t()
    assert lib.lrfg_plan_workspace_bytes(plan, 3, C.byref(nb)) == 0
    assert nb.value > (128 << 20)
    c = L.Coeff()
    r = L.Result()
    assert lib.lrfg_solve_noalloc(plan, C.byref(c), None, 3, None, C.byref(r)) == -3
    assert b"allocation-free" in lib.lrfg_last_error()
    lib.lrfg_plan_destroy(plan)
