"""Benchmark: A_H solves per second at 1e-6 relative A_H error on one MI355X.

Workload: 3D cell problem on a 135^3 grid with the smooth coefficient
a = 1 + 0.5 sum_{j=1..8} c_j prod_i cos(2 pi k_ji x_i + phi_ji) (seed 0; no
clipping occurs, CP rank 9).  One step = one A_H solve: the d = 3 correctors
(E = e_1, e_2, e_3) and the 3 x 3 energy matrix, inputs resident in HBM.

Equal-accuracy protocol: the reference A_H* is the full-grid FP64 PCG solve
to 1e-12 (validated against the CPU oracle by the GPU tests); each timed
path uses the loosest setting whose A_H error max|A - A*| / max|A*| is at
most 1e-6.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TARGET_ERR = 1e-6
N = 135
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def rel_err(A, B):
    return float(np.max(np.abs(A - B)) / np.max(np.abs(B)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget-s", type=float, default=30.0)
    ap.add_argument("--tt-steps", type=int, default=10)
    ap.add_argument("--no-tt", action="store_true", help="skip the tensor-train leg")
    ap.add_argument("--full-tol", type=float, default=None,
                    help="full-grid PCG tolerance (skips the sweep; the A_H error is still checked)")
    ap.add_argument("--tt-cap", type=int, default=None, help="TT rank cap (skips the cap sweep)")
    ap.add_argument("--tt-tol", type=float, default=None, help="TT solver tolerance (skips the tol sweep)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size first (scale for HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the path shards by "
              "independent correctors and requests, which this build does not launch.", file=sys.stderr)
        return 2

    import torch

    import paper_1902_07455_amd as P
    import workloads as W

    dev = "cuda:0"
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {n * 8} bytes read, {n * 8} bytes written")
        del src, dst
    p = W.smooth_params(0)
    cp = W.smooth_cp(N, p)
    a_np = cp.full()
    assert a_np.min() >= 0.1 and a_np.max() <= 10.0  # clipping inactive: rank 9 exact
    a_dev = torch.from_numpy(a_np).to(dev)
    torch.cuda.synchronize()

    # ---------------------------------------------------------------- reference
    log("reference A_H* (full grid, PCG to 1e-12)")
    ref = P.Solver(d=3, N=(N, N, N), format="full", solver_tol=1e-12, max_iter=500, device=dev)
    A_ref = ref.solve(full=a_dev).A_H
    ref.close()

    # ---------------------------------------------------------------- full-grid tolerance sweep
    full_tol = None
    sweep = []
    full_tols = [args.full_tol] if args.full_tol else [1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 3e-4, 1e-4, 3e-5,
                                                        1e-5, 1e-6, 1e-7, 1e-8]
    for tol in full_tols:
        s = P.Solver(d=3, N=(N, N, N), format="full", solver_tol=tol, max_iter=500, device=dev)
        r = s.solve(full=a_dev)
        e = rel_err(r.A_H, A_ref)
        sweep.append((tol, e, int(r.iters.max())))
        s.close()
        if e <= TARGET_ERR:
            full_tol = tol
            break
    log(f"full-grid sweep (tol, err, iters): {sweep}")
    assert full_tol is not None

    solver = P.Solver(d=3, N=(N, N, N), format="full", solver_tol=full_tol, max_iter=500, device=dev)
    for _ in range(args.warmup):
        r = solver.solve(full=a_dev)
    torch.cuda.synchronize()

    # ---------------------------------------------------------------- timed region
    P.prof_enable("fft_axis2")
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        r = solver.solve(full=a_dev)    # returns after the stream is synchronised
        lat.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nlaunch, kms = P.prof_read()
    P.prof_enable(None)
    err = rel_err(r.A_H, A_ref)
    total = t1 - t0
    value = args.steps / total
    iters = int(r.iters.max())

    # dominant kernel: axis-2 FFT pass of the matvec, all 3 correctors x 3
    # gradient components per launch; algorithmic bytes = read + write of
    # 9 half spectra of N*N*(N+1)/2 complex FP64 values.
    S = N * N * ((N + 1) // 2)
    bytes_per_launch = 2 * 9 * S * 16
    avg_s = (kms / 1e3) / max(nlaunch, 1)
    achieved = bytes_per_launch / avg_s / 1e9
    roofline = {"bound": "hbm", "kernel": "fft_axis2 (k_fft_lines, axis-2 pass of the PCG matvec)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "launches": nlaunch, "avg_us": round(avg_s * 1e6, 2),
                "bytes_per_launch": bytes_per_launch}

    out = {
        "metric": "A_H solves/sec at 1e-6 rel. err (TT vs full-FFT, same GPU); p50/p99 latency",
        "value": round(value, 3),
        "unit": "A_H solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D cell problem, N=135^3, smooth coefficient (8 cosine products, "
                               "seed 0, CP rank 9), E=e1,e2,e3, A_H to 1e-6 relative error",
                   "path": "full-grid FFT PCG", "solver_tol": full_tol, "iters": iters,
                   "A_H_rel_err": err},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3)},
        "full_fft": {"solves_per_s": round(value, 3), "solver_tol": full_tol, "iters": iters,
                     "A_H_rel_err": err, "sweep": sweep},
        "roofline": roofline,
    }

    # ---------------------------------------------------------------- TT leg
    if not args.no_tt:
        w_dev = torch.from_numpy(cp.weights).to(dev)
        f_dev = [torch.from_numpy(f).to(dev) for f in cp.factors]

        def tt_solver(cap, tol):
            return P.Solver(d=3, N=(N, N, N), format="tt", rank_cap=cap, trunc_tol=0.0,
                            solver_tol=tol, max_iter=100, coeff_rank=cp.rank, device=dev)

        tt_sweep = []
        tt_cap = None
        for cap in ([args.tt_cap] if args.tt_cap else [4, 6, 8, 10, 12, 16, 20]):
            s = tt_solver(cap, 1e-8)
            r = s.solve(cp=(w_dev, f_dev))
            e = rel_err(r.A_H, A_ref)
            tt_sweep.append(("cap", cap, e, r.iters.tolist()))
            s.close()
            if e <= TARGET_ERR:
                tt_cap = cap
                break
        tt_tol = None
        if tt_cap is not None:
            for tol in ([args.tt_tol] if args.tt_tol else [1e-2, 3e-3, 1e-3, 3e-4, 1e-4, 1e-5, 1e-6, 1e-8]):
                s = tt_solver(tt_cap, tol)
                r = s.solve(cp=(w_dev, f_dev))
                e = rel_err(r.A_H, A_ref)
                tt_sweep.append(("tol", tol, e, r.iters.tolist()))
                s.close()
                if e <= TARGET_ERR:
                    tt_tol = tol
                    break
        log(f"TT sweep: {tt_sweep}")
        if tt_tol is not None:
            tts = tt_solver(tt_cap, tt_tol)
            r = tts.solve(cp=(w_dev, f_dev))
            torch.cuda.synchronize()
            tlat = []
            t0 = time.perf_counter()
            for _ in range(args.tt_steps):
                ts = time.perf_counter()
                r = tts.solve(cp=(w_dev, f_dev))
                tlat.append((time.perf_counter() - ts) * 1e3)
            torch.cuda.synchronize()
            ttot = time.perf_counter() - t0
            terr = rel_err(r.A_H, A_ref)
            out["tt"] = {"solves_per_s": round(args.tt_steps / ttot, 3), "rank_cap": tt_cap,
                         "solver_tol": tt_tol, "iters": r.iters.tolist(), "ranks": r.ranks.tolist(),
                         "A_H_rel_err": terr, "ms_per_solve": round(1e3 * ttot / args.tt_steps, 3),
                         "latency_ms": {"p50": round(float(np.percentile(tlat, 50)), 3),
                                        "p99": round(float(np.percentile(tlat, 99)), 3)},
                         "sweep": tt_sweep}
        else:
            out["tt"] = {"solves_per_s": None, "sweep": tt_sweep}

    # ---------------------------------------------------------------- CPU oracle baseline
    if not args.no_cpu:
        from oracle import fg
        log("CPU oracle baseline")
        t = time.perf_counter()
        o = fg.solve(a_np, [[1.0, 0.0, 0.0]], tol=full_tol, max_iter=500)
        one = time.perf_counter() - t
        out["cpu_baseline"] = {
            "value": round(1.0 / (3.0 * one), 5), "unit": "A_H solves/s", "cores": 1,
            "kind": "oracle",
            "sample": f"oracle.fg full-grid PCG, one corrector (E=e1) of the 135^3 workload at "
                      f"tol {full_tol} ({o.iters[0]} iterations, {one:.1f} s), scaled x3 to one "
                      "A_H solve; numpy FFT single-threaded"}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
