"""Benchmark of the twisted-mass clover propagator solve on one MI355X.

Workload (one step): 12 spin-colour point-source columns on a 24^3 x 64
lattice (the MILC12 shape and masses of Table 1: m = -0.0695, c_sw = 1.0509,
twist mu = 0.01), links exp(i 0.2 H) from seed 1001, solved with the
even-odd (symmetric Schur) BiCGStab in FP32 storage with FP64 reliable
updates to a 1e-10 FP64 relative true residual of the full operator.  Gauge
field, clover term and sources are resident in HBM before the timed region.

Printed: one JSON line with solves/s (columns converged per second), the
roofline of the dominant stencil kernel (HIP-event average duration and its
algorithmic bytes), the plain FP64 single-column solver for comparison, and
the FP64 CPU oracle timed on a bounded slab of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dslash HBM GB/s (% peak); solves/s at 1e-10 mixed vs FP64; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
LAT = (24, 24, 24, 64)
M, CSW, MU = -0.0695, 1.0509, 0.01
EPS, SEED = 0.2, 1001


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stencil_bytes_per_site(epi: str, n_rhs: int) -> float:
    """Algorithmic bytes per output site of one FP32 Schur half-application:
    8 links (18 reals) + the site inverse (2 x 36 complex) read once, each
    input column read once, each output column written once (+ x for the
    second half)."""
    links = 8 * 18 * 4
    clov = 144 * 4
    spin = 24 * 4
    # xmyd also reads rhat for the fused <rhat, v>; xmyt reuses x for <t, s>
    nfield = {"clovinv": 2, "xmy": 3, "xmyd": 4, "xmyt": 3}[epi]
    return links + clov + n_rhs * nfield * spin


def cpu_baseline(n_iter_fp64: int, n_rhs: int):
    """FP64 oracle on a 24^3 x 8 slab (1/8 of the volume), one core: setup of
    the even-odd operator plus two Schur applications, scaled to the full
    volume and to a whole solve with the FP64 GPU solver's iteration count."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import wilson as W

    slab = (24, 24, 24, 8)
    U = synth.su3_field(slab, EPS, SEED)
    b = synth.point_sources(slab)[0]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        eo = W.EvenOdd(U, M, CSW, MU)
        t1 = time.perf_counter()
        y = eo.mhat(b)
        y = eo.mhat(y)
        t2 = time.perf_counter()
    assert np.isfinite(y).all()
    scale = (LAT[3] / slab[3])
    t_setup = (t1 - t0) * scale
    t_mhat = (t2 - t1) / 2 * scale
    per_col = t_setup / n_rhs + 2 * n_iter_fp64 * t_mhat
    return {"value": 1.0 / per_col, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 numpy oracle, 1 thread: EvenOdd setup + 2 Schur applications on a 24^3x8 slab "
                       f"({t2 - t0:.1f} s), scaled x{scale:.0f} to 24^3x64 and to {2 * n_iter_fp64} Schur "
                       f"applications per column (FP64 GPU BiCGStab iterations) + setup/{n_rhs}; extrapolated"),
            "t_setup_s": t_setup, "t_schur_s": t_mhat}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 single-column comparison")
    ap.add_argument("--recon12", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is not part of this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2201_09004_amd import lq as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n_rhs = 12
    log("generating synthetic gauge field", LAT)
    U = synth.su3_field(LAT, EPS, SEED)
    b_host = synth.point_sources(LAT)
    U_d = torch.from_numpy(U).to(dev)
    b_d = torch.from_numpy(b_host).to(dev)
    x_d = torch.zeros_like(b_d)
    del U
    ctx = L.lq_init(0)
    field = L.lq_gauge_load(ctx, LAT, U_d)
    del U_d
    act = L.action(L.LQ_TM_CLOVER, m=M, mu=MU, c_sw=CSW)
    prm = L.params(tol=1e-10, sloppy_bits=32, recon12=args.recon12)

    log("warmup")
    for _ in range(args.warmup):
        x_d.zero_()
        _, st = L.lq_solve(ctx, act, field, prm, b_d, x_d)
        log("warmup stats", st)
    torch.cuda.synchronize()
    L.lq_profile(ctx, True)
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = L.lq_solve(ctx, act, field, prm, b_d, x_d)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / args.steps * 1e3
    value = n_rhs * args.steps / (t1 - t0)
    worst = max(s["true_rel_res"] for s in stats)
    ok = all(s["status"] == 0 for s in stats) and worst <= 1e-10
    log("timed", args.steps, "steps:", ms_step, "ms/step; worst residual", worst)

    # roofline of the dominant stencil kernel from the HIP events of the timed region
    kernels = {}
    for name in ("wilson32_clovinv", "wilson32_xmy", "wilson32_xmyd", "wilson32_xmyt", "wilson64_clovinv",
                 "wilson64_xmy", "wilson64_site", "wilson64_xpay", "blas", "site"):
        n, avg = L.lq_profile_get(ctx, name)
        if n:
            kernels[name] = {"count": n, "avg_ms": avg, "total_ms": n * avg}
    L.lq_profile(ctx, False)
    dom = max((k for k in kernels if k.startswith("wilson32")), key=lambda k: kernels[k]["total_ms"])
    Vh = int(np.prod(LAT)) // 2
    epi = dom.split("_")[1]
    alg_bytes = stencil_bytes_per_site(epi, n_rhs) * Vh
    achieved = alg_bytes / (kernels[dom]["avg_ms"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                "alg_bytes_per_launch": alg_bytes, "avg_ms": kernels[dom]["avg_ms"]}

    fp64 = None
    if not args.no_fp64:
        log("FP64 single-column solve")
        p64 = L.params(tol=1e-10, sloppy_bits=64)
        b1 = b_d[:1].contiguous()
        x1 = torch.zeros_like(b1)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        _, st64 = L.lq_solve(ctx, act, field, p64, b1, x1)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        fp64 = {"solves_per_s": 1.0 / (tb - ta), "seconds": tb - ta, "iters": st64["iters"],
                "true_rel_res": st64["true_rel_res"]}
        log("fp64", fp64)

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        n_it = fp64["iters"] if fp64 else max(s["iters"] for s in stats)
        cpu = cpu_baseline(n_it, n_rhs)
        log("cpu", cpu)

    L.lq_field_free(field)
    L.lq_finalize(ctx)
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tm_clover_eo_bicgstab_24x24x24x64_12rhs", "lattice": list(LAT), "n_rhs": n_rhs,
                   "m": M, "c_sw": CSW, "mu": MU, "links": "exp(i*0.2*H) seed 1001", "sources": "point",
                   "sloppy": "fp32", "reliable": "fp64", "tol": 1e-10, "recon12": args.recon12},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "converged": ok, "worst_true_rel_res": worst,
        "iters": [s["iters"] for s in stats], "reliable_updates": [s["reliable_updates"] for s in stats],
        "fp64_single_column": fp64,
        "speedup_vs_fp64_single_column": (value / fp64["solves_per_s"]) if fp64 else None,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
