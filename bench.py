"""Benchmarks of the propagator solvers on one MI355X.

Default workload (one step): the 12 spin-colour point-source columns of a
twisted-mass clover propagator on a 24^3 x 64 lattice (the MILC12 shape and
parameters of Table 1: m = -0.0695, c_sw = 1.0509, twist mu = 0.01), links
exp(i 0.2 H) from seed 1001, solved with the even-odd (symmetric Schur)
BiCGStab in FP32 storage with FP64 reliable updates to a 1e-10 FP64 relative
true residual of the full operator.  Gauge field, clover term and sources are
resident in HBM before the timed region.

Other workloads (--workload):
  hisq     multi-shift CG for 8 masses 0.002..0.05 (log-spaced) on 32^3 x 96
           (the MILC09 shape), 12 colour point sources, FP16 sloppy storage,
           per-shift refinement to 1e-10 (sec. 2.2, Table 3)
  overlap  the overlap propagator on 24^3 x 64 (the RBC11 shape, rho = 1.5,
           m = 0.015): 12 point sources solved to 1e-10 with the chirally
           projected normal equations, the order-200 Chebyshev sign function
           in FP16 storage and FP64 reliable updates (sec. 2.3, eq. 5)
  overlap_mm  the same propagator for the masses 0.03, 0.05, 0.10 to 1e-8
           (multi-shift CG in the chiral sector, then per-mass refinement)
  overlap_sign  one application of the order-200 sign function eps(H_W) to
           12 columns in FP16 storage (sec. 2.3, Fig. 2)
  overlap_lowmodes  the 16 lowest |lambda| eigenpairs of H_W at 24^3 x 64
           (Chebyshev-filtered implicitly restarted Lanczos) and the order-200
           FP16 sign function with them treated exactly
  overlap_deflated  8 chiral-sector low modes of the overlap operator per
           chirality, then the overlap workload's propagator with deflation
  serve    the serving loop: Poisson arrivals of 12-column twisted-clover and
           HISQ requests on 16^3x32, 24^3x64 and 32^3x64, p50/p99 latency
  wilson   plain Wilson CG on the normal equations, FP64, 8^4, kappa = 0.12

Printed: one JSON line with the workload's throughput, the roofline of its
dominant stencil kernel (HIP-event average duration on the kernel's stream and
its algorithmic bytes per launch), and the FP64 CPU oracle timed on a bounded
sample of the same workload.
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
TM_LAT = (24, 24, 24, 64)
M, CSW, MU = -0.0695, 1.0509, 0.01
EPS, SEED = 0.2, 1001
HISQ_LAT = (32, 32, 32, 96)
HISQ_MASSES = [0.002 * 25.0 ** (i / 7.0) for i in range(8)]
OV_LAT = (24, 24, 24, 64)
OV_RHO, OV_M, OV_N = 1.5, 0.015, 200
OV_MASSES, OV_MM_TOL = [0.03, 0.05, 0.10], 1e-8  # multi-mass overlap propagators of sec. 2.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ algorithmic bytes per output site
def wilson_site_bytes(prec: int, epi: str, n_rhs: int, recon: int = 0) -> float:
    """One Wilson-type stencil launch, per output site: the 8 links of the
    site's hops (each link of the lattice is read by exactly one output site
    per parity), the site matrix A^-1 (2 x 36 complex) for the clover
    epilogues, and each column operand once (neighbour input, own-site
    operands, output)."""
    r = {64: 8, 32: 4, 16: 2}[prec]
    links = 8 * (12 if recon and prec != 64 else 18) * r
    spin = 24 * r + (4 if prec == 16 else 0)
    clov = 144 * (8 if prec == 64 else 4) if epi in ("clovinv", "xmy", "xmyt") else 0
    # fields per column: clovinv in+out; xmy and xmyt in+x+out; xpay_g5 in+out
    # (x is the input itself); cheb in+v+b1+b2 (b2 is also the output)
    nfield = {"hop": 2, "xpay": 3, "xpay_g5": 2, "clovinv": 2, "xmy": 3, "xmyt": 3, "cheb": 4}[epi]
    return links + clov + n_rhs * nfield * spin


def stag_site_bytes(prec: int, epi: str, n_rhs: int) -> float:
    """HISQ half-stencil per output site: 8 one-hop + 8 three-hop links and each
    column operand once (hop: in + out; xpay: in + x + out)."""
    r = {64: 8, 32: 4, 16: 2}[prec]
    links = 16 * 18 * r
    spin = 6 * r + (4 if prec == 16 else 0)
    return links + n_rhs * {"hop": 2, "xpay": 3}[epi] * spin


def profile_table(L, ctx, names):
    out = {}
    for name in names:
        n, avg = L.lq_profile_get(ctx, name)
        if n:
            out[name] = {"count": n, "avg_ms": avg, "total_ms": n * avg}
            b = L.lq_profile_bytes(ctx, name)
            if b > 0:
                out[name]["alg_bytes"] = b
                out[name]["alg_gbs"] = round(b / (n * avg * 1e-3) / 1e9, 1)
    return out


BLAS_OPS = ["axpy", "axmy", "xpay", "cg", "bicg_xr", "bicg_p", "dot", "norm2", "dot_norm", "xmy_norm", "zero",
            "scale", "g5", "lc_g5", "copy", "plc"]


def family_roofline(kernels, families):
    """Roofline of the family (one kernel, all its launch widths) with the most
    time: its algorithmic bytes over its total time, i.e. the average bytes of
    a launch over the average launch duration."""
    fam = {k: kernels[k] for k in families if k in kernels and kernels[k].get("alg_bytes")}
    dom = max(fam, key=lambda k: fam[k]["total_ms"])
    f = fam[dom]
    achieved = f["alg_bytes"] / (f["total_ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
            "alg_bytes_per_launch": f["alg_bytes"] / f["count"], "avg_ms": f["avg_ms"], "launches": f["count"],
            "share_of_step": None}


# Sources that define each workload's measured kernels; its measured HBM
# traffic is reported only while they are unchanged since the counters were taken.
_CSRC = "paper_2201_09004_amd/csrc/"
_COMMON_SOURCES = ["lq_common.h", "lq_kernels.h", "blas.hip"]
KERNEL_SOURCES = {
    "tm_clover_eo_bicgstab_24x24x24x64_12rhs": _COMMON_SOURCES + ["wilson_impl.h", "wilson32.hip", "wilson.hip"],
    "overlap_sign_cheb200_24x24x24x64_12rhs": _COMMON_SOURCES + ["wilson_impl.h", "wilson16.hip", "wilson.hip"],
    "hisq_multishift_cg_32x32x32x96_12rhs_8mass": _COMMON_SOURCES + ["staggered.hip"],
}


def kernel_sources_sha(workload):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[workload]:
        with open(os.path.join(ROOT, _CSRC + f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (profiles/traffic.json), scaled by the copy-kernel
    calibration; None if absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(workload, {}).get(kernel)
    if not e or e.get("sources_sha256") != kernel_sources_sha(workload):
        return None
    return e["hbm_bytes_per_launch"]


def roofline_for(kernels, dom, alg_bytes, traffic=None):
    avg = kernels[dom]["avg_ms"]
    achieved = alg_bytes / (avg * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
            "alg_bytes_per_launch": alg_bytes, "avg_ms": avg}


def copy_peak(L, ctx):
    try:
        return round(L.lq_copy_bandwidth(ctx, 2 << 30, 10), 1)
    except Exception as e:  # noqa: BLE001
        log("copy calibration failed:", e)
        return None


# ------------------------------------------------------------------ CPU oracle samples
def cpu_info():
    """Host CPU of this run: logical CPUs visible to the process and the model name."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": n, "cpu_count": os.cpu_count(), "model": model}


def _tm_slab_worker(seed):
    """One column's share of the CPU baseline: setup + 2 Schur applications on
    the 24^3 x 8 slab, one thread; returns the elapsed seconds."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import wilson as W

    slab = (24, 24, 24, 8)
    U = synth.su3_field(slab, EPS, SEED)
    b = synth.point_sources(slab)[seed % 12]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        eo = W.EvenOdd(U, M, CSW, MU)
        y = eo.mhat(eo.mhat(b))
        t1 = time.perf_counter()
    assert np.isfinite(y).all()
    return t1 - t0


def cpu_tm_pool(n_rhs: int, one_core: dict):
    """The slab sample of cpu_tm run by min(n_rhs, nproc) worker processes at
    once (one column each): the throughput of the oracle over the machine's cores."""
    import multiprocessing as mp

    info = cpu_info()
    nw = max(1, min(n_rhs, info["nproc"] or 1))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(nw) as pool:
        per = pool.map(_tm_slab_worker, range(nw))
    wall = time.perf_counter() - t0
    # each worker did what one column's extrapolation starts from; scale as cpu_tm does
    slow = max(per) / (one_core["t_setup_s"] / (TM_LAT[3] / 8) + 2 * one_core["t_schur_s"] / (TM_LAT[3] / 8))
    return {"workers": nw, "wall_s": round(wall, 2), "worker_s_max": round(max(per), 2),
            "value": round(one_core["value"] * nw / slow, 8), "unit": "solves/s",
            "note": ("min(n_rhs, nproc) processes, one column each, at once; per-column time scaled as the "
                     "one-core sample (slow-down under load x%.2f)" % slow)}


def cpu_tm(n_iter_fp64: int, n_rhs: int):
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
    scale = TM_LAT[3] / slab[3]
    t_setup = (t1 - t0) * scale
    t_mhat = (t2 - t1) / 2 * scale
    per_col = t_setup / n_rhs + 2 * n_iter_fp64 * t_mhat
    return {"value": 1.0 / per_col, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 numpy oracle, 1 thread: EvenOdd setup + 2 Schur applications on a 24^3x8 slab "
                       f"({t2 - t0:.1f} s), scaled x{scale:.0f} to 24^3x64 and to {2 * n_iter_fp64} Schur "
                       f"applications per column (FP64 GPU BiCGStab iterations) + setup/{n_rhs}; extrapolated"),
            "t_setup_s": t_setup, "t_schur_s": t_mhat}


def cpu_hisq(n_iter: int):
    """FP64 oracle M_e(m) on a 32^3 x 8 slab, one core, two applications,
    scaled to 32^3 x 96 and to the GPU solve's operator applications."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import staggered as S

    slab = (32, 32, 32, 8)
    V, Wl = synth.hisq_fields(slab, 2001)
    b = synth.staggered_point_sources(slab, [0], colours=(0,))[0] * S.even_mask(slab)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        y = S.even_normal(V, Wl, b, 0.01)
        y = S.even_normal(V, Wl, y, 0.01)
        t1 = time.perf_counter()
    assert np.isfinite(y).all()
    scale = HISQ_LAT[3] / slab[3]
    t_app = (t1 - t0) / 2 * scale
    per_col = n_iter * t_app
    return {"value": 1.0 / per_col, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 numpy oracle, 1 thread: 2 applications of M_e on a 32^3x8 slab ({t1 - t0:.1f} s), "
                       f"scaled x{scale:.0f} to 32^3x96 and to {n_iter} applications per column (the GPU "
                       f"multi-shift + refinement iterations); extrapolated"),
            "t_apply_s": t_app}


def cpu_overlap():
    """FP64 oracle eps_N(H_W) with N = 200 on a 24^3 x 2 slab, one core, one
    column, scaled to 24^3 x 64."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import overlap as O

    slab = (24, 24, 24, 2)
    U = synth.su3_field(slab, EPS, SEED)
    v = synth.gaussian_spinor(slab, 1, 7)[0]
    c = O.cheb_coeffs(0.3, 48.0, OV_N)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        y = O.sign_hw(U, v, OV_RHO, c, 0.3, 48.0)
        t1 = time.perf_counter()
    assert np.isfinite(y).all()
    scale = OV_LAT[3] / slab[3]
    t_col = (t1 - t0) * scale
    return {"value": 1.0 / t_col, "unit": "column-applications/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 numpy oracle, 1 thread: one order-{OV_N} sign-function application (2N+1 H_W "
                       f"products) to one column on a 24^3x2 slab ({t1 - t0:.1f} s), scaled x{scale:.0f} to "
                       f"24^3x64; extrapolated")}


# ------------------------------------------------------------------ workloads
def bench_tm(args, L, torch):
    import numpy as np

    import synth

    dev = torch.device("cuda:0")
    n_rhs = 12
    log("generating synthetic gauge field", TM_LAT)
    U = synth.su3_field(TM_LAT, EPS, SEED)
    b_host = synth.point_sources(TM_LAT)
    U_d = torch.from_numpy(U).to(dev)
    b_d = torch.from_numpy(b_host).to(dev)
    x_d = torch.zeros_like(b_d)
    del U
    ctx = L.lq_init(0)
    field = L.lq_gauge_load(ctx, TM_LAT, U_d)
    del U_d
    act = L.action(L.LQ_TM_CLOVER, m=M, mu=MU, c_sw=CSW)
    prm = L.params(tol=1e-10, sloppy_bits=32, recon12=args.recon12, reliable_delta=args.delta)

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

    names = [f"wilson{p}_{e}" for p in (32, 64) for e in ("clovinv", "xmy", "xmyt", "xpay", "site")]
    kernels = profile_table(L, ctx, names + [f"{k}_n{n_rhs}" for k in names] + ["blas", "site"])
    L.lq_profile(ctx, False)
    # dominant kernel by total time; its roofline from the launches at the full
    # 12-column width (converged columns leave the batch near the end)
    dom = max((k for k in kernels if k.startswith("wilson32") and "_n" not in k),
              key=lambda k: kernels[k]["total_ms"])
    Vh = int(np.prod(TM_LAT)) // 2
    alg = wilson_site_bytes(32, dom.split("_")[1], n_rhs, args.recon12) * Vh
    kernels_w = {dom: kernels[f"{dom}_n{n_rhs}"]} if f"{dom}_n{n_rhs}" in kernels else kernels
    roof = roofline_for(kernels_w, dom, alg, measured_traffic(dom, "tm_clover_eo_bicgstab_24x24x24x64_12rhs"))
    roof["launches_at_full_width"] = kernels_w[dom]["count"]
    roof["copy_kernel_gbs"] = copy_peak(L, ctx)

    mg = None
    if not args.no_mg:
        # the same propagator by the two-level multigrid GCR (NEXT-4 row), timed beside
        # the bench line: setup once, one untimed solve, then the median of three
        log("multigrid propagator")
        torch.cuda.synchronize()
        ts = time.perf_counter()
        L.lq_mg_setup(ctx, act, field, L.mg_params(block=(4, 4, 4, 4), n_vec=30, seed=11))
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - ts
        pmg = L.params(tol=1e-10, solver=3, maxiter=300)
        x_d.zero_()
        L.lq_solve(ctx, act, field, pmg, b_d, x_d)
        runs, its, worst_mg = [], [], 0.0
        for _ in range(3):
            x_d.zero_()
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, smg = L.lq_solve(ctx, act, field, pmg, b_d, x_d)
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - ta)
            its.append(smg["iters"])
            worst_mg = max(worst_mg, smg["true_rel_res"])
        tmg = sorted(runs)[1]
        mg = {"solves_per_s": round(n_rhs / tmg, 4), "seconds_median_of_3": round(tmg, 4),
              "setup_seconds_incl_first_tuning": round(t_setup, 3), "outer_steps": its,
              "worst_true_rel_res": worst_mg, "speedup_vs_bicgstab": round((n_rhs / tmg) / value, 3),
              "config": "4^4 aggregates, 30 vectors, FP32 V-cycles, flexible GCR(8)"}
        log("multigrid", mg)

    fp64 = None
    if not args.no_fp64:
        # the plain FP64 solver on one column: one untimed solve (it also tunes
        # the one-column launch shapes), then the median of three timed solves
        log("FP64 single-column solve")
        p64 = L.params(tol=1e-10, sloppy_bits=64)
        b1 = b_d[:1].contiguous()
        x1 = torch.zeros_like(b1)
        L.lq_solve(ctx, act, field, p64, b1, x1)
        runs = []
        for _ in range(3):
            x1.zero_()
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, st64 = L.lq_solve(ctx, act, field, p64, b1, x1)
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - ta)
        t64 = sorted(runs)[1]
        fp64 = {"solves_per_s": 1.0 / t64, "seconds_median_of_3": t64, "seconds_all": runs, "iters": st64["iters"],
                "true_rel_res": st64["true_rel_res"], "warmup": 1}
        log("fp64", fp64)
        if mg:
            # the multigrid propagator is mixed precision and batched as well
            mg["speedup_vs_fp64_single_column"] = round(mg["solves_per_s"] / fp64["solves_per_s"], 3)
    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_tm(fp64["iters"] if fp64 else max(s["iters"] for s in stats), n_rhs)
        cpu["host"] = cpu_info()
        log("cpu", cpu)
        try:
            cpu["pool"] = cpu_tm_pool(n_rhs, cpu)
        except Exception as e:  # noqa: BLE001
            cpu["pool"] = {"error": repr(e)}
        log("cpu pool", cpu["pool"])
    L.lq_field_free(field)
    L.lq_finalize(ctx)
    return {
        "metric": METRIC, "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tm_clover_eo_bicgstab_24x24x24x64_12rhs", "lattice": list(TM_LAT), "n_rhs": n_rhs,
                   "m": M, "c_sw": CSW, "mu": MU, "links": "exp(i*0.2*H) seed 1001", "sources": "point",
                   "sloppy": "fp32", "reliable": "fp64", "tol": 1e-10, "recon12": args.recon12},
        "roofline": roof, "cpu_baseline": cpu,
        "converged": ok, "worst_true_rel_res": worst,
        "iters": [s["iters"] for s in stats], "reliable_updates": [s["reliable_updates"] for s in stats],
        # dslash rate: standard 1320 flops per output site and column (hopping term) of
        # the dominant stencil at 12 columns, and all stencil flops of the solve over its wall time
        "dslash_gflops": round(1320.0 * n_rhs * Vh / (roof["avg_ms"] * 1e-3) / 1e9, 1),
        "solve_stencil_gflops": round(sum(s["gflops"] for s in stats) / len(stats), 1),
        "fp64_single_column": fp64,
        "speedup_vs_fp64_single_column": (value / fp64["solves_per_s"]) if fp64 else None,
        "multigrid": mg,
        "kernels": kernels,
    }


def bench_tm_mg(args, L, torch):
    """The twisted-clover propagator of the bench line (24^3x64, 12 point
    sources, 1e-10) solved by GCR with the two-level multigrid preconditioner
    (sec. 2.1, Table 2): the setup is timed once, then the solves."""
    import synth

    dev = torch.device("cuda:0")
    n_rhs = 12
    log("generating synthetic gauge field", TM_LAT)
    U = synth.su3_field(TM_LAT, EPS, SEED)
    U_d = torch.from_numpy(U).to(dev)
    b_d = torch.from_numpy(synth.point_sources(TM_LAT)).to(dev)
    x_d = torch.zeros_like(b_d)
    del U
    ctx = L.lq_init(0)
    field = L.lq_gauge_load(ctx, TM_LAT, U_d)
    del U_d
    act = L.action(L.LQ_TM_CLOVER, m=M, mu=MU, c_sw=CSW)
    block = tuple(int(v) for v in args.mg_block.split(","))
    mp = L.mg_params(block=block, n_vec=args.mg_nvec, coarse_tol=args.mg_coarse_tol, nu_post=args.mg_nu,
                     setup_passes=args.mg_passes, gcr_kmax=args.mg_kmax, seed=11, nu_pre=args.mg_nu_pre)
    log("multigrid setup", block, args.mg_nvec)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    setup = L.lq_mg_setup(ctx, act, field, mp)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - ts
    log("setup", round(t_setup, 3), "s", setup)
    prm = L.params(tol=1e-10, solver=3, maxiter=300)
    for _ in range(args.warmup):
        x_d.zero_()
        _, st = L.lq_solve(ctx, act, field, prm, b_d, x_d)
        log("warmup stats", st)
    torch.cuda.synchronize()
    L.lq_profile(ctx, True)
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x_d.zero_()
        _, st = L.lq_solve(ctx, act, field, prm, b_d, x_d)
        stats.append(st)
        log("step", st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / args.steps * 1e3
    value = n_rhs * args.steps / (t1 - t0)
    worst = max(s["true_rel_res"] for s in stats)
    names = ([f"wilson{p}_{e}" for p in (32, 64) for e in ("site", "clovinv", "xmy", "xmyt", "xpay")] +
             ["mg_restrict", "mg_prolong", "mg_coarse32", "mg_coarse64", "mg_hop32", "mg_hop64", "mg_cgs", "site"])
    vec_names = [f"blas{p}_{o}" for p in (32, 64) for o in BLAS_OPS]
    kernels = profile_table(L, ctx, names + vec_names + ["blas"])
    L.lq_profile(ctx, False)
    roof = family_roofline(kernels, names + vec_names)
    roof["share_of_step"] = round(kernels[roof["kernel"]]["total_ms"] / (ms_step * args.steps), 4)
    L.lq_field_free(field)
    L.lq_finalize(ctx)
    return {
        "metric": METRIC, "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tm_clover_mg_gcr_24x24x24x64_12rhs", "lattice": list(TM_LAT), "n_rhs": n_rhs,
                   "m": M, "c_sw": CSW, "mu": MU, "sources": "point", "tol": 1e-10, "block": list(block),
                   "n_vec": args.mg_nvec, "coarse_tol": args.mg_coarse_tol, "nu_post": args.mg_nu,
                   "setup_passes": args.mg_passes, "gcr_kmax": args.mg_kmax, "nu_pre": args.mg_nu_pre},
        "setup_seconds": round(t_setup, 3), "setup_iters": setup["iters"],
        "roofline": roof, "cpu_baseline": None, "worst_true_rel_res": worst,
        "outer_iters": [s["iters"] for s in stats], "restarts": [s["reliable_updates"] for s in stats],
        "kernels": kernels,
    }


def bench_hisq(args, L, torch):
    import numpy as np

    import synth

    dev = torch.device("cuda:0")
    times = [0, 24, 48, 72]
    n_rhs = 3 * len(times)
    log("generating synthetic HISQ fields", HISQ_LAT)
    V, Wl = synth.hisq_fields(HISQ_LAT, 2001)
    V_d = torch.from_numpy(V).to(dev)
    del V
    W_d = torch.from_numpy(Wl).to(dev)
    del Wl
    b_d = torch.from_numpy(synth.staggered_point_sources(HISQ_LAT, times)).to(dev)
    ctx = L.lq_init(0)
    field = L.lq_hisq_load(ctx, HISQ_LAT, V_d, W_d)
    del V_d, W_d
    torch.cuda.empty_cache()
    act = L.action(L.LQ_HISQ, m=HISQ_MASSES[0])
    prm = L.params(tol=1e-10, sloppy_bits=args.hisq_sloppy, masses=HISQ_MASSES, reliable_delta=args.delta)
    x_d = torch.zeros((len(HISQ_MASSES),) + tuple(b_d.shape), dtype=b_d.dtype, device=dev)
    for _ in range(args.warmup):
        _, st = L.lq_solve(ctx, act, field, prm, b_d, x_d)
        log("warmup stats", st)
    torch.cuda.synchronize()
    L.lq_profile(ctx, True)
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = L.lq_solve(ctx, act, field, prm, b_d, x_d)
        stats.append(st)
        log("step", st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / args.steps * 1e3
    value = n_rhs * args.steps / (t1 - t0)
    worst = max(s["true_rel_res"] for s in stats)
    names = [f"stag{p}_{e}" for p in (16, 32, 64) for e in ("hop", "xpay", "xpayd")]
    vec_names = [f"blas{p}_{o}" for p in (16, 32, 64) for o in BLAS_OPS] + [f"ms{p}_{k}" for p in (16, 32)
                                                                             for k in ("xr", "p")]
    kernels = profile_table(L, ctx, names + [f"{k}_n{n_rhs}" for k in names] + vec_names + ["blas"])
    L.lq_profile(ctx, False)
    # roofline of the kernel family (all launch widths) with the most time in
    # the step: the FP16 refinement stencils, the FP32 multi-shift stencils or
    # one of the vector kernels
    roof = family_roofline(kernels, names + vec_names)
    roof["share_of_step"] = round(kernels[roof["kernel"]]["total_ms"] / (ms_step * args.steps), 4)
    roof["traffic"] = measured_traffic(roof["kernel"], "hisq_multishift_cg_32x32x32x96_12rhs_8mass")
    step_ms = ms_step * args.steps
    shares = {"stencils": round(sum(kernels[k]["total_ms"] for k in names if k in kernels) / step_ms, 3),
              "vector_kernels": round(kernels["blas"]["total_ms"] / step_ms, 3) if "blas" in kernels else None}
    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_hisq(max(s["iters"] for s in stats))
        log("cpu", cpu)
    L.lq_field_free(field)
    L.lq_finalize(ctx)
    return {
        "metric": METRIC, "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "hisq_multishift_cg_32x32x32x96_12rhs_8mass", "lattice": list(HISQ_LAT),
                   "n_rhs": n_rhs, "masses": HISQ_MASSES,
                   "sloppy": f"fp32 multi-shift, fp{args.hisq_sloppy} refinement, fp64 reliable", "tol": 1e-10},
        "roofline": roof, "cpu_baseline": cpu, "worst_true_rel_res": worst,
        "time_shares": shares,
        "mass_columns_per_s": round(value * len(HISQ_MASSES), 3),
        "iters": [s["iters"] for s in stats], "kernels": kernels,
    }


def bench_wilson(args, L, torch):
    """Plain Wilson CG on the normal equations, FP64, 8^4, kappa = 0.12 (m = 1/6),
    links exp(i 0.3 H) seed 1001, one Gaussian source: a cache-resident latency
    configuration (working set 3.9 MB)."""
    import numpy as np

    import synth

    Lw = (8, 8, 8, 8)
    m = 1.0 / (2 * 0.12) - 4.0
    dev = torch.device("cuda:0")
    U = synth.su3_field(Lw, 0.3, SEED)
    b = synth.gaussian_spinor(Lw, 1, 2001)
    ctx = L.lq_init(0)
    field = L.lq_gauge_load(ctx, Lw, torch.from_numpy(U).to(dev))
    act = L.action(L.LQ_WILSON, m=m)
    prm = L.params(tol=1e-10, sloppy_bits=64)
    b_d = torch.from_numpy(b).to(dev)
    for _ in range(args.warmup):
        L.lq_solve(ctx, act, field, prm, b_d)
    torch.cuda.synchronize()
    L.lq_profile(ctx, True)
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, st = L.lq_solve(ctx, act, field, prm, b_d)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernels = profile_table(L, ctx, ["wilson64_xpay", "blas"])
    L.lq_profile(ctx, False)
    cpu = None
    if not args.no_cpu:
        from threadpoolctl import threadpool_limits

        from oracle import solve as OS
        from oracle import wilson as W
        with threadpool_limits(1):
            ta = time.perf_counter()
            xo, it = OS.cgne(lambda v: W.wilson(U, v, m), lambda v: W.gamma5(W.wilson(U, W.gamma5(v), m)), b[0],
                             tol=1e-10)
            tb = time.perf_counter()
        cpu = {"value": 1.0 / (tb - ta), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"FP64 numpy oracle CGNE, 1 thread, the same 8^4 solve ({tb - ta:.1f} s, {it} iterations)"}
    L.lq_field_free(field)
    L.lq_finalize(ctx)
    value = args.steps / (t1 - t0)
    return {
        "metric": METRIC, "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round((t1 - t0) / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "wilson_cgne_fp64_8x8x8x8_1rhs", "lattice": list(Lw), "kappa": 0.12, "m": m,
                   "links": "exp(i*0.3*H) seed 1001", "tol": 1e-10},
        "roofline": None, "cpu_baseline": cpu, "iters": [s["iters"] for s in stats],
        "worst_true_rel_res": max(s["true_rel_res"] for s in stats), "kernels": kernels,
    }


def bench_overlap_sign(args, L, torch):
    import numpy as np

    import synth

    dev = torch.device("cuda:0")
    n_rhs = 12
    log("generating synthetic gauge field", OV_LAT)
    U = synth.su3_field(OV_LAT, EPS, SEED)
    U_d = torch.from_numpy(U).to(dev)
    del U
    v_d = torch.from_numpy(synth.point_sources(OV_LAT)).to(dev)
    ctx = L.lq_init(0)
    field = L.lq_gauge_load(ctx, OV_LAT, U_d)
    del U_d
    lo, hi = L.lq_hw_bounds(ctx, L.action(L.LQ_OVERLAP, m=OV_M, rho=OV_RHO), field, 300)
    a, b = 0.9 * lo * lo, 1.1 * hi * hi
    log("H_W spectrum", lo, hi, "interval", a, b)
    act = L.action(L.LQ_OVERLAP, m=OV_M, rho=OV_RHO, cheb_N=OV_N, cheb_a=a, cheb_b=b)
    out = torch.empty_like(v_d)
    for _ in range(args.warmup):
        L.lq_apply(ctx, act, field, L.LQ_OP_SIGN, 16, v_d, out)
    torch.cuda.synchronize()
    L.lq_profile(ctx, True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        L.lq_apply(ctx, act, field, L.LQ_OP_SIGN, 16, v_d, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / args.steps * 1e3
    value = n_rhs * args.steps / (t1 - t0)
    kernels = profile_table(L, ctx, ["wilson16_cheb", "wilson16_xpay_g5", "blas"])
    L.lq_profile(ctx, False)
    # accuracy of the FP16 application against the FP32 one on the same columns
    ref = torch.empty_like(v_d)
    L.lq_apply(ctx, act, field, L.LQ_OP_SIGN, 32, v_d, ref)
    torch.cuda.synchronize()
    finite = {"fp16": bool(torch.isfinite(torch.view_as_real(out)).all()),
              "fp32": bool(torch.isfinite(torch.view_as_real(ref)).all())}
    rel16 = float(torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(ref))
    log("finite", finite, "fp16 vs fp32", rel16)
    Vh = int(np.prod(OV_LAT)) // 2
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"] if k != "blas" else -1)
    alg = wilson_site_bytes(16, "cheb" if dom.endswith("cheb") else "xpay_g5", n_rhs) * 2 * Vh
    roof = roofline_for(kernels, dom, alg, measured_traffic(dom, "overlap_sign_cheb200_24x24x24x64_12rhs"))
    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_overlap()
        log("cpu", cpu)
    L.lq_field_free(field)
    L.lq_finalize(ctx)
    return {
        "metric": METRIC, "value": round(value, 4), "unit": "column-applications/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": "overlap_sign_cheb200_24x24x24x64_12rhs", "lattice": list(OV_LAT), "n_rhs": n_rhs,
                   "rho": OV_RHO, "N": OV_N, "interval": [a, b], "hw_spectrum": [lo, hi], "storage": "fp16"},
        "roofline": roof, "cpu_baseline": cpu, "fp16_vs_fp32_rel_l2": rel16, "finite": finite, "kernels": kernels,
    }


def cpu_overlap_solve(n_eps_per_col: int):
    """FP64 oracle H_W on a 24^3 x 2 slab, one core: an order-20 sign function
    (41 H_W products) timed and scaled per H_W product to 24^3 x 64, then to
    401 products per order-200 sign function and to the sign functions one
    column of the GPU solve used."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import overlap as O

    slab = (24, 24, 24, 2)
    U = synth.su3_field(slab, EPS, SEED)
    v = synth.gaussian_spinor(slab, 1, 7)[0]
    n = 20
    c = O.cheb_coeffs(0.3, 48.0, n)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        y = O.sign_hw(U, v, OV_RHO, c, 0.3, 48.0)
        t1 = time.perf_counter()
    assert np.isfinite(y).all()
    scale = OV_LAT[3] / slab[3]
    t_hw = (t1 - t0) / (2 * n + 1) * scale
    t_col = t_hw * (2 * OV_N + 1) * n_eps_per_col
    return {"value": 1.0 / t_col, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 numpy oracle, 1 thread: an order-{n} sign function ({2 * n + 1} H_W products) on "
                       f"one column of a 24^3x2 slab ({t1 - t0:.1f} s), scaled x{scale:.0f} to 24^3x64, to "
                       f"{2 * OV_N + 1} H_W per order-{OV_N} sign function and to {n_eps_per_col} sign functions "
                       f"per column (the GPU solve's count); extrapolated"),
            "t_hw_s": t_hw}


def _overlap_solve_leg(args, L, torch, masses, tol, workload):
    import numpy as np

    import synth

    dev = torch.device("cuda:0")
    n_rhs = 12
    log("generating synthetic gauge field", OV_LAT)
    U = synth.su3_field(OV_LAT, EPS, SEED)
    U_d = torch.from_numpy(U).to(dev)
    del U
    b_d = torch.from_numpy(synth.point_sources(OV_LAT)).to(dev)
    ctx = L.lq_init(0)
    field = L.lq_gauge_load(ctx, OV_LAT, U_d)
    del U_d
    torch.cuda.empty_cache()
    lo, hi = L.lq_hw_bounds(ctx, L.action(L.LQ_OVERLAP, m=OV_M, rho=OV_RHO), field, 300)
    log("certified H_W interval", lo, hi, "Chebyshev interval", 0.9 * lo * lo, 1.1 * hi * hi)
    act = L.action(L.LQ_OVERLAP, m=masses[0], rho=OV_RHO, cheb_N=OV_N)
    prm = L.params(tol=tol, sloppy_bits=16, masses=masses if len(masses) > 1 else None)
    nm = len(masses)
    x_d = torch.zeros(((nm,) if nm > 1 else ()) + tuple(b_d.shape), dtype=b_d.dtype, device=dev)
    for _ in range(args.warmup):
        _, st = L.lq_solve(ctx, act, field, prm, b_d, x_d)
        log("warmup stats", st)
    torch.cuda.synchronize()
    L.lq_profile(ctx, True)
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = L.lq_solve(ctx, act, field, prm, b_d, x_d)
        stats.append(st)
        log("step", st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / args.steps * 1e3
    value = n_rhs * args.steps / (t1 - t0)
    worst = max(s["true_rel_res"] for s in stats)
    ok = all(s["status"] == 0 for s in stats) and worst <= tol
    names = [f"wilson{p}_{e}" for p in (16, 32, 64) for e in ("cheb", "xpay_g5")]
    kernels = profile_table(L, ctx, names + [f"{k}_n{n_rhs}" for k in names] + ["blas"])
    L.lq_profile(ctx, False)
    Vh = int(np.prod(OV_LAT)) // 2
    # dominant kernel by total time; its roofline from its 12-column launches
    dom = max((k for k in kernels if k.startswith("wilson") and "_n" not in k), key=lambda k: kernels[k]["total_ms"])
    prec = int(dom[6:8])
    kw = {dom: kernels[f"{dom}_n{n_rhs}"]} if f"{dom}_n{n_rhs}" in kernels else kernels
    alg = wilson_site_bytes(prec, "cheb" if dom.endswith("cheb") else "xpay_g5", n_rhs) * 2 * Vh
    roof = roofline_for(kw, dom, alg, measured_traffic(dom, "overlap_sign_cheb200_24x24x24x64_12rhs"))
    roof["launches_at_full_width"] = kw[dom]["count"]
    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        s0 = stats[0]
        cpu = cpu_overlap_solve(int(np.ceil((s0["iters"] + s0["reliable_updates"]) * nm / max(nm, 1))) + 3)
        log("cpu", cpu)
    L.lq_field_free(field)
    L.lq_finalize(ctx)
    return {
        "metric": METRIC, "value": round(value, 5), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": workload, "lattice": list(OV_LAT), "n_rhs": n_rhs, "rho": OV_RHO, "masses": masses,
                   "N": OV_N, "hw_interval": [lo, hi], "sources": "point", "links": "exp(i*0.2*H) seed 1001",
                   "solver": "chirally projected CG, fp16 sign function, fp64 reliable updates", "tol": tol},
        "roofline": roof, "cpu_baseline": cpu, "converged": ok, "worst_true_rel_res": worst,
        "iters": [s["iters"] for s in stats], "reliable_updates": [s["reliable_updates"] for s in stats],
        "mass_columns_per_s": round(value * nm, 5), "kernels": kernels,
    }


def bench_overlap(args, L, torch):
    return _overlap_solve_leg(args, L, torch, [OV_M], 1e-10, "overlap_chiral_cg_24x24x24x64_12rhs_cheb200_fp16")


def bench_overlap_mm(args, L, torch):
    return _overlap_solve_leg(args, L, torch, OV_MASSES, OV_MM_TOL,
                              "overlap_multimass_chiral_cg_24x24x24x64_12rhs_3mass_cheb200_fp16")


def _overlap_setup(L, torch):
    import synth
    dev = torch.device("cuda:0")
    U = synth.su3_field(OV_LAT, EPS, SEED)
    U_d = torch.from_numpy(U).to(dev)
    del U
    ctx = L.lq_init(0)
    field = L.lq_gauge_load(ctx, OV_LAT, U_d)
    del U_d
    torch.cuda.empty_cache()
    return ctx, field


def bench_overlap_lowmodes(args, L, torch):
    """Low modes of H_W (sec. 2.3) at the overlap workload's size and their use
    in the sign function: eigensolver time and accuracy, then the FP16 order-200
    sign function on 12 point sources with 15 modes treated exactly."""
    import synth

    nev, n_rhs = 16, 12
    ctx, field = _overlap_setup(L, torch)
    act = L.action(L.LQ_OVERLAP, m=OV_M, rho=OV_RHO, cheb_N=OV_N)
    t0 = time.perf_counter()
    ev, st = L.lq_eigs(ctx, act, field, L.LQ_EIG_HW, nev, tol=1e-10)
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    log("H_W low modes", ev, st, t_eig, "s")
    v_d = torch.from_numpy(synth.point_sources(OV_LAT)).to(torch.device("cuda:0"))
    proj = L.action(L.LQ_OVERLAP, m=OV_M, rho=OV_RHO, cheb_N=OV_N, n_lowmodes=nev - 1)
    out = torch.empty_like(v_d)
    for _ in range(args.warmup):
        L.lq_apply(ctx, proj, field, L.LQ_OP_SIGN, 16, v_d, out)
    torch.cuda.synchronize()
    L.lq_profile(ctx, True)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        L.lq_apply(ctx, proj, field, L.LQ_OP_SIGN, 16, v_d, out)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    kernels = profile_table(L, ctx, ["wilson16_cheb", "wilson16_xpay_g5", "blas"])
    L.lq_profile(ctx, False)
    ref = torch.empty_like(v_d)
    L.lq_apply(ctx, proj, field, L.LQ_OP_SIGN, 64, v_d, ref)
    torch.cuda.synchronize()
    rel16 = float(torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(ref))
    L.lq_field_free(field)
    L.lq_finalize(ctx)
    ms = (t2 - t1) / args.steps * 1e3
    return {
        "metric": METRIC, "value": round(n_rhs * args.steps / (t2 - t1), 4), "unit": "column-applications/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": "overlap_lowmodes_hw16_24x24x24x64_cheb200_fp16", "lattice": list(OV_LAT),
                   "nev": nev, "n_lowmodes": nev - 1, "rho": OV_RHO, "N": OV_N},
        "roofline": None, "cpu_baseline": None,
        "eigensolver": {"seconds": round(t_eig, 2), "restarts": st["iters"], "hw_applications": st["n_apply"],
                        "max_residual": st["true_rel_res"], "eigenvalues": [float(x) for x in ev]},
        "fp16_vs_fp64_projected_rel_l2": rel16, "kernels": kernels,
    }


def bench_overlap_deflated(args, L, torch):
    """Deflated overlap propagator (sec. 2.3): 8 low modes of the chirally
    projected overlap operator per chirality (FP32 sign function, residual
    1e-6), then the overlap workload's 12-column solve with them as the
    initial guess of every sector solve."""
    import synth

    ndefl, n_rhs = 8, 12
    ctx, field = _overlap_setup(L, torch)
    act = L.action(L.LQ_OVERLAP, m=OV_M, rho=OV_RHO, cheb_N=OV_N)
    b_d = torch.from_numpy(synth.point_sources(OV_LAT)).to(torch.device("cuda:0"))
    x_d = torch.zeros_like(b_d)
    t0 = time.perf_counter()
    ev, est = L.lq_eigs(ctx, act, field, L.LQ_EIG_OVERLAP, ndefl, tol=1e-6)
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    log("sector modes", ev, est, t_eig, "s")
    prm = L.params(tol=1e-10, sloppy_bits=16, deflate=ndefl)
    stats = []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        _, st = L.lq_solve(ctx, act, field, prm, b_d, x_d)
        stats.append(st)
        log("step", st)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    L.lq_field_free(field)
    L.lq_finalize(ctx)
    worst = max(s["true_rel_res"] for s in stats)
    return {
        "metric": METRIC, "value": round(n_rhs * args.steps / (t2 - t1), 5), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 0, "ms_per_step": round((t2 - t1) / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": "overlap_deflated_chiral_cg_24x24x24x64_12rhs_cheb200_fp16", "lattice": list(OV_LAT),
                   "deflate": ndefl, "rho": OV_RHO, "m": OV_M, "N": OV_N, "tol": 1e-10},
        "roofline": None, "cpu_baseline": None, "converged": all(s["status"] == 0 for s in stats) and worst <= 1e-10,
        "worst_true_rel_res": worst, "iters": [s["iters"] for s in stats],
        "eigensolver": {"seconds": round(t_eig, 2), "restarts": est["iters"], "applications": est["n_apply"],
                        "max_residual": est["true_rel_res"], "eigenvalues": [float(x) for x in ev]},
    }


def bench_serve(args, L, torch):
    """Poisson arrivals of 12-column solves at fractions of the measured
    closed-loop capacity; latency = completion - arrival."""
    import numpy as np

    import synth

    sizes = [(16, 16, 16, 32), (24, 24, 24, 64), (32, 32, 32, 64)]
    ctx = L.lq_init(0)
    fields, sources = {}, {}
    for k, lat in enumerate(sizes):
        log("fields", lat)
        fields[(lat, "tm")] = L.lq_gauge_load(ctx, lat, synth.su3_field(lat, EPS, 1005 + k))
        V, Wl = synth.hisq_fields(lat, 2005 + k)
        fields[(lat, "hisq")] = L.lq_hisq_load(ctx, lat, V, Wl)
        del V, Wl
        sources[(lat, "tm")] = synth.point_sources(lat)
        sources[(lat, "hisq")] = synth.staggered_point_sources(lat, [0, lat[3] // 4, lat[3] // 2, 3 * lat[3] // 4])
    tm = L.action(L.LQ_TM_CLOVER, m=M, mu=MU, c_sw=CSW)
    hq = L.action(L.LQ_HISQ, m=0.01)
    p_tm = L.params(tol=1e-10, sloppy_bits=32)
    p_hq = L.params(tol=1e-10, sloppy_bits=16)
    kinds = [(lat, kind) for lat in sizes for kind in ("tm", "hisq")]
    rng = np.random.default_rng(3005)

    # Solutions are host arrays of 12 columns (4.8 GB for a 32^3x64 twisted-
    # clover request): a finished request's solution is dropped at once, and a
    # new one is submitted only while the solutions in flight stay under
    # HOST_INFLIGHT_BYTES (the closed loop keeps at most that much queued; in the
    # open loop a held-back arrival counts its wait in its latency).
    HOST_INFLIGHT_BYTES = 96e9

    def run(n_req, rate, tag):
        srv = L.lq_server_create(ctx, 0, 24)
        order = [kinds[i] for i in rng.integers(0, len(kinds), n_req)]
        reqs = []  # [ticket, stats, solution or None, key, arrival time, submit time, completion time]
        n_done = 0
        inflight = 0

        def collect(block_one):
            nonlocal n_done, inflight
            for r in reqs:
                if r[2] is None:
                    continue
                if block_one:
                    L.lq_wait(srv, r[0])
                    block_one = False
                elif not L.lq_poll(srv, r[0]):
                    continue
                r[6] = time.perf_counter()
                inflight -= r[2].nbytes
                r[2] = None
                n_done += 1
                if n_done % 16 == 0 or n_done == n_req:
                    log(f"{tag}: {n_done}/{n_req} requests done, {time.perf_counter() - t_start:.0f} s")

        t_start = time.perf_counter()
        t_arr = t_start
        for key in order:
            if rate:
                t_arr += rng.exponential(1.0 / rate)
                d = t_arr - time.perf_counter()
                if d > 0:
                    time.sleep(d)
            b = sources[key]
            while inflight > 0 and inflight + b.nbytes > HOST_INFLIGHT_BYTES:
                collect(True)
            x = np.zeros_like(b)
            st = L.lq_stats()
            act, prm = (tm, p_tm) if key[1] == "tm" else (hq, p_hq)
            t_sub = time.perf_counter()
            t = L.lq_submit(srv, act, fields[key], prm, b, x, st)
            inflight += x.nbytes
            reqs.append([t, st, x, key, t_arr if rate else t_start, t_sub, None])
            collect(False)
        while n_done < n_req:
            collect(True)
        span = time.perf_counter() - t_start
        # latency from arrival: the server's submit-to-completion time plus any
        # wait for host memory before the submission
        lat = np.array([r[1].seconds + (r[5] - r[4]) for r in reqs])
        ok = all(r[1].status == 0 for r in reqs)
        L.lq_server_destroy(srv)
        by_kind = {}
        for r, l in zip(reqs, lat):
            by_kind.setdefault(f"{'x'.join(map(str, r[3][0]))}_{r[3][1]}", []).append(l)
        return {"requests": n_req, "rate_req_per_s": rate, "span_s": span, "req_per_s": n_req / span,
                "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "all_converged": ok,
                "p50_by_kind_s": {k: round(float(np.percentile(v, 50)), 3) for k, v in sorted(by_kind.items())}}

    log("warm engines")
    run(len(kinds), 0, "warm")
    if args.serve_capacity > 0:
        closed = {"req_per_s": args.serve_capacity, "given": True}
    else:
        log("closed loop")
        closed = run(args.serve_requests, 0, "closed")
    mu_max = closed["req_per_s"]
    log("capacity", mu_max, "req/s")
    open_loop = []
    for f in [float(v) for v in args.serve_rates.split(",") if v]:
        log("rate", f)
        r = run(args.serve_requests, f * mu_max, f"rate {f}")
        r["fraction"] = f
        open_loop.append(r)
        log(r)
    for f in fields.values():
        L.lq_field_free(f)
    L.lq_finalize(ctx)
    worst = open_loop[-1] if open_loop else closed
    return {
        "metric": METRIC, "value": round(closed["req_per_s"] * 12, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.serve_requests, "warmup": len(kinds), "ms_per_step": round(1e3 / closed["req_per_s"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serve_mixed_tm_hisq_16x32_24x64_32x64_12rhs", "sizes": [list(s) for s in sizes],
                   "actions": ["tm_clover fp32", "hisq m=0.01 fp16"], "max_cols": 24},
        "roofline": None, "cpu_baseline": None,
        "closed_loop": closed, "poisson": open_loop, "p50_s": worst.get("p50_s"), "p99_s": worst.get("p99_s"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("tm", "tm_mg", "hisq", "overlap", "overlap_mm", "overlap_sign", "overlap_lowmodes",
                                           "overlap_deflated", "serve", "wilson"), default="tm")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 single-column comparison")
    ap.add_argument("--no-mg", action="store_true", help="skip the multigrid propagator beside the bench line (tm)")
    ap.add_argument("--hisq-sloppy", type=int, default=16, choices=(16, 32), help="refinement storage (hisq)")
    ap.add_argument("--recon12", type=int, default=0)
    ap.add_argument("--delta", type=float, default=0.0, help="reliable-update threshold (tm, hisq; 0: the library default 0.1)")
    ap.add_argument("--serve-requests", type=int, default=256, help="requests per arrival rate (serve)")
    ap.add_argument("--serve-rates", default="0.5,0.8,0.95", help="arrival rates as fractions of capacity (serve)")
    ap.add_argument("--serve-capacity", type=float, default=0.0,
                    help="closed-loop capacity in requests/s from an earlier run (serve; 0: measure it)")
    ap.add_argument("--mg-block", default="4,4,4,4", help="multigrid aggregate extents x,y,z,t (tm_mg)")
    ap.add_argument("--mg-nvec", type=int, default=30, help="multigrid near-null vectors (tm_mg)")
    ap.add_argument("--mg-coarse-tol", type=float, default=0.1, help="coarse solve tolerance (tm_mg)")
    ap.add_argument("--mg-nu", type=int, default=4, help="post-smoothing steps (tm_mg)")
    ap.add_argument("--mg-passes", type=int, default=2, help="setup inverse-iteration passes (tm_mg)")
    ap.add_argument("--mg-nu-pre", type=int, default=0, help="pre-smoothing steps of the V-cycle (tm_mg)")
    ap.add_argument("--mg-kmax", type=int, default=8, help="outer GCR restart length (tm_mg)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2201_09004_amd import lq as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    fn = {"tm": bench_tm, "tm_mg": bench_tm_mg, "hisq": bench_hisq, "overlap": bench_overlap, "overlap_mm": bench_overlap_mm,
          "overlap_sign": bench_overlap_sign, "overlap_lowmodes": bench_overlap_lowmodes,
          "overlap_deflated": bench_overlap_deflated, "serve": bench_serve, "wilson": bench_wilson}[args.workload]
    out = fn(args, L, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
