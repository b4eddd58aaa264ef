"""Benchmark: Newton-step solves/s of the coupled VIV Jacobian on one MI355X.

One step = one Newton-step solve of the paper's linear problem J dU = -NL(U)
(Sec. 3.4): mf_factor with the step's values (symbolic analysis reused, as the
paper does once per pattern, Sec. 6) followed by mf_solve with FP64 refinement
to a componentwise backward error <= 1e-10.  Workload: the 2D construction at
256x128 cells (n = 540,606), seed 1, five Newton steps whose values change by
1 % relative N(0,1) noise each (cycled), one N(0,1) right-hand side per step.
All inputs are resident in HBM before the timed region.

Prints ONE JSON line (rank 0).  --gpus above 1 is refused: this build measures
one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Newton-step solves/s & front TFLOP/s, mixed vs FP64 @1e-10 bwd err; p99"
PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}      # dense MFMA TFLOP/s, MI355X
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(seconds_cap=60.0):
    """The oracle (left-looking sparse LU + FP64 refinement, single thread) on a
    bounded sample: one Newton step of the same construction at 128x64 cells,
    scaled to the 256x128 workload by the ratio of nominal front flops."""
    import numpy as np
    from oracle import splu, sym
    from vivjac import build_2d
    s = build_2d(128, 64, 1)
    S = sym.analyze(s.n, s.rowptr, s.colind, s.root)
    t0 = time.perf_counter()
    F = splu.SparseLU(s.n, s.rowptr, s.colind, s.values, S.perm, tau=0.1)
    x, om, st = F.solve(s.b0[0], tol=1e-10, max_steps=3)
    dt = time.perf_counter() - t0
    npiv = np.diff(S.front_ptr).astype(np.float64)
    m = np.diff(S.rows_ptr).astype(np.float64)
    flops_sample = float(sum(((a := np.arange(mm - pp, mm)) + 2 * a * a).sum() for mm, pp in zip(m, npiv)))
    return dt, flops_sample, float(om[0])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--ny", type=int, default=128)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--target-omega", type=float, default=1e-10)
    ap.add_argument("--panel-nb", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the separate event-timed profiling pass")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2609_31477_amd as mf
    from vivjac import build_2d, newton_rhs, newton_values

    dev = torch.device("cuda:0")
    t = time.perf_counter()
    s = build_2d(args.nx, args.ny, args.seed)
    log(f"generated n={s.n} nnz={s.nnz} in {time.perf_counter() - t:.1f}s")
    nsteps_newton = 5
    vals = [torch.from_numpy(newton_values(s, k)).to(dev) for k in range(nsteps_newton)]
    rhs = [torch.from_numpy(newton_rhs(s, k)[0].copy()).to(dev) for k in range(nsteps_newton)]
    x = torch.empty(s.n, dtype=torch.float64, device=dev)
    t = time.perf_counter()
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    t_analyze = time.perf_counter() - t
    view = S.export()
    log(f"analyze {t_analyze:.2f}s: fronts={view.nfronts} levels={view.nlevels} "
        f"nominal flops={view.nominal_flops:.3e} nnz(L+U)={view.nominal_nnz_lu:.3e}")
    opts = dict(prec=args.prec, target_omega=args.target_omega, panel_nb=args.panel_nb)
    stream = torch.cuda.current_stream()

    num = None
    step_ms = []
    omegas = []
    iters = []

    def step(i, timed):
        nonlocal num
        k = i % nsteps_newton
        t0 = time.perf_counter()
        num = S.factor(vals[k], numeric=num, stream=stream, **opts)
        _, info = num.solve(rhs[k], x=x, stream=stream)
        torch.cuda.synchronize()
        if timed:
            step_ms.append(1e3 * (time.perf_counter() - t0))
            omegas.append(info.omega)
            iters.append(info.outer_iters)

    for i in range(args.warmup):
        step(i, False)
        log(f"warmup step {i} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {elapsed:.3f}s")

    # separate pass with per-phase HIP events (not part of the timed region)
    finfo = None
    if not args.no_profile:
        num = S.factor(vals[0], numeric=num, stream=stream, profile=1, **opts)
        torch.cuda.synchronize()
        finfo = num.info()
    else:
        finfo = num.info()

    # front TFLOP/s: nominal algorithmic flops over the mean factor time of a step
    t_f0 = time.perf_counter()
    nf_rep = 3
    for i in range(nf_rep):
        num = S.factor(vals[i % nsteps_newton], numeric=num, stream=stream, **opts)
    torch.cuda.synchronize()
    t_factor = (time.perf_counter() - t_f0) / nf_rep

    dtype = {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[args.prec]
    value = args.steps / elapsed
    res = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": f"2D VIV Newton Jacobian {args.nx}x{args.ny} cells (P2-P1 flow, P2 mesh displacement, "
                        f"P2 multiplier, 2 position dofs), seed {args.seed}, {nsteps_newton} Newton steps cycled, "
                        f"1 RHS, multifrontal factor+solve, omega<=" + f"{args.target_omega:g}",
            "n": s.n, "nnz": s.nnz, "fronts": view.nfronts, "levels": view.nlevels,
            "precision": args.prec, "panel_nb": args.panel_nb,
        },
        "front_tflops": round(view.nominal_flops / t_factor / 1e12, 4),
        "factor_ms": round(1e3 * t_factor, 3),
        "p50_ms": round(float(np.percentile(step_ms, 50)), 3),
        "p99_ms": round(float(np.percentile(step_ms, 99)), 3),
        "omega_max": float(max(omegas)),
        "refine_steps_max": int(max(iters)),
        "delayed_pivots": int(finfo.delayed_pivots),
        "analyze_s": round(t_analyze, 3),
    }
    if finfo is not None and finfo.schur_launches:
        res["phases_ms"] = {"assemble": round(finfo.t_assemble_ms, 3), "panel": round(finfo.t_panel_ms, 3),
                            "schur": round(finfo.t_schur_ms, 3), "finalize": round(finfo.t_finalize_ms, 3)}
        ach = finfo.schur_flops / (finfo.t_schur_ms * 1e-3) / 1e12
        res["roofline"] = {"bound": "mfma", "kernel": "k_gemm (contribution-block Schur update)",
                           "achieved": round(ach, 4), "peak": PEAK[dtype], "unit": "TFLOP/s",
                           "frac": round(ach / PEAK[dtype], 5), "traffic": None,
                           "per_launch": f"sum over a level's fronts of 2 (m-P)^2 k flops; "
                                         f"{finfo.schur_launches} launches, {finfo.schur_flops:.3e} flops"}
    if not args.no_cpu_baseline:
        dt, fl_sample, om = cpu_baseline()
        scaled = dt * view.nominal_flops / fl_sample
        res["cpu_baseline"] = {"value": round(1.0 / scaled, 6), "unit": "solves/s", "cores": 1, "kind": "oracle",
                               "sample": f"one Newton step (factor+solve+refinement, omega {om:.1e}) of the 128x64 "
                                         f"mesh of the same construction took {dt:.2f}s single-threaded; scaled by "
                                         f"nominal front flops ({fl_sample:.3e} -> {view.nominal_flops:.3e})"}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
