"""Benchmark: Newton-step solves/s of the coupled VIV Jacobian on one MI355X.

One step = one Newton-step solve of the paper's linear problem J dU = -NL(U)
(Sec. 3.4): mf_factor with the step's values (symbolic analysis reused, as the
paper does once per pattern, Sec. 6) followed by mf_solve with FP64 refinement
to a componentwise backward error <= 1e-10.  Workload: the 2D construction at
256x128 cells (n = 540,606), seed 1, five Newton steps whose values change by
1 % relative N(0,1) noise each (cycled), one N(0,1) right-hand side per step.
All inputs are resident in HBM before the timed region.

Beside the headline it reports, on the same line: the mixed path on the same
workload (FP32 fronts, FP64 root, adaptive FP64 refinement: classical steps
while each cuts omega tenfold, then GMRES-IR); the same matrix with eight
right-hand sides in FP64, FP32 and BF16 (the precision comparison); the
dominant kernel against its roofline and the Schur GEMM, solve sweeps and
extend-add against theirs; a large-K Schur GEMM on one dense front in each
precision; the 64-system batch; a short serving stream (40 requests at 16/s);
and the CPU oracle on a bounded sample.

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
PANEL_TRAFFIC = {(256, 128, "fp64"): 10685912}  # bytes per panel launch, profiles/panel_traffic_256x128.txt
PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}      # dense MFMA TFLOP/s, MI355X
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_step(nx, ny, seed=1):
    """One Newton step of the oracle (nested-dissection order, left-looking sparse
    LU with threshold tau = 0.1, FP64 refinement to 1e-10), single-threaded C.
    Returns (seconds, nominal front flops of the same order, omega)."""
    import numpy as np
    from oracle import splu, sym
    from vivjac import build_2d
    s = build_2d(nx, ny, seed)
    S = sym.analyze(s.n, s.rowptr, s.colind, s.root)
    npiv = np.diff(S.front_ptr).astype(np.float64)
    m = np.diff(S.rows_ptr).astype(np.float64)
    flops = float(sum(((a := np.arange(mm - pp, mm)) + 2 * a * a).sum() for mm, pp in zip(m, npiv)))
    t0 = time.perf_counter()
    F = splu.SparseLU(s.n, s.rowptr, s.colind, s.values, S.perm, tau=0.1)
    x, om, st = F.solve(s.b0[0], tol=1e-10, max_steps=3)
    return time.perf_counter() - t0, flops, float(om[0])


def cpu_baseline(target_flops, full=True, nx=256, ny=128):
    """The oracle on this host's cores, single-threaded.  Default (full): one Newton
    step of the workload itself (step 0 at nx x ny: analysis untimed, then the
    factorization, solve and refinement), about 20-30 s.  full=False: a bounded
    sample instead, one step at 64x32 and at 128x64 cells of the same construction,
    with the full-size time extrapolated by the power law in nominal front flops
    fitted through the two (on the GPU host it came out 19% below the measured
    full-size step)."""
    import math
    if full:
        dt, fl, om = _oracle_step(nx, ny)
        return {"value": round(1.0 / dt, 6), "unit": "solves/s", "cores": 1, "kind": "oracle",
                "sample": f"one full Newton step of the {nx}x{ny} workload (factor+solve+refinement, omega {om:.1e}) "
                          f"took {dt:.1f}s single-threaded",
                "cpu": _cpu_model(), "nproc": os.cpu_count()}
    t1, f1, _ = _oracle_step(64, 32)
    t2, f2, om = _oracle_step(128, 64)
    alpha = math.log(t2 / t1) / math.log(f2 / f1)
    est = t2 * (target_flops / f2) ** alpha
    return {"value": round(1.0 / est, 6), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"one Newton step at 64x32 ({t1:.2f}s) and 128x64 ({t2:.2f}s, omega {om:.1e}) of the same "
                      f"construction, single-threaded; time taken as a power of nominal front flops fitted through "
                      f"the two (exponent {alpha:.2f}) and evaluated at the workload's {target_flops:.3e} flops: "
                      f"{est:.1f}s per step",
            "cpu": _cpu_model(), "nproc": os.cpu_count()}


def gemm_micro(prec, N=4096, nroot=2048):
    """Large-K Schur GEMM: one dense front of order N whose last nroot variables are
    the root list, so the front eliminates N - nroot pivots and updates an nroot x
    nroot contribution block with K = N - nroot (k_gemm / k_gemm_bf16 through a
    profiled factorization).  Returns achieved TFLOP/s of the Schur phase."""
    import numpy as np
    import scipy.sparse as sp
    import torch

    import paper_2609_31477_amd as mf
    rng = np.random.default_rng(5)
    A = rng.standard_normal((N, N)) + np.sqrt(N) * np.eye(N)
    M = sp.csr_matrix(A)
    M.sort_indices()
    S = mf.Symbolic(N, M.indptr, M.indices, np.arange(N - nroot, N, dtype=np.int32), leaf_max=N)
    v = torch.from_numpy(M.data.copy()).cuda()
    num = S.factor(v, prec=prec, profile=1)
    num = S.factor(v, numeric=num, prec=prec, profile=1)
    torch.cuda.synchronize()
    fi = num.info()
    num.release()
    return fi.schur_flops / (fi.t_schur_ms * 1e-3) / 1e12, fi.schur_flops


def bench_ale(nx=256, ny=128, seed=1):
    """The full ALE Newton iteration on the GPU (row f1): assembly of NL(U) and of
    J(U) with its shape-derivative blocks, FP64 factorization and solve, to
    max |NL| <= 1e-10 from the previous time level."""
    import torch

    import paper_2609_31477_amd as mf
    from paper_2609_31477_amd.ale import Assembly, newton
    from vivjac.ale2d import build_ale_2d
    prob = build_ale_2d(nx, ny, seed)
    A = Assembly(prob)
    S = mf.Symbolic(prob.n, prob.rowptr, prob.colind, prob.root)
    U = torch.from_numpy(prob.initial_guess()).cuda()
    R = torch.empty_like(U)
    vals = A.jacobian(U, R=R)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(5):
        A.jacobian(U, values=vals, R=R, stream=st)
    e1.record(st)
    torch.cuda.synchronize()
    t_jac = e0.elapsed_time(e1) / 5
    e0.record(st)
    for _ in range(5):
        A.residual(U, R=R, stream=st)
    e1.record(st)
    torch.cuda.synchronize()
    t_res = e0.elapsed_time(e1) / 5
    out = None
    for _ in range(2):                                   # the second run is timed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, norms, infos = newton(prob, iters=8, tol=1e-10, prec="fp64", target_omega=1e-12, assembly=A, symbolic=S)
        torch.cuda.synchronize()
        out = (time.perf_counter() - t0, norms, infos)
    dt, norms, infos = out
    A.release()
    return {"workload": f"2D ALE Newton iteration {nx}x{ny} cells (P2-P1 flow on the current mesh, P1 position, "
                        "P2 multiplier, 2 position dofs; BDF1, nu 0.01, dt 0.01), from the previous level to "
                        "max|NL| <= 1e-10, FP64 factors",
            "n": prob.n, "nnz": prob.nnz, "newton_iterations": len(infos), "seconds": round(dt, 4),
            "ms_per_iteration": round(1e3 * dt / max(1, len(infos)), 3),
            "residual_history": [float("%.3e" % v) for v in norms],
            "assembly_ms": round(t_jac, 4), "residual_ms": round(t_res, 4)}


def bench_mixed_3d(steps=4, warmup=1):
    """FP64 against FP32 and BF16 fronts (FP64 root, adaptive FP64 refinement to 1e-10) on the
    3D box of the serving mix (24x12x6 hexahedra, n = 84,825): Newton steps with
    the 1% value stream, one right-hand side each."""
    import numpy as np
    import torch

    import paper_2609_31477_amd as mf
    from vivjac import build_3d, newton_rhs, newton_values
    s = build_3d(24, 12, 6, seed=3)
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    dev = torch.device("cuda:0")
    vals = [torch.from_numpy(newton_values(s, k)).to(dev) for k in range(3)]
    rhs = [torch.from_numpy(newton_rhs(s, k)[0].copy()).to(dev) for k in range(3)]
    x = torch.empty_like(rhs[0])
    out = {"workload": "3D box 24x12x6 hexahedra (n 84,825), Newton steps with 1% value changes, 1 RHS, "
                       "omega <= 1e-10; mixed: FP64 root and adaptive FP64 refinement (classical, then GMRES-IR)"}
    for prec in ("fp64", "fp32", "bf16"):
        num, ts, tf, inner, om = None, [], [], [], []
        for it in range(warmup + steps):
            k = it % 3
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            num = S.factor(vals[k], numeric=num, prec=prec, target_omega=1e-10, max_outer=30)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, info = num.solve(rhs[k], x=x)
            torch.cuda.synchronize()
            if it >= warmup:
                ts.append(time.perf_counter() - t0)
                tf.append(t1 - t0)
                inner.append(info.inner_iters)
                om.append(info.omega)
        num.release()
        out[prec] = {"ms_per_step": round(1e3 * float(np.mean(ts)), 3), "factor_ms": round(1e3 * float(np.mean(tf)), 3),
                     "inner_per_step": round(float(np.mean(inner)), 2), "omega_max": float(max(om))}
    for prec in ("fp32", "bf16"):
        out[prec]["speedup_vs_fp64"] = round(out["fp64"]["ms_per_step"] / out[prec]["ms_per_step"], 4)
    return out


def bench_batch(args, summary_only=False):
    """64 independent 2D systems (seeds 100-163, nx = 16 + 4 U{0..12}, ny = nx/2) factored
    and solved together, FP32 fronts (FP64 roots) with adaptive FP64 refinement to omega <= 1e-10."""
    import numpy as np
    import torch

    import paper_2609_31477_amd as mf
    from vivjac import build_2d
    dev = torch.device("cuda:0")
    systems = []
    for i in range(64):
        rng = np.random.default_rng(100 + i)
        nx = 16 + 4 * int(rng.integers(0, 13))
        systems.append(build_2d(nx, nx // 2, 100 + i))
    syms = [mf.Symbolic(s.n, s.rowptr, s.colind, s.root) for s in systems]
    B = mf.Batch(syms)
    view = B.export()
    vals = [torch.from_numpy(s.values).to(dev) for s in systems]
    bs = [torch.from_numpy(s.b0[0].copy()).to(dev) for s in systems]
    xs = [torch.empty_like(b) for b in bs]
    prec = "fp32" if args.prec == "fp64" else args.prec
    stream = torch.cuda.current_stream()
    def step():
        # the planned schedule replayed as a captured HIP graph (one synchronization
        # per factorization; bitwise equal to level by level)
        B.factor(vals, stream=stream, prec=prec, target_omega=args.target_omega, plan=2)
        _, infos = B.solve(bs, xs=xs, stream=stream)
        torch.cuda.synchronize()
        return infos
    for _ in range(args.warmup):
        step()
    ts = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t1 = time.perf_counter()
        infos = step()
        ts.append(time.perf_counter() - t1)
    el = time.perf_counter() - t0
    if summary_only:
        B.release()
        return {"workload": "64 uneven 2D systems (16x8..64x32 cells), one batched factor+solve per step, FP32 fronts, "
                            "FP64 roots, adaptive FP64 refinement to omega<=1e-10, factorization replayed as a captured HIP graph",
                "value": round(64 * args.steps / el, 3), "unit": "solves/s",
                "ms_per_step": round(1e3 * el / args.steps, 3), "p99_ms": round(1e3 * float(np.percentile(ts, 99)), 3),
                "omega_max": float(max(i.omega for i in infos)), "steps": args.steps}
    res = {"metric": METRIC, "value": round(64 * args.steps / el, 3), "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * el / args.steps, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "64 uneven 2D VIV Jacobians (16x8..64x32 cells, seeds 100-163), one batched "
                                  "factor+solve per step, FP32 fronts, FP64 roots, adaptive FP64 refinement, omega<=1e-10",
                      "n_total": int(sum(s.n for s in systems)), "fronts": view.nfronts, "levels": view.nlevels},
           "front_tflops": round(view.nominal_flops * args.steps / el / 1e12, 4),
           "p99_ms": round(1e3 * float(np.percentile(ts, 99)), 3),
           "omega_max": float(max(i.omega for i in infos)), "outer_max": int(max(i.outer_iters for i in infos))}
    print(json.dumps(res), flush=True)


class DevicePayloads:
    """What a serving request brings, formed on the device from its mesh's value
    parts (two host assemblies per mesh, done before the clock starts): step-0
    values base + nu * visc + k * spring for the request's own nu and k, then the
    Newton stream's 1% relative N(0,1) perturbation per step and one N(0,1)
    right-hand side per step, drawn from a device generator seeded with the
    request's seed (input synthesis: no solver arithmetic)."""

    def __init__(self, parts):
        import threading
        self.parts = parts            # mesh -> (system, base, visc, spring) on the host
        self.dev_parts = {}
        self.lock = threading.Lock()

    def __call__(self, req, dev):
        import torch
        s, base, visc, spring = self.parts[req.mesh]
        with self.lock:
            dp = self.dev_parts.get(req.mesh)
            if dp is None:
                # uploaded and waited for before any other thread's stream can read it
                dp = tuple(torch.from_numpy(a).to(dev) for a in (base, visc, spring))
                torch.cuda.current_stream(dev).synchronize()
                self.dev_parts[req.mesh] = dp
        g = torch.Generator(device=dev)
        g.manual_seed(int(req.seed))
        v = dp[0] + req.nu * dp[1] + req.k * dp[2]
        vals, rhs = [], []
        for t in range(req.newton_steps):
            if t:
                v = v * (1.0 + 0.01 * torch.randn(s.nnz, generator=g, dtype=torch.float64, device=dev))
            vals.append(v)
            rhs.append(torch.randn(s.n, generator=g, dtype=torch.float64, device=dev))
        return s, vals, rhs


def serving_parts(meshes, seed=11):
    """Value parts of every mesh, assembled in parallel host processes."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp

    from vivjac import value_parts
    meshes = sorted(set(meshes))
    # 3D assemblies first: they are the long ones
    meshes.sort(key=lambda m: m[0] != "3d")
    workers = max(1, min(12, len(meshes), os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return dict(zip(meshes, ex.map(value_parts, meshes, [seed] * len(meshes))))


def bench_serving(args, summary_only=False):
    """Poisson streams of mixed requests (70% 2D meshes 32x16..128x64 cells, 30% 3D
    boxes of 24x12x6 hexahedra; Re ~ U[100,300]; U_r ~ U[2,12] in 2D, U[2.5,17.5] in
    3D), 5 Newton steps each, FP32 fronts + adaptive FP64 refinement to 1e-10, continuous
    batching; one run per arrival rate.  summary_only: return the per-rate lines
    (no JSON line of its own)."""
    import torch

    from paper_2609_31477_amd.serving import MFBackend, Scheduler, poisson_requests, summarize
    rates = [float(r) for r in str(args.rates).split(",")] if args.rates else [args.rate]
    streams = {rate: poisson_requests(args.requests, rate=rate, seed=args.seed + i, mix_3d=args.mix_3d)
               for i, rate in enumerate(rates)}
    warm = poisson_requests(12, rate=1e3, seed=99, mix_3d=0.5)
    t = time.perf_counter()
    parts = serving_parts([r.mesh for rs in list(streams.values()) + [warm] for r in rs])
    log(f"assembled value parts of {len(parts)} meshes in {time.perf_counter() - t:.1f}s: "
        + ", ".join(f"{m[0]} {'x'.join(map(str, m[1:]))} n={p[0].n}" for m, p in parts.items() if m[0] == "3d"))
    payloads = DevicePayloads(parts)

    def serve(reqs):
        be = MFBackend(prec="fp32", target_omega=args.target_omega, payloads=payloads)
        sch = Scheduler(be, hbm_budget=200 << 30, max_slots=64, max_cohorts=args.max_cohorts or None)
        for r in reqs:
            sch.submit(r)
        t0 = time.perf_counter()
        last = [t0]

        def progress(sc):
            if time.perf_counter() - last[0] > 20.0:
                last[0] = time.perf_counter()
                log(f"  t={last[0] - t0:.0f}s: {len(sc.done)} done, {len(sc.active)} active, "
                    f"{len(sc.waiting)} not admitted, {sc.ticks} ticks")

        done = sch.run(on_tick=progress)
        wall = time.perf_counter() - t0
        be.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()       # the next run starts from the same free memory
        worst = max(max(x["omega"] for x in r.results) for r in done)
        return summarize(done), sch, be, wall, worst

    serve(warm)                       # module load, first-touch allocations
    log("warm-up stream served")
    lines = []
    for rate, reqs in streams.items():
        s, sch, be, wall, worst = serve(reqs)
        n3 = sum(r.mesh[0] == "3d" for r in reqs)
        line = {"rate": rate, "requests": s["requests"], "requests_3d": n3, "solves": s["solves"],
                "solves_per_s": round(s["solves_per_s"], 3),
                "p50_request_ms": round(1e3 * s["p50_request_s"], 2), "p99_request_ms": round(1e3 * s["p99_request_s"], 2),
                "p50_step_ms": round(1e3 * s["p50_step_s"], 2), "p99_step_ms": round(1e3 * s["p99_step_s"], 2),
                "mean_batch": round(sum(sch.batch_sizes) / len(sch.batch_sizes), 2), "ticks": sch.ticks,
                "cohorts": sch.cohorts, "wall_s": round(wall, 2), "omega_max": worst,
                "host_phase_s": {k: round(v, 3) for k, v in be.times.items()}}
        log(json.dumps(line))
        lines.append(line)
    if summary_only:
        return {"workload": f"serving: {args.requests} Poisson requests per rate, {100 * (1 - args.mix_3d):.0f}% 2D "
                            f"meshes 32x16..128x64 cells, {100 * args.mix_3d:.0f}% 3D boxes 24x12x6, 5 Newton steps "
                            "each, FP32 fronts + adaptive FP64 refinement, continuous batching, at most "
                            f"{args.max_cohorts} cohorts at once, omega<={args.target_omega:g} (the full rate sweep: "
                            "--workload serving)",
                "per_rate": [{k: l[k] for k in ("rate", "requests", "requests_3d", "solves", "solves_per_s",
                                                 "p50_request_ms", "p99_request_ms", "p50_step_ms", "p99_step_ms",
                                                 "mean_batch", "omega_max")} for l in lines]}
    top = max(lines, key=lambda l: l["solves_per_s"])
    res = {"metric": METRIC, "value": top["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
           "steps": top["solves"], "warmup": len(warm), "ms_per_step": round(1e3 / top["solves_per_s"], 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"serving: {args.requests} Poisson requests per rate, {100 * (1 - args.mix_3d):.0f}% "
                                  f"2D meshes 32x16..128x64 cells, {100 * args.mix_3d:.0f}% 3D boxes 24x12x6, "
                                  "5 Newton steps each, FP32 fronts + adaptive FP64 refinement, continuous batching, "
                                  f"at most {args.max_cohorts or 'any number of'} cohorts at once, "
                                  f"omega<={args.target_omega:g}", "rates": rates},
           "p50_request_ms": top["p50_request_ms"], "p99_request_ms": top["p99_request_ms"],
           "p50_step_ms": top["p50_step_ms"], "p99_step_ms": top["p99_step_ms"], "per_rate": lines}
    print(json.dumps(res), flush=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--nrhs", type=int, default=1, choices=[1, 8],
                    help="right-hand sides per Newton step of the timed leg (8: the precision comparison's shape)")
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--ny", type=int, default=128)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--target-omega", type=float, default=1e-10)
    ap.add_argument("--workload", default="newton", choices=["newton", "batch", "serving", "ale"],
                    help="newton: 256x128 Newton steps (default); batch: 64 uneven systems in one batched "
                         "factor+solve; serving: Poisson request stream through the continuous-batching loop; "
                         "ale: the full ALE Newton iteration (GPU assembly with shape derivatives) at 256x128")
    ap.add_argument("--rate", type=float, default=20.0, help="serving: arrival rate (requests/s)")
    ap.add_argument("--rates", default="", help="serving: comma-separated arrival rates, one run each")
    ap.add_argument("--requests", type=int, default=60, help="serving: number of requests per rate")
    ap.add_argument("--mix-3d", type=float, default=0.3, help="serving: fraction of 3D requests")
    ap.add_argument("--max-cohorts", type=int, default=2,
                    help="serving: cohorts active at once (0: no cap); arrivals beyond it gather into the next")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 5 times (HBM counter calibration) and exit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-fit", action="store_true",
                    help="estimate the oracle's time from one step at 64x32 and 128x64 cells (power law in nominal "
                         "front flops) instead of timing the full-size step (about 20-30 s on one core)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the eight-right-hand-side precision comparison, GEMM microbenchmark and batch line")
    ap.add_argument("--no-profile", action="store_true", help="skip the separate event-timed profiling pass")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision (FP32 fronts) comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2609_31477_amd as mf
    from vivjac import build_2d, newton_rhs, newton_values

    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy << 17, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": src.numel() * 8}))
        return
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "ale":
        r = bench_ale(args.nx, args.ny, args.seed)
        res = {"metric": METRIC, "value": round(r["newton_iterations"] / r["seconds"], 4), "unit": "Newton iterations/s",
               "n_gpus": 1, "steps": r["newton_iterations"], "warmup": 1, "ms_per_step": r["ms_per_iteration"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": r.pop("workload"), "n": r["n"], "nnz": r["nnz"]}, "ale": r}
        print(json.dumps(res), flush=True)
        return res
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    s = build_2d(args.nx, args.ny, args.seed)
    log(f"generated n={s.n} nnz={s.nnz} in {time.perf_counter() - t:.1f}s")
    nsteps_newton = 5
    vals = [torch.from_numpy(newton_values(s, k)).to(dev) for k in range(nsteps_newton)]
    rhs = [torch.from_numpy(newton_rhs(s, k)[0].copy()).to(dev) for k in range(nsteps_newton)]
    x = torch.empty(s.n, dtype=torch.float64, device=dev)
    x.zero_()
    # the precision comparison: the same matrices with eight right-hand sides
    # (the first eight rows of each step's seeded stream)
    rhs8 = [] if args.no_extras and args.nrhs == 1 else [torch.from_numpy(newton_rhs(s, k, nrhs=8).copy()).to(dev)
                                                         for k in range(nsteps_newton)]
    x8 = torch.empty(8, s.n, dtype=torch.float64, device=dev) if rhs8 else None
    t = time.perf_counter()
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    t_analyze = time.perf_counter() - t
    view = S.export()
    log(f"analyze {t_analyze:.2f}s: fronts={view.nfronts} levels={view.nlevels} "
        f"nominal flops={view.nominal_flops:.3e} nnz(L+U)={view.nominal_nnz_lu:.3e}")
    stream = torch.cuda.current_stream()

    def run_path(prec, nrhs=1, steps=None, warmup=None, profile=True):
        """Time Newton-step solves (factor + solve + refinement) in one precision."""
        steps = args.steps if steps is None else steps
        warmup = args.warmup if warmup is None else warmup
        opts = dict(prec=prec, target_omega=args.target_omega)
        state = {"num": None}
        step_ms, omegas, iters, inner = [], [], [], []
        rr = rhs if nrhs == 1 else rhs8
        xx = x if nrhs == 1 else x8

        def step(i, timed):
            k = i % nsteps_newton
            t0 = time.perf_counter()
            state["num"] = S.factor(vals[k], numeric=state["num"], stream=stream, **opts)
            _, info = state["num"].solve(rr[k], x=xx, stream=stream)
            torch.cuda.synchronize()
            if timed:
                step_ms.append(1e3 * (time.perf_counter() - t0))
                omegas.append(info.omega)
                iters.append(info.outer_iters)
                inner.append(info.inner_iters)

        for i in range(warmup):
            step(i, False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(i, True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        log(f"{prec} ({nrhs} rhs): timed {steps} steps in {elapsed:.3f}s")
        num = state["num"]
        finfo = None
        if profile and not args.no_profile:
            num = S.factor(vals[0], numeric=num, stream=stream, profile=1, **opts)
            torch.cuda.synchronize()
            finfo = num.info()
        t_f0 = time.perf_counter()
        nf_rep = 3
        for i in range(nf_rep):
            num = S.factor(vals[i % nsteps_newton], numeric=num, stream=stream, **opts)
        torch.cuda.synchronize()
        t_factor = (time.perf_counter() - t_f0) / nf_rep
        if finfo is None:
            finfo = num.info()
        # one sweep pair alone (no refinement), timed with events on the stream
        t_sweep = None
        if profile and not args.no_profile:
            num = S.factor(vals[0], numeric=num, stream=stream, prec=prec, refine=0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            num.solve(rr[0], x=xx, stream=stream)
            e0.record(stream)
            for _ in range(3):
                num.solve(rr[0], x=xx, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            t_sweep = e0.elapsed_time(e1) / 3
        num.release()
        return dict(elapsed=elapsed, step_ms=step_ms, omegas=omegas, iters=iters, inner=inner, finfo=finfo,
                    t_factor=t_factor, t_sweep=t_sweep, steps=steps)

    def run_reuse(prec, seq=None, repeats=2):
        """The Newton sequence with one reduced-precision factorization kept as the
        GMRES-IR preconditioner across steps (refreshed by the reuse policy)."""
        from paper_2609_31477_amd.newton import ReusedFactorNewton
        seq = vals if seq is None else seq
        out = None
        for rep in range(repeats):
            solver = ReusedFactorNewton(S, prec=prec, target_omega=args.target_omega, stream=stream)
            ms = []
            for k in range(nsteps_newton):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info, rec = solver.step(seq[k], rhs[k], x=x)
                torch.cuda.synchronize()
                ms.append(1e3 * (time.perf_counter() - t0))
            out = dict(step_ms=ms, history=solver.history)
            solver.release()
        return out

    main = run_path(args.prec, nrhs=args.nrhs)
    mixed = None if args.no_mixed or args.prec != "fp64" else run_path("fp32", nrhs=args.nrhs)
    eight = {}
    if rhs8 and args.prec == "fp64" and not args.no_mixed and not args.no_extras and args.nrhs == 1:
        for pr in ("fp64", "fp32", "bf16"):
            # the FP64 leg also times one 8-column sweep pair alone
            eight[pr] = run_path(pr, nrhs=8, steps=3, warmup=1, profile=(pr == "fp64"))
    elapsed, step_ms, omegas, iters, finfo, t_factor = (main["elapsed"], main["step_ms"], main["omegas"],
                                                         main["iters"], main["finfo"], main["t_factor"])

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
                        f"{args.nrhs} RHS, multifrontal factor+solve, omega<=" + f"{args.target_omega:g}",
            "n": s.n, "nnz": s.nnz, "fronts": view.nfronts, "levels": view.nlevels,
            "precision": args.prec,
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
    if mixed is not None:
        mv = args.steps / mixed["elapsed"]
        res["mixed"] = {"precision": "fp32 fronts, fp64 root + adaptive refinement (classical, then GMRES-IR)", "value": round(mv, 4), "unit": "solves/s",
                        "ms_per_step": round(1e3 * mixed["elapsed"] / args.steps, 3),
                        "p99_ms": round(float(np.percentile(mixed["step_ms"], 99)), 3),
                        "factor_ms": round(1e3 * mixed["t_factor"], 3),
                        "front_tflops": round(view.nominal_flops / mixed["t_factor"] / 1e12, 4),
                        "omega_max": float(max(mixed["omegas"])), "outer_max": int(max(mixed["iters"])),
                        "inner_total": int(sum(mixed["inner"])),
                        "speedup_vs_fp64": round(mv / value, 4)}
    if eight:
        base = eight["fp64"]["steps"] / eight["fp64"]["elapsed"]
        res["eight_rhs"] = {"workload": "the same 256x128 Newton steps with 8 right-hand sides N(0,1) per step; "
                                        "mixed paths: FP64 root, FP64 residual, adaptive refinement over the 8 in lockstep",
                            "unit": "solves/s (one solve = factor + 8-column solve)"}
        for pr, r in eight.items():
            v = r["steps"] / r["elapsed"]
            res["eight_rhs"][pr] = {"value": round(v, 4), "ms_per_step": round(1e3 * r["elapsed"] / r["steps"], 3),
                                    "omega_max": float(max(r["omegas"])), "outer_max": int(max(r["iters"])),
                                    "inner_per_step": round(sum(r["inner"]) / len(r["inner"]), 1),
                                    "speedup_vs_fp64": round(v / base, 4)}
            if r["t_sweep"]:
                # every factor entry is read once for all eight columns
                b8 = view.nominal_nnz_lu * 8.0
                res["eight_rhs"][pr]["sweep_pair"] = {
                    "bound": "hbm", "ms": round(r["t_sweep"], 4), "bytes": b8,
                    "achieved": round(b8 / (r["t_sweep"] * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(b8 / (r["t_sweep"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                    "kernel": "forward + backward sweep pair over 8 columns plus one residual"}
    if finfo is not None and finfo.schur_launches:
        res["phases_ms"] = {"assemble": round(finfo.t_assemble_ms, 3), "panel_loop": round(finfo.t_panel_ms, 3),
                            "panel_kernel": round(finfo.t_panel_kernel_ms, 3), "schur": round(finfo.t_schur_ms, 3),
                            "finalize": round(finfo.t_finalize_ms, 3)}
        # dominant kernel: the threshold-pivoting panel (per launch: every front of a tree
        # level factors one window); FP64 arithmetic on the vector ALUs
        avg_ms = finfo.t_panel_kernel_ms / max(1, finfo.panel_launches)
        ach = finfo.panel_flops / (finfo.t_panel_kernel_ms * 1e-3) / 1e12
        # HBM bytes per panel launch from rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by the same
        # counters read for a 1 GiB device copy (profiles/panel_traffic_256x128.txt); known only
        # for that workload and the panel kernel as profiled there
        traffic = PANEL_TRAFFIC.get((args.nx, args.ny, args.prec))
        res["roofline"] = {"bound": "alu", "kernel": "k_panel (threshold-pivoting window factorization)",
                           "achieved": round(ach, 5), "peak": PEAK[dtype], "unit": "TFLOP/s",
                           "frac": round(ach / PEAK[dtype], 6), "traffic": traffic,
                           "traffic_unit": "bytes per launch (HBM, measured)",
                           "avg_launch_ms": round(avg_ms, 4), "launches": int(finfo.panel_launches),
                           "per_launch": "nominal window flops of one panel round over a tree level: "
                                         f"{finfo.panel_flops / max(1, finfo.panel_launches):.3e} flops"}
        # front TFLOP/s of the whole factorization against the MFMA peak of its precision
        res["front_tflops_frac"] = round(view.nominal_flops / t_factor / 1e12 / PEAK[dtype], 5)
        # extend-add and scatter (assembly phase): every contribution-block entry read
        # once and added into the parent (read-modify-write), every original entry
        # read once and added into its front
        import numpy as _np
        mm = _np.diff(view.rows_ptr).astype(_np.float64)
        pp = _np.diff(view.front_ptr).astype(_np.float64)
        cb = (mm - pp)[view.front_parent >= 0]
        sf = 8.0 if args.prec == "fp64" else 4.0
        asm_bytes = 3.0 * sf * float((cb * cb).sum()) + s.nnz * (8.0 + 2.0 * sf)
        res["roofline_assembly"] = {"bound": "hbm", "kernel": "k_gather + k_scatter (extend-add and value scatter)",
                                    "achieved": round(asm_bytes / (finfo.t_assemble_ms * 1e-3) / 1e9, 2),
                                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": round(asm_bytes / (finfo.t_assemble_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                                    "per_factorization_bytes": asm_bytes}
        if main["t_sweep"]:
            sw_bytes = view.nominal_nnz_lu * sf
            res["roofline_sweeps"] = {"bound": "hbm", "kernel": "forward + backward sweep pair (persistent upper tree, "
                                                                "level launches below) plus one residual",
                                      "achieved": round(sw_bytes / (main["t_sweep"] * 1e-3) / 1e9, 2),
                                      "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                      "frac": round(sw_bytes / (main["t_sweep"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                                      "ms": round(main["t_sweep"], 4), "bytes": sw_bytes}
        sch = finfo.schur_flops / (finfo.t_schur_ms * 1e-3) / 1e12
        res["roofline_schur"] = {"bound": "mfma", "kernel": "k_gemm mode 1 (contribution-block Schur update)",
                                 "achieved": round(sch, 4), "peak": PEAK[dtype], "unit": "TFLOP/s",
                                 "frac": round(sch / PEAK[dtype], 5),
                                 "per_launch": f"sum over a level's fronts of 2 (m-P)^2 k flops; "
                                               f"{finfo.schur_flops / max(1, finfo.schur_launches):.3e} flops"}
    if not args.no_extras and args.prec == "fp64" and not args.no_mixed:
        ru = run_reuse("fp32")
        tot = sum(ru["step_ms"])
        res["reuse"] = {"workload": f"the {nsteps_newton} Newton steps once, FP32 factors kept as the FP64 GMRES-IR "
                                    "preconditioner across steps (a reuse is capped at 20 GMRES iterations; "
                                    "refresh after > 10, back-off after a failed reuse)",
                        "ms_per_step": round(tot / nsteps_newton, 3),
                        "speedup_vs_fp64": round(1e3 * elapsed / args.steps / (tot / nsteps_newton), 4),
                        "steps": [{"ms": round(m, 3), "refactored": h.refactored, "retried": h.retried,
                                   "inner": h.inner_iters, "omega": h.omega}
                                  for m, h in zip(ru["step_ms"], ru["history"])]}
        log(f"reuse: {json.dumps(res['reuse'])}")
        # the same policy on Newton streams that change less per step (eps N(0,1)
        # relative, drawn on the device): where reuse starts to pay
        sens = {}
        for eps in (1e-3, 1e-4):
            g = torch.Generator(device=dev)
            g.manual_seed(17)
            seq = [vals[0]]
            for k in range(1, nsteps_newton):
                seq.append(seq[-1] * (1.0 + eps * torch.randn(s.nnz, generator=g, dtype=torch.float64, device=dev)))
            r = run_reuse("fp32", seq)
            t = sum(r["step_ms"]) / nsteps_newton
            sens[f"{eps:g}"] = {"ms_per_step": round(t, 3), "speedup_vs_fp64": round(1e3 * elapsed / args.steps / t, 4),
                                "refactored_steps": sum(h.refactored for h in r["history"]),
                                "inner": [h.inner_iters for h in r["history"]],
                                "omega_max": max(h.omega for h in r["history"])}
        res["reuse"]["smaller_changes"] = sens
        log(f"reuse with smaller changes per step: {json.dumps(sens)}")
    if not args.no_extras and args.prec == "fp64":
        res["ale_newton"] = bench_ale()
        log(f"ale newton: {json.dumps(res['ale_newton'])}")
        res["mixed_3d"] = bench_mixed_3d()
        log(f"mixed 3d: {json.dumps(res['mixed_3d'])}")
        gm = {}
        for pr in ("fp64", "fp32", "bf16"):
            tf, fl = gemm_micro(pr)
            pk = PEAK[{"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[pr]]
            gm[pr] = {"achieved": round(tf, 3), "peak": pk, "unit": "TFLOP/s", "frac": round(tf / pk, 5)}
        gm["workload"] = ("one dense front of order 4096 eliminating 2048 pivots: Schur GEMM of a 2048 x 2048 "
                          f"contribution block with K = 2048 ({fl:.3e} flops), timed with events")
        res["gemm_large_k"] = gm
        res["batch"] = bench_batch(argparse.Namespace(steps=5, warmup=1, prec="fp32", target_omega=args.target_omega),
                                   summary_only=True)
        log(f"batch: {json.dumps(res['batch'])}")
        # a short serving stream at one moderate rate (config 4's shape)
        res["serving"] = bench_serving(argparse.Namespace(rates="16", rate=16.0, requests=40, seed=args.seed,
                                                          mix_3d=0.3, target_omega=args.target_omega, max_cohorts=2),
                                       summary_only=True)
        log(f"serving: {json.dumps(res['serving'])}")
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(view.nominal_flops, full=not args.cpu_fit, nx=args.nx, ny=args.ny)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
