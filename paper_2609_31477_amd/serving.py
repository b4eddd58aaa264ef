"""Continuous-batching request loop for parametric VIV Newton-step solves.

Each request is one time step of the paper's solver (Sec. 3.4: Newton-Raphson
iterations, each a linear solve with the fixed-pattern Jacobian) for its own
mesh, Reynolds number and spring stiffness (the reduced velocity of Sec. 1 gives
k = pi^3 / U_r^2 for a massless cylinder with rho = L = U_inf = D = 1).  A request
runs ``newton_steps`` factor+solve steps with its symbolic analysis done once
(Sec. 6, "Scaling").

Scheduling (continuous batching, not a queue): requests arrive on a Poisson
clock; each arrival's preparation (its mesh's pattern analysis, done once per
mesh: the paper's analysis reuse, Sec. 6) starts at once on a host thread pool,
off the tick path; a prepared request is admitted when a slot and its HBM
footprint fit; every tick runs one Newton step of every admitted request.
Requests admitted together form a cohort, which shares one batched
factorization and one batched solve per step (shared launches); the cohort's
merged analysis is built once, when it is admitted, and reused for all its
steps.  A cohort is closed before its merged tree would pass the library's
limit of fronts per level.  The cohorts of a tick run at the same time, each
from its own host thread on its own stream (up to four), so work admitted at
different times overlaps on the device.  Requests that arrive while others are
on the GPU join at the next tick as a new cohort; finished requests free their
slot and memory immediately, and the analyses cached per mesh are counted
against the same HBM budget.  Because the batched kernels keep every system's
arithmetic separate, a request's result is the same alone and in any mix.

The scheduler is backend-agnostic: ``MFBackend`` drives libmf on the GPU;
``FakeBackend`` simulates durations and footprints for CPU tests of the logic.
"""
from __future__ import annotations

import heapq
import math
import threading
import time
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float                  # seconds on the scheduler clock
    mesh: tuple                     # ("2d", nx, ny) or ("3d", nx, ny, nz)
    reynolds: float
    reduced_velocity: float
    seed: int
    newton_steps: int = 5
    # filled by the scheduler
    admitted: float | None = None
    finished: float | None = None
    steps_done: int = 0
    step_latency: list = field(default_factory=list)
    footprint: int = 0
    cohort: int = -1                               # requests admitted together
    results: list = field(default_factory=list)   # per-step info (omega, ...)
    state: object = None                           # backend state
    prepared: object = None                        # Future of the backend's preparation (footprint)
    level_fronts: tuple = ()                       # fronts per tree level of its pattern

    @property
    def nu(self) -> float:
        return 1.0 / self.reynolds

    @property
    def k(self) -> float:
        return math.pi ** 3 / self.reduced_velocity ** 2


def poisson_requests(n, rate, seed=0, mix_3d=0.3, newton_steps=5, mesh_2d=range(32, 129, 4), allow_3d=True):
    """Poisson arrivals (rate per second) of mixed 2D/3D requests with Re ~ U[100,300],
    U_r ~ U[2,12] (2D) or U[2.5,17.5] (3D)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    meshes = list(mesh_2d)
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        is3d = allow_3d and rng.random() < mix_3d
        if is3d:
            mesh = ("3d", 24, 12, 6)
            ur = rng.uniform(2.5, 17.5)
        else:
            nx = int(meshes[rng.integers(len(meshes))])
            mesh = ("2d", nx, nx // 2)
            ur = rng.uniform(2.0, 12.0)
        out.append(Request(rid=i, arrival=t, mesh=mesh, reynolds=float(rng.uniform(100, 300)),
                           reduced_velocity=float(ur), seed=1000 + i, newton_steps=newton_steps))
    return out


MAX_LEVEL_FRONTS = 65535  # fronts per tree level of one batch (library limit)


class Scheduler:
    """Admission by footprint + continuous batching over Newton steps."""

    def __init__(self, backend, hbm_budget: int, max_slots: int = 64, max_cohorts: int | None = None):
        """``max_cohorts``: at most this many cohorts active at once (None: no cap).
        With a cap, arrivals wait while it is reached and then form one larger
        cohort, so a tick runs a few large batches instead of many small ones
        (each batch has a fixed cost per tree level)."""
        self.backend = backend
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.max_cohorts = max_cohorts
        self.used = 0
        self.active: list[Request] = []
        self.waiting: list = []       # heap of (arrival, rid, request)
        self.done: list[Request] = []
        self.ticks = 0
        self.batch_sizes = []
        self.cohorts = 0

    def submit(self, req: Request):
        heapq.heappush(self.waiting, (req.arrival, req.rid, req))

    def _start_preparation(self, now):
        # every request that has arrived starts its preparation at once (in the
        # background), whether or not a slot is free
        for _, _, req in self.waiting:
            if req.arrival <= now and req.prepared is None:
                req.prepared = self.backend.prepare_async(req)

    def _admit(self, now):
        self._start_preparation(now)
        if self.max_cohorts is not None and len({r.cohort for r in self.active}) >= self.max_cohorts:
            return                     # cohort cap reached: arrivals gather for the next cohort
        cohort = self.cohorts
        admitted = 0
        levels = []
        while self.waiting and self.waiting[0][0] <= now and len(self.active) < self.max_slots:
            _, _, req = self.waiting[0]
            if not req.prepared.done():
                break                  # FIFO: the head is still being analyzed
            req.footprint = req.prepared.result()
            if req.footprint > self.budget:
                raise MemoryError(f"request {req.rid} needs {req.footprint} B, above the whole budget")
            if self.used + self.backend.resident_bytes() + req.footprint > self.budget:
                break                  # wait until memory frees up (FIFO admission)
            lf = list(req.level_fronts)
            merged = [a + b for a, b in zip(levels + [0] * len(lf), lf + [0] * len(levels))]
            if admitted and max(merged, default=0) > MAX_LEVEL_FRONTS:
                cohort += 1            # close the cohort before it passes the fronts-per-level limit
                admitted = 0
                merged = lf
            heapq.heappop(self.waiting)
            self.used += req.footprint
            req.admitted = now
            req.cohort = cohort
            admitted += 1
            levels = merged
            self.active.append(req)
        if admitted:
            cohort += 1
        form = getattr(self.backend, "form_cohort", None)
        if form is not None:
            for c in range(self.cohorts, cohort):
                form(c, [r for r in self.active if r.cohort == c])
        self.cohorts = cohort

    def run(self, clock=None, idle_sleep=True, on_tick=None):
        """Serve until every submitted request is done.  ``clock()`` returns seconds
        since the start (wall clock by default; the fake backend advances its own);
        ``on_tick(scheduler)``, if given, is called after every tick."""
        t0 = time.perf_counter()
        clock = clock or (lambda: time.perf_counter() - t0)
        while self.waiting or self.active:
            now = clock()
            self._admit(now)
            if not self.active:
                nxt = self.waiting[0][0]
                if nxt <= now:         # the head has arrived: its analysis is still running
                    self.waiting[0][2].prepared.result()
                elif idle_sleep:
                    self.backend.idle_until(nxt, clock)
                continue
            ready = getattr(self.backend, "cohort_ready", None)
            batch = [r for r in self.active if ready is None or ready(r.cohort)]
            if not batch:              # every admitted cohort is still being merged
                self.backend.wait_cohort(self.active[0].cohort)
                continue
            ts = clock()
            infos = self.backend.step(batch)
            te = clock()
            self.ticks += 1
            self.batch_sizes.append(len(batch))
            for req, inf in zip(batch, infos):
                req.step_latency.append(te - ts)
                req.results.append(inf)
                req.steps_done += 1
                if req.steps_done >= req.newton_steps:
                    req.finished = te
                    self.active.remove(req)
                    self.used -= req.footprint
                    self.backend.release(req)
                    self.done.append(req)
            if on_tick is not None:
                on_tick(self)
        return self.done


def summarize(done):
    lat = np.array([r.finished - r.arrival for r in done])
    steps = np.array([s for r in done for s in r.step_latency])
    span = max(r.finished for r in done) - min(r.arrival for r in done)
    return {"requests": len(done), "solves": int(sum(r.steps_done for r in done)),
            "solves_per_s": float(sum(r.steps_done for r in done) / span),
            "p50_request_s": float(np.percentile(lat, 50)), "p99_request_s": float(np.percentile(lat, 99)),
            "p50_step_s": float(np.percentile(steps, 50)), "p99_step_s": float(np.percentile(steps, 99))}


class FakeBackend:
    """CPU stand-in: footprint and step time proportional to the mesh size; the
    clock is simulated so the scheduling logic is testable without a GPU."""

    def __init__(self, sec_per_dof=1e-8, bytes_per_dof=4000):
        self.sec_per_dof = sec_per_dof
        self.bytes_per_dof = bytes_per_dof
        self.now = 0.0
        self.calls = []

    def dofs(self, req):
        m = req.mesh
        return m[1] * m[2] * 8 if m[0] == "2d" else m[1] * m[2] * m[3] * 50

    def clock(self):
        return self.now

    def prepare(self, req):
        # a synthetic tree: leaves hold about 64 dofs, each level above half as many fronts
        f = max(1, self.dofs(req) // 64)
        lv = []
        while f >= 1:
            lv.append(f)
            f //= 2
        req.level_fronts = tuple(lv)
        return self.dofs(req) * self.bytes_per_dof

    def prepare_async(self, req):
        fut = Future()
        fut.set_result(self.prepare(req))
        return fut

    def resident_bytes(self):
        return 0

    def step(self, batch):
        self.calls.append([r.rid for r in batch])
        self.now += self.sec_per_dof * sum(self.dofs(r) for r in batch) + 1e-4
        return [{"omega": 0.0} for _ in batch]

    def release(self, req):
        pass

    def idle_until(self, t, clock):
        self.now = max(self.now, t)


class MFBackend:
    """libmf on the GPU: one symbolic handle per mesh pattern (analysis once), the
    request's Newton values and right-hand sides resident in HBM, and per cohort one
    merged batch (mf_batch_analyze once, its numeric handle reused across steps)
    driving one batched factorization + batched solve per tick.

    ``payloads`` (optional) gives what a server receives with the request: either a
    dict from request id to (system, [Newton values per step], [right-hand side per
    step]) as host arrays, or a callable ``payloads(req, device)`` returning the same
    triple with the values and right-hand sides already as device tensors; without
    it the backend assembles the request itself.  ``times`` keeps the host-side wall
    time spent per phase (prepare, merge, factor+solve)."""

    def __init__(self, prec="fp32", target_omega=1e-10, margin=0.5, device="cuda:0", payloads=None,
                 streams=4, prep_threads=4):
        import torch

        from . import Symbolic
        self.torch = torch
        self.Symbolic = Symbolic
        self.prec = prec
        self.target = target_omega
        self.margin = margin
        self.dev = torch.device(device)
        self.stream = torch.cuda.current_stream(self.dev)
        # cohorts of a tick run concurrently, each from its own thread and stream
        # (all streams at the default priority)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(max(1, streams))]
        self.pool = ThreadPoolExecutor(max_workers=len(self.streams))
        self.prep_pool = ThreadPoolExecutor(max_workers=max(1, prep_threads))
        self.lock = threading.Lock()
        self.tls = threading.local()    # per preparation thread: its upload stream
        self.payloads = payloads if payloads is not None else {}
        self.sym_cache = {}     # mesh -> Future of its analysis (Symbolic, level fronts)
        self.sym_bytes = {}     # mesh -> device bytes of its pattern data (charged to the budget)
        self.times = {"prepare": 0.0, "analyze": 0.0, "merge": 0.0, "factor_solve": 0.0}
        self.cohort_futs = {}   # cohort -> Future of its merged Batch
        self.cohort_left = {}   # cohort -> requests not finished yet

    def build(self, req):
        from vivjac import build_2d, build_3d
        if req.mesh[0] == "2d":
            return build_2d(req.mesh[1], req.mesh[2], req.seed, nu=req.nu, k=req.k)
        return build_3d(req.mesh[1], req.mesh[2], req.mesh[3], req.seed, nu=req.nu, k=req.k)

    def _analyze(self, s, mesh):
        ta = time.perf_counter()
        sym = self.Symbolic(s.n, s.rowptr, s.colind, s.root)
        v = sym.export()
        h = [0] * v.nfronts
        for f in range(v.nfronts):  # front heights (postorder: children first)
            p = int(v.front_parent[f])
            if p >= 0:
                h[p] = max(h[p], h[f] + 1)
        lf = [0] * (max(h) + 1 if h else 0)
        for x in h:
            lf[x] += 1
        with self.lock:
            self.times["analyze"] += time.perf_counter() - ta
            # pattern data resident on the device once the first factorization uploads it
            self.sym_bytes[mesh] = 4 * (v.rows_ptr[-1] * 3 + 8 * v.nfronts) + 12 * s.nnz + 16 * s.n
        return sym, tuple(lf)

    def prepare(self, req):
        t0 = time.perf_counter()
        # each preparation thread uploads on a stream of its own and waits for that
        # stream alone, so it never waits for the cohorts running on the device
        ps = getattr(self.tls, "stream", None)
        if ps is None:
            ps = self.tls.stream = self.torch.cuda.Stream(device=self.dev)
        with self.torch.cuda.stream(ps):
            return self._prepare_on(req, ps, t0)

    def _prepare_on(self, req, ps, t0):
        on_device = callable(self.payloads)
        if on_device:
            s, vals, rhs = self.payloads(req, self.dev)
        elif req.rid in self.payloads:
            s, hv, hb = self.payloads[req.rid]
        else:
            from vivjac import newton_rhs, newton_values
            s = self.build(req)
            hv = [newton_values(s, t) for t in range(req.newton_steps)]
            hb = [newton_rhs(s, t)[0].copy() for t in range(req.newton_steps)]
        with self.lock:
            fut = self.sym_cache.get(req.mesh)
            mine = fut is None
            if mine:
                fut = self.sym_cache[req.mesh] = Future()
        if mine:
            try:
                fut.set_result(self._analyze(s, req.mesh))
            except BaseException as e:  # hand the failure to every waiter
                fut.set_exception(e)
                raise
        sym, lf = fut.result()
        req.level_fronts = lf
        if not on_device:
            vals = [self.torch.from_numpy(v).to(self.dev) for v in hv]
            rhs = [self.torch.from_numpy(b).to(self.dev) for b in hb]
        if len(vals) < req.newton_steps or len(rhs) < req.newton_steps:
            raise ValueError(f"request {req.rid}: payload holds fewer than {req.newton_steps} Newton steps")
        xs = [self.torch.empty(s.n, dtype=self.torch.float64, device=self.dev) for _ in range(req.newton_steps)]
        ps.synchronize()
        req.state = dict(system=s, sym=sym, vals=vals, rhs=rhs, xs=xs)
        with self.lock:
            self.times["prepare"] += time.perf_counter() - t0
        return sym.footprint_bytes(self.prec, self.margin) + 8 * (s.nnz + 2 * s.n) * req.newton_steps

    def prepare_async(self, req):
        return self.prep_pool.submit(self.prepare, req)

    def resident_bytes(self):
        with self.lock:
            return int(sum(self.sym_bytes.values()))

    def _merge(self, members):
        from . import Batch
        tm = time.perf_counter()
        B = Batch([r.state["sym"] for r in members])
        with self.lock:
            self.times["merge"] += time.perf_counter() - tm
        return B

    def form_cohort(self, cohort, members):
        """A new cohort's merged analysis is built on the preparation pool, off the
        tick path: the cohort takes its first step in the first tick after it."""
        with self.lock:
            self.cohort_left[cohort] = len(members)
        self.cohort_futs[cohort] = self.prep_pool.submit(self._merge, members)

    def cohort_ready(self, cohort):
        f = self.cohort_futs.get(cohort)
        return f is not None and f.done()

    def wait_cohort(self, cohort):
        self.cohort_futs[cohort].result()

    def _run_cohort(self, cohort, members, stream):
        B = self.cohort_futs[cohort].result()
        vals = [r.state["vals"][r.steps_done] for r in members]
        bs = [r.state["rhs"][r.steps_done] for r in members]
        xs = [r.state["xs"][r.steps_done] for r in members]
        with self.torch.cuda.stream(stream):
            # a cohort factors once per Newton step: from its second step on, the
            # planned schedule enqueues every level at once (one synchronization);
            # cohorts run from several threads, so no graph is captured here
            B.factor(vals, stream=stream, prec=self.prec, target_omega=self.target, plan=1)
            _, out = B.solve(bs, xs=xs, stream=stream)
        stream.synchronize()
        return {r.rid: {"omega": inf.omega, "outer": inf.outer_iters, "inner": inf.inner_iters}
                for r, inf in zip(members, out)}

    def step(self, batch):
        t0 = time.perf_counter()
        groups = {}
        for r in batch:
            groups.setdefault(r.cohort, []).append(r)
        infos = {}
        futs = []
        for i, (cohort, members) in enumerate(groups.items()):
            if len({r.steps_done for r in members}) != 1:
                raise AssertionError("the requests of a cohort step together")
            if cohort not in self.cohort_futs:   # stepped without a scheduler: merge now
                self.form_cohort(cohort, members)
            futs.append(self.pool.submit(self._run_cohort, cohort, members, self.streams[i % len(self.streams)]))
        for f in futs:                 # each cohort waits for its own stream
            infos.update(f.result())
        self.times["factor_solve"] += time.perf_counter() - t0
        return [infos[r.rid] for r in batch]

    def release(self, req):
        st = req.state
        st["sym"] = None
        st["vals"] = None
        st["rhs"] = None
        with self.lock:
            self.cohort_left[req.cohort] -= 1
            last = self.cohort_left[req.cohort] == 0
        if last:                       # the cohort's batch goes with its last request
            del self.cohort_left[req.cohort]
            self.cohort_futs.pop(req.cohort).result().release()

    def close(self):
        self.pool.shutdown(wait=True)
        self.prep_pool.shutdown(wait=True)
        for f in self.cohort_futs.values():
            f.result().release()
        self.cohort_futs.clear()

    def idle_until(self, t, clock):
        dt = t - clock()
        if dt > 0:
            time.sleep(min(dt, 0.05))
