"""Serving loop: admission by footprint and continuous batching (CPU, fake device
backend), plus a GPU check that each request's result is the same alone and in
the mix."""
import numpy as np
import pytest

from paper_2609_31477_amd.serving import FakeBackend, Request, Scheduler, poisson_requests, summarize


def run_fake(reqs, budget, slots=64):
    be = FakeBackend()
    sch = Scheduler(be, hbm_budget=budget, max_slots=slots)
    for r in reqs:
        sch.submit(r)
    done = sch.run(clock=be.clock)
    return sch, be, done


def test_all_requests_complete_with_all_steps():
    reqs = poisson_requests(40, rate=50.0, seed=1, allow_3d=True)
    sch, be, done = run_fake(reqs, budget=10 ** 12)
    assert len(done) == 40
    assert all(r.steps_done == r.newton_steps == 5 for r in done)
    assert all(r.finished >= r.admitted >= r.arrival for r in done)
    s = summarize(done)
    assert s["solves"] == 200 and s["p99_request_s"] >= s["p50_request_s"] > 0


def test_continuous_batching_admits_during_service():
    # requests arriving while others run join later ticks (batches overlap in time)
    reqs = poisson_requests(30, rate=200.0, seed=2, allow_3d=False)
    sch, be, done = run_fake(reqs, budget=10 ** 12)
    assert max(sch.batch_sizes) > 1
    # some request was admitted while another was mid-way through its Newton steps
    mixed = any(len(set(c1) & set(c2)) and set(c2) - set(c1) for c1, c2 in zip(be.calls, be.calls[1:]))
    assert mixed


def test_admission_respects_hbm_budget():
    reqs = poisson_requests(20, rate=1000.0, seed=3, allow_3d=False)
    be = FakeBackend()
    fp = max(be.prepare(r) for r in reqs)
    budget = 2 * fp + 1
    sch = Scheduler(be, hbm_budget=budget)
    for r in reqs:
        sch.submit(r)
    seen = []
    orig = be.step

    def step(batch):
        seen.append(sum(r.footprint for r in batch))
        return orig(batch)
    be.step = step
    done = sch.run(clock=be.clock)
    assert len(done) == 20
    assert max(seen) <= budget
    assert sch.used == 0


def test_slot_limit():
    reqs = poisson_requests(12, rate=1000.0, seed=4, allow_3d=False)
    sch, be, done = run_fake(reqs, budget=10 ** 12, slots=3)
    assert max(sch.batch_sizes) <= 3 and len(done) == 12


def test_oversized_request_rejected():
    be = FakeBackend()
    sch = Scheduler(be, hbm_budget=10)
    sch.submit(Request(rid=0, arrival=0.0, mesh=("2d", 32, 16), reynolds=150, reduced_velocity=5, seed=1))
    with pytest.raises(MemoryError):
        sch.run(clock=be.clock)


def test_request_parameters_follow_reduced_velocity():
    r = Request(rid=0, arrival=0.0, mesh=("2d", 32, 16), reynolds=200.0, reduced_velocity=np.pi, seed=0)
    assert r.k == pytest.approx(np.pi) and r.nu == pytest.approx(1 / 200)


@pytest.mark.gpu
def test_gpu_serving_mix_equals_alone():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_31477_amd.serving import MFBackend
    reqs = poisson_requests(6, rate=200.0, seed=7, allow_3d=False, mesh_2d=range(16, 41, 4), newton_steps=2)
    be = MFBackend(prec="fp32", target_omega=1e-10)
    sch = Scheduler(be, hbm_budget=64 << 30)
    for r in reqs:
        sch.submit(r)
    done = sch.run()
    be.close()
    assert max(sch.batch_sizes) > 1
    for r in done:
        for t in range(r.newton_steps):
            xm = r.state["xs"][t].cpu().numpy()
            be1 = MFBackend(prec="fp32", target_omega=1e-10)
            alone = Request(rid=r.rid, arrival=0.0, mesh=r.mesh, reynolds=r.reynolds,
                            reduced_velocity=r.reduced_velocity, seed=r.seed, newton_steps=r.newton_steps)
            be1.prepare(alone)
            alone.steps_done = t
            be1.step([alone])
            xa = alone.state["xs"][t].cpu().numpy()
            be1.close()
            assert np.array_equal(xm, xa), f"request {r.rid} step {t} differs alone vs in the mix"
            assert r.results[t]["omega"] <= 1e-10


def test_cohorts_group_requests_admitted_together():
    # requests admitted in the same admission pass share a cohort id; later arrivals get
    # new ids, and a cohort's members always run the same Newton step together
    reqs = poisson_requests(30, rate=300.0, seed=5, allow_3d=False)
    sch, be, done = run_fake(reqs, budget=10 ** 12)
    assert sch.cohorts >= 2
    by_cohort = {}
    for r in done:
        assert r.cohort >= 0
        by_cohort.setdefault(r.cohort, []).append(r)
    for members in by_cohort.values():
        assert len({r.admitted for r in members}) == 1
        assert len({r.finished for r in members}) == 1


def test_cohort_closed_before_level_limit():
    # patterns whose widest level holds 40,000 fronts: two of them would pass the
    # library's 65,535 fronts per level, so each admission pass splits them into
    # separate cohorts (and separate batched launches)
    class Wide(FakeBackend):
        def prepare(self, req):
            fp = super().prepare(req)
            req.level_fronts = (40000, 20000, 1)
            return fp
    be = Wide()
    sch = Scheduler(be, hbm_budget=10 ** 12)
    reqs = poisson_requests(6, rate=1e6, seed=9, allow_3d=False)
    for r in reqs:
        sch.submit(r)
    done = sch.run(clock=be.clock)
    assert len(done) == 6
    for call in be.calls:
        by = {}
        for rid in call:
            c = next(r.cohort for r in done if r.rid == rid)
            by[c] = by.get(c, 0) + 1
        assert max(by.values()) == 1


def test_preparation_runs_off_the_tick_path():
    # a request whose analysis is still running does not block the ticks of the
    # requests already admitted; it is admitted once its preparation completes
    from concurrent.futures import Future
    pending = {}

    class Slow(FakeBackend):
        def prepare_async(self, req):
            fut = Future()
            if req.rid == 1:
                pending[1] = (fut, self.prepare(req))
            else:
                fut.set_result(self.prepare(req))
            return fut

        def step(self, batch):
            out = super().step(batch)
            if 1 in pending and len(self.calls) == 3:   # the analysis finishes during the third tick
                fut, fp = pending.pop(1)
                fut.set_result(fp)
            return out
    be = Slow()
    sch = Scheduler(be, hbm_budget=10 ** 12)
    r0 = Request(rid=0, arrival=0.0, mesh=("2d", 32, 16), reynolds=150, reduced_velocity=5, seed=1)
    r1 = Request(rid=1, arrival=0.0, mesh=("2d", 64, 32), reynolds=150, reduced_velocity=5, seed=2)
    sch.submit(r0)
    sch.submit(r1)
    sch.run(clock=be.clock)
    assert be.calls[0] == [0] and be.calls[1] == [0] and be.calls[2] == [0]
    assert 1 in be.calls[3]
    assert r1.admitted is not None and r1.admitted > r0.admitted


def test_cohort_cap_bounds_concurrent_cohorts():
    """With max_cohorts = 2 no tick runs more than two cohorts; every request
    still finishes, and arrivals held back join a later, larger cohort."""
    reqs = poisson_requests(60, rate=400.0, seed=11, allow_3d=False)
    be = FakeBackend()
    sch = Scheduler(be, hbm_budget=10 ** 12, max_cohorts=2)
    for r in reqs:
        sch.submit(r)
    seen = []
    done = sch.run(clock=be.clock, on_tick=lambda sc: seen.append(len({r.cohort for r in sc.active})))
    assert len(done) == 60
    assert max(seen) <= 2
    free = Scheduler(FakeBackend(), hbm_budget=10 ** 12)
    for r in poisson_requests(60, rate=400.0, seed=11, allow_3d=False):
        free.submit(r)
    free.run(clock=free.backend.clock)
    assert sch.cohorts < free.cohorts            # fewer, larger cohorts under the cap
