"""Planned schedule (options.plan = 1, and 2 with graph replay): once a handle
has factored once level by level, the next factorizations reuse its front
capacities and enqueue every tree level at once.  They must produce exactly the factors of the level-by-level
schedule (same arithmetic in every kernel, only storage and launch shapes
differ), and a front that outgrows its capacity must make the call continue
level by level from that front's level, again with the same result."""
import numpy as np
import pytest

import paper_2609_31477_amd as mf
from vivjac import build_2d, newton_rhs, newton_values

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run(torch, S, vals, b, num=None, **opts):
    dev = torch.device("cuda:0")
    num = S.factor(torch.from_numpy(vals).to(dev), numeric=num, **opts)
    x, info = num.solve(torch.from_numpy(b.copy()).to(dev))
    torch.cuda.synchronize()
    return num, x.cpu().numpy(), info


@pytest.mark.parametrize("prec,plan", [("fp64", 1), ("fp32", 1), ("fp64", 2), ("fp32", 2)])
def test_planned_equals_levelwise(torch_cuda, prec, plan):
    """plan = 2 replays the captured graph on steps 1-3, with the solves' own
    work and synchronizations between the replays; every replay is checked."""
    s = build_2d(32, 16, 1)
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    num_p = num_l = None
    for t in range(4):
        v, b = newton_values(s, t), newton_rhs(s, t)[0]
        num_l, x_l, _ = run(torch_cuda, S, v, b, num_l, prec=prec, plan=0)
        num_p, x_p, _ = run(torch_cuda, S, v, b, num_p, prec=prec, plan=plan)
        fl, fp = num_l.info(), num_p.info()
        print(f"{prec} step {t}: planned={fp.planned} fallbacks={fp.plan_fallbacks} "
              f"delayed {fp.delayed_pivots} (level-wise {fl.delayed_pivots})", flush=True)
        assert fl.planned == 0
        assert fp.planned == (plan if t > 0 else 0)
        assert fp.delayed_pivots == fl.delayed_pivots
        assert fp.max_front == fl.max_front
        assert np.array_equal(x_p, x_l)


@pytest.mark.parametrize("plan", [1, 2])
def test_plan_overflow_falls_back(torch_cuda, plan):
    """The overflowing run keeps the planned levels below the first front that
    outgrew its capacity and factors the rest level by level."""
    s = build_2d(32, 16, 1)
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    v, b = newton_values(s, 0), newton_rhs(s, 0)[0]
    # u = 0 accepts any nonzero pivot: few delays, so small capacities (no solve:
    # such factors are too inaccurate for refinement to reach the target) ...
    num = S.factor(torch_cuda.from_numpy(v).to(torch_cuda.device("cuda:0")), pivot_u=0.0, plan=plan)
    few = num.info().delayed_pivots
    # ... which u = 1 (pivot must be the largest entry of its column) outgrows
    num, x1, _ = run(torch_cuda, S, v, b, num, pivot_u=1.0, plan=plan)
    f1 = num.info()
    _, x_ref, _ = run(torch_cuda, S, v, b, None, pivot_u=1.0, plan=0)
    print(f"delayed: u=0 {few}, u=1 {f1.delayed_pivots}; planned={f1.planned} fallbacks={f1.plan_fallbacks}",
          flush=True)
    assert f1.delayed_pivots > few
    assert f1.planned == 0 and f1.plan_fallbacks == 1
    assert np.array_equal(x1, x_ref)
    # the enlarged plan now holds
    num, x2, _ = run(torch_cuda, S, v, b, num, pivot_u=1.0, plan=plan)
    f2 = num.info()
    assert f2.planned == plan and f2.plan_fallbacks == 1
    assert np.array_equal(x2, x_ref)


@pytest.mark.parametrize("plan", [0, 1])
def test_tuner_keeps_results(torch_cuda, plan):
    """options.tune: the four trial factorizations (each launch shape on every
    level) and the tuned ones after them give exactly the results of the fixed
    heuristic shapes."""
    s = build_2d(32, 16, 1)
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    num_t = num_f = None
    for t in range(7):
        v, b = newton_values(s, t % 5), newton_rhs(s, t % 5)[0]
        num_f, x_f, _ = run(torch_cuda, S, v, b, num_f, plan=0, tune=0)
        num_t, x_t, _ = run(torch_cuda, S, v, b, num_t, plan=plan, tune=1)
        fi = num_t.info()
        print(f"factorization {t}: tuned={fi.tuned} planned={fi.planned}", flush=True)
        assert fi.tuned == (1 if t >= 4 else 0)
        assert np.array_equal(x_t, x_f)
