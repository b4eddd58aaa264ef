"""GPU parity on the 3D box Jacobians (Kuhn tetrahedra, P2-P1 flow, P2 mesh
displacement, multiplier on the cylinder's lateral faces, two position dofs).

Small boxes against the oracle's sparse LU directly; the serving workload's
24x12x6 box (n = 84,825) against the oracle's solution at sampled entries,
stored by tests/golden/make_box_24x12x6.py (which calls only the oracle).
Bars as in 2D: FP64 relative error 1e-8 overall and per unknown block and
backward error 1e-12; mixed paths backward error 1e-10."""
import json
import os

import numpy as np
import pytest

import paper_2609_31477_amd as mf
from oracle import check, splu, sym as osym
from vivjac import build_3d, newton_rhs, newton_values

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "box_24x12x6_seed3.json")
BLOCKS = ("u", "p", "d", "lam", "s")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def per_block(s, x, xo):
    out = {}
    for k in BLOCKS:
        lo, hi = s.blocks[k]
        out[k] = float(np.abs(x[lo:hi] - xo[lo:hi]).max() / np.abs(xo[lo:hi]).max())
    return out


@pytest.mark.timeout(300)
@pytest.mark.parametrize("dims,prec", [((8, 4, 2), "fp64"), ((12, 6, 3), "fp64"), ((12, 6, 3), "fp32"),
                                       ((12, 6, 3), "bf16")])
def test_small_box_vs_oracle(torch_cuda, dims, prec):
    torch = torch_cuda
    s = build_3d(*dims, 1)
    b = s.b0[0]
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    target = 1e-12 if prec == "fp64" else 1e-10
    num = S.factor(torch.from_numpy(s.values).cuda(), prec=prec, target_omega=target)
    x, info = num.solve(torch.from_numpy(b.copy()).cuda())
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    Os = osym.analyze(s.n, s.rowptr, s.colind, s.root)
    xo, om, _ = splu.SparseLU(s.n, s.rowptr, s.colind, s.values, Os.perm).solve(b)
    A = s.to_scipy()
    w = check.omega(A, x, b)
    rel = float(np.abs(x - xo).max() / np.abs(xo).max())
    pb = per_block(s, x, xo)
    print(f"{dims} {prec}: n={s.n} omega={w:.2e} rel={rel:.2e} delayed={num.info().delayed_pivots} "
          f"max front {num.info().max_front} outer {info.outer_iters} inner {info.inner_iters} "
          + " ".join(f"{k}={v:.1e}" for k, v in pb.items()), flush=True)
    assert w <= target
    assert rel <= 1e-8
    assert max(pb.values()) <= 1e-8
    assert info.fp64_fallback == 0


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_box_24x12x6_sampled(torch_cuda, prec):
    torch = torch_cuda
    g = json.load(open(GOLDEN))
    s = build_3d(*g["mesh"], g["seed"])
    assert (s.n, s.nnz) == (g["n"], g["nnz"])
    idx = np.asarray(g["index"], dtype=np.int64)
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    v = newton_values(s, 0)
    b = newton_rhs(s, 0)[0]
    target = 1e-12 if prec == "fp64" else 1e-10
    num = S.factor(torch.from_numpy(v).cuda(), prec=prec, target_omega=target)
    fi = num.info()
    x, info = num.solve(torch.from_numpy(b.copy()).cuda())
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    xo = np.asarray(g["x"])
    err = float(np.abs(x[idx] - xo).max() / g["xinf"])
    om = check.omega_fast(s.to_scipy(v), x, b)
    be = {}
    for k in BLOCKS:
        lo, hi = g["blocks"][k]
        sel = (idx >= lo) & (idx < hi)
        be[k] = float(np.abs(x[idx][sel] - xo[sel]).max() / g["block_inf"][k])
    print(f"24x12x6 {prec}: omega={om:.2e} sampled rel err={err:.2e} delayed={fi.delayed_pivots} "
          f"max front {fi.max_front} flops {fi.factor_flops:.3e} outer {info.outer_iters} inner {info.inner_iters} "
          + " ".join(f"{k}={v_:.1e}" for k, v_ in be.items()), flush=True)
    assert om <= target
    assert err <= 1e-8
    assert max(be.values()) <= 1e-8
    num.release()
