"""GPU parity at the benchmark's full size: the 256x128 Newton sequence (seed 1,
n = 540,606, nnz = 14,008,134), five steps on one symbolic analysis, FP64 path
in the benchmark's launch configuration.

Expected values are the oracle's solutions at 2,050 sampled entries (2,048
random + the two position unknowns), stored by tests/golden/make_newton_256x128.py,
which calls only the oracle, with the infinity norm of each unknown block.  Bar:
|x - x_oracle| <= 1e-8 * ||x_oracle||_inf on every sampled entry, the same bar
per block (velocity, pressure, mesh displacement, multiplier, and the two
position unknowns measured against their own magnitude), and the componentwise
backward error of the whole GPU solution (computed on the CPU from the
generator's matrix) <= 1e-12 for the FP64 path, <= 1e-10 for the mixed paths."""
import json
import os

import numpy as np
import pytest

import paper_2609_31477_amd as mf
from oracle import check
from vivjac import build_2d, newton_rhs, newton_values

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "newton_256x128_seed1.json")
BLOCKS = ("u", "p", "d", "lam", "s")
# The mixed paths' target bounds the backward error (1e-10) rather than the
# forward error of each block; observed per-block errors stay below 1e-10, and
# they are held to the FP64 path's bar.
MIXED_BLOCK_TOL = 1e-8


def block_errors(g, idx, x_sampled, ref):
    """Largest sampled error of each unknown block relative to that block's own
    infinity norm (ref: one golden solution record with "x" and "block_inf")."""
    xo = np.asarray(ref["x"])
    out = {}
    for k in BLOCKS:
        lo, hi = g["blocks"][k]
        sel = (idx >= lo) & (idx < hi)
        out[k] = float(np.abs(x_sampled[sel] - xo[sel]).max() / ref["block_inf"][k]) if sel.any() else 0.0
    return out


def assert_blocks(g, idx, x, ref, tol=1e-8):
    be = block_errors(g, idx, x[idx], ref)
    print("  per-block rel err: " + " ".join(f"{k}={v:.1e}" for k, v in be.items()), flush=True)
    assert max(be.values()) <= tol, be
    # the two position unknowns are both sampled
    lo, hi = g["blocks"]["s"]
    assert np.isin(np.arange(lo, hi), idx).all()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.timeout(900)
def test_newton_256x128_sampled(torch_cuda):
    torch = torch_cuda
    g = json.load(open(GOLDEN))
    print("generating the 256x128 system", flush=True)
    s = build_2d(*g["mesh"], g["seed"])
    assert (s.n, s.nnz) == (g["n"], g["nnz"])
    idx = np.asarray(g["index"], dtype=np.int64)
    dev = torch.device("cuda:0")
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    for st in g["steps"]:
        t = st["step"]
        v = newton_values(s, t)
        b = newton_rhs(s, t)[0]
        num = S.factor(torch.from_numpy(v).to(dev))
        x, info = num.solve(torch.from_numpy(b.copy()).to(dev))
        torch.cuda.synchronize()
        x = x.cpu().numpy()
        err = np.abs(x[idx] - np.asarray(st["x"])).max() / st["xinf"]
        A = s.to_scipy(v)
        om = check.omega_fast(A, x, b)
        fi = num.info()
        print(f"step {t}: sampled rel err={err:.2e} omega={om:.2e} (device {info.omega:.2e}, "
              f"refinement {info.outer_iters}) delayed={fi.delayed_pivots}", flush=True)
        assert err <= 1e-8
        assert om <= 1e-12
        assert info.outer_iters <= 2
        assert_blocks(g, idx, x, st)
        assert info.delayed_pivots == fi.delayed_pivots
        num.release()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_newton_256x128_mixed(torch_cuda, prec):
    """The mixed paths at full size (FP32 fronts, or BF16 Schur-update operands
    with FP32 accumulation; FP64 root; FP64 GMRES-IR): the componentwise backward
    error of every step's solution, recomputed on the CPU from the generator's
    matrix, meets the mixed target 1e-10, and the sampled entries agree with the
    oracle's FP64 solution to the plain FP64 path's bar (1e-8 relative to the
    largest entry, and per block), without the FP64 fallback."""
    torch = torch_cuda
    g = json.load(open(GOLDEN))
    s = build_2d(*g["mesh"], g["seed"])
    idx = np.asarray(g["index"], dtype=np.int64)
    dev = torch.device("cuda:0")
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    num = None
    for st in g["steps"]:
        t = st["step"]
        v = newton_values(s, t)
        b = newton_rhs(s, t)[0]
        num = S.factor(torch.from_numpy(v).to(dev), numeric=num, prec=prec, target_omega=1e-10)
        x, info = num.solve(torch.from_numpy(b.copy()).to(dev))
        torch.cuda.synchronize()
        x = x.cpu().numpy()
        err = np.abs(x[idx] - np.asarray(st["x"])).max() / st["xinf"]
        om = check.omega_fast(s.to_scipy(v), x, b)
        print(f"{prec} step {t}: sampled rel err={err:.2e} omega={om:.2e} (device {info.omega:.2e}, "
              f"eta {info.eta:.1e}, outer {info.outer_iters}, inner {info.inner_iters})", flush=True)
        assert om <= 1e-10
        assert err <= 1e-8
        assert info.fp64_fallback == 0
        assert_blocks(g, idx, x, st, tol=MIXED_BLOCK_TOL)
    num.release()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_newton_256x128_mixed_eight_rhs(torch_cuda, prec):
    """Eight right-hand sides on the step-0 matrix in one mixed solve (GMRES-IR
    runs the eight instances in lockstep): every column's backward error meets
    1e-10 and its sampled entries agree with the oracle's solution of that column
    to 1e-8, overall and per block."""
    torch = torch_cuda
    g = json.load(open(GOLDEN))
    s = build_2d(*g["mesh"], g["seed"])
    idx = np.asarray(g["index"], dtype=np.int64)
    dev = torch.device("cuda:0")
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    v = newton_values(s, 0)
    B = newton_rhs(s, 0, nrhs=8)
    num = S.factor(torch.from_numpy(v).to(dev), prec=prec, target_omega=1e-10)
    X, info = num.solve(torch.from_numpy(B.copy()).to(dev))
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    A = s.to_scipy(v)
    print(f"{prec} 8 rhs: device omega {info.omega:.2e} outer {info.outer_iters} inner {info.inner_iters}", flush=True)
    assert info.fp64_fallback == 0
    for c in range(8):
        ref = g["eight_rhs"][c]
        om = check.omega_fast(A, X[c], B[c])
        err = np.abs(X[c][idx] - np.asarray(ref["x"])).max() / ref["xinf"]
        print(f" rhs {c}: omega={om:.2e} sampled rel err={err:.2e}", flush=True)
        assert om <= 1e-10
        assert err <= 1e-8
        assert_blocks(g, idx, X[c], ref, tol=MIXED_BLOCK_TOL)
    num.release()


@pytest.mark.timeout(900)
def test_newton_256x128_eight_rhs(torch_cuda):
    """Eight right-hand sides at full size in one solve: the largest front (order
    1,464) then needs 94 KB of sweep vectors in LDS beside the staged diagonal
    block, so the chunking of right-hand sides against the device's LDS limit is
    exercised.  Every column meets the FP64 target (componentwise backward error
    recomputed on the CPU) and matches the same column solved alone to 1e-12
    relative to its largest entry."""
    torch = torch_cuda
    props = torch.cuda.get_device_properties(0)
    print("LDS per block:", getattr(props, "shared_memory_per_block", "n/a"), flush=True)
    g = json.load(open(GOLDEN))
    s = build_2d(*g["mesh"], g["seed"])
    dev = torch.device("cuda:0")
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    v = newton_values(s, 0)
    rng = np.random.default_rng(7)
    B = np.vstack([newton_rhs(s, 0)[0], rng.standard_normal((7, s.n))])
    num = S.factor(torch.from_numpy(v).to(dev))
    X, info = num.solve(torch.from_numpy(B.copy()).to(dev))
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    A = s.to_scipy(v)
    for c in range(8):
        om = check.omega_fast(A, X[c], B[c])
        x1, _ = num.solve(torch.from_numpy(B[c].copy()).to(dev))
        x1 = x1.cpu().numpy()
        d = np.abs(X[c] - x1).max() / np.abs(x1).max()
        print(f"rhs {c}: omega={om:.2e} vs alone {d:.2e}", flush=True)
        assert om <= 1e-12
        assert d <= 1e-12
    num.release()


@pytest.mark.timeout(900)
def test_newton_256x128_planned_bitwise(torch_cuda):
    """The planned schedule with graph replay at full size, over four Newton
    steps: fronts are stored at planned capacities above their orders, the front
    with 57 children is gathered in row chunks, and capacity overflows repeat the
    factorization level by level.  Every step's solution equals the
    level-by-level one bitwise."""
    torch = torch_cuda
    g = json.load(open(GOLDEN))
    s = build_2d(*g["mesh"], g["seed"])
    dev = torch.device("cuda:0")
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    num_l = num_p = None
    for t in range(4):
        v = torch.from_numpy(newton_values(s, t)).to(dev)
        b = torch.from_numpy(newton_rhs(s, t)[0].copy()).to(dev)
        num_l = S.factor(v, numeric=num_l, plan=0)
        xl, _ = num_l.solve(b)
        num_p = S.factor(v, numeric=num_p, plan=2)
        xp, _ = num_p.solve(b)
        torch.cuda.synchronize()
        fi = num_p.info()
        same = bool(torch.equal(xl, xp))
        print(f"step {t}: planned={fi.planned} fallbacks={fi.plan_fallbacks} bitwise equal={same}", flush=True)
        assert same
    num_l.release()
    num_p.release()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_newton_256x128_columns_bitwise_alone(torch_cuda, prec):
    """The sweeps take up to eight right-hand sides per pass (each factor entry
    loaded once for all of them) with every column's arithmetic that of a column
    alone.  Without refinement, each of eleven columns (a pass of eight, then one
    of three: the one-wave small-front kernels take them four at a time, so the
    passes have 4+4 and 3 live columns there, 8 and 3 elsewhere) equals the same
    column swept alone, bit for bit, through the persistent upper tree and the
    level kernels of the lower levels."""
    torch = torch_cuda
    s = build_2d(256, 128, 1)
    dev = torch.device("cuda:0")
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    rng = np.random.default_rng(11)
    B = rng.standard_normal((11, s.n))
    num = S.factor(torch.from_numpy(newton_values(s, 1)).to(dev), prec=prec, refine=0)
    X, _ = num.solve(torch.from_numpy(B.copy()).to(dev), check=False)
    X = X.cpu().numpy()
    for c in range(11):
        x1, _ = num.solve(torch.from_numpy(B[c].copy()).to(dev), check=False)
        x1 = x1.cpu().numpy()
        nd = int((X[c] != x1).sum())
        print(f"{prec} column {c}: {nd} entries differ from the column alone", flush=True)
        assert nd == 0
    num.release()
