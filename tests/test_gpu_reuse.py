"""The Krylov solver with a kept multifrontal preconditioner (mf_set_operator):
factors of one Newton step precondition FP64 GMRES-IR on a later step's Jacobian.

Bar: the solution of the NEW matrix meets omega <= 1e-10 (recomputed here on the
CPU against that matrix) and agrees with the oracle's solution of it to 1e-6
relative (the mixed-precision bar); batched reuse equals single-system reuse
bitwise; bad values and failed reuse take their documented paths."""
import ctypes

import numpy as np
import pytest

import paper_2609_31477_amd as mf
from oracle import check, splu, sym as osym
from vivjac import build_2d, newton_rhs, newton_values

pytestmark = pytest.mark.gpu

TARGET = 1e-10


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def oracle_solve(s, vals, B):
    S = osym.analyze(s.n, s.rowptr, s.colind, s.root)
    X, _, _ = splu.SparseLU(s.n, s.rowptr, s.colind, vals, S.perm, tau=1.0).solve(B)
    return X


@pytest.mark.parametrize("prec,step", [("fp32", 1), ("bf16", 1), ("fp64", 2)])
def test_set_operator_solves_the_new_matrix(torch_cuda, prec, step):
    torch = torch_cuda
    dev = torch.device("cuda:0")
    s = build_2d(32, 16, 5)
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    v0 = torch.from_numpy(newton_values(s, 0)).to(dev)
    vt_h = newton_values(s, step)
    bt_h = newton_rhs(s, step)[0]
    num = S.factor(v0, prec=prec, target_omega=TARGET, max_outer=10)
    num.set_operator(torch.from_numpy(vt_h).to(dev))
    x, info = num.solve(torch.from_numpy(bt_h).to(dev))
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    A = s.to_scipy(vt_h)
    om = check.omega(A, x, bt_h)
    xo = oracle_solve(s, vt_h, bt_h)
    rel = np.abs(x - xo).max() / np.abs(xo).max()
    print(f"{prec} step {step}: omega={om:.2e} rel={rel:.2e} omega0={info.omega0:.2e} outer={info.outer_iters} "
          f"inner={info.inner_iters} fallback={info.fp64_fallback}", flush=True)
    assert info.fp64_fallback == 0
    assert info.inner_iters > 0          # the Krylov correction ran, also for FP64 factors
    assert om <= TARGET and info.omega <= TARGET
    assert rel <= 1e-6
    # the kept factors are those of step 0: the unrefined solution is far from the new one
    assert info.omega0 > TARGET


def test_set_operator_batched_equals_alone(torch_cuda):
    torch = torch_cuda
    dev = torch.device("cuda:0")
    systems = [build_2d(nx, nx // 2, 200 + nx) for nx in (16, 24, 20)]
    syms = [mf.Symbolic(s.n, s.rowptr, s.colind, s.root) for s in systems]
    v0 = [torch.from_numpy(newton_values(s, 0)).to(dev) for s in systems]
    v1 = [torch.from_numpy(newton_values(s, 1)).to(dev) for s in systems]
    b1 = [torch.from_numpy(newton_rhs(s, 1)[0]).to(dev) for s in systems]
    alone = []
    for S, a, b, c in zip(syms, v0, v1, b1):
        num = S.factor(a, prec="fp32", target_omega=TARGET)
        num.set_operator(b)
        alone.append(num.solve(c)[0].cpu().numpy())
    B = mf.Batch(syms)
    B.factor(v0, prec="fp32", target_omega=TARGET)
    B.set_operator(v1)
    xs, infos = B.solve(b1)
    torch.cuda.synchronize()
    for s, x, xa, inf, vh in zip(systems, xs, alone, infos, v1):
        xb = x.cpu().numpy()
        om = check.omega(s.to_scipy(vh.cpu().numpy()), xb, b1[systems.index(s)].cpu().numpy())
        print(f"n={s.n} omega={om:.2e} inner={inf.inner_iters}", flush=True)
        assert np.array_equal(xb, xa)
        assert om <= TARGET


def test_set_operator_rejects_nonfinite_and_wrong_kind(torch_cuda):
    torch = torch_cuda
    dev = torch.device("cuda:0")
    s = build_2d(16, 8, 0)
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    v = torch.from_numpy(s.values).to(dev)
    num = S.factor(v, prec="fp32", target_omega=TARGET)
    B = mf.Batch([S, S])
    B.factor([v, v], prec="fp32", target_omega=TARGET)
    with pytest.raises(mf.MFError) as e:      # a batch handle through the single-system call
        mf._check(mf.lib().mf_set_operator(B._num, ctypes.c_void_p(v.data_ptr()), None, None))
    assert e.value.status == mf.MF_ERR_ARG and "batched" in str(e.value)
    B.release()
    bad = v.clone()
    bad[17] = float("nan")
    with pytest.raises(mf.MFError) as e:
        num.set_operator(bad)
    assert e.value.status == mf.MF_ERR_ARG and "[17]" in str(e.value)
    with pytest.raises(mf.MFError) as e:      # the handle must be factored again
        num.solve(torch.from_numpy(s.b0[0]).to(dev))
    assert e.value.status == mf.MF_ERR_STATE
    num = S.factor(v, numeric=num, prec="fp32", target_omega=TARGET)
    _, info = num.solve(torch.from_numpy(s.b0[0]).to(dev))
    assert info.omega <= TARGET


def test_failed_reuse_falls_back_to_fp64(torch_cuda):
    """A kept factorization too far from the new matrix for the allowed iterations:
    the handle's FP64 fallback factors the new values and solves them."""
    torch = torch_cuda
    dev = torch.device("cuda:0")
    s = build_2d(32, 16, 6)
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    num = S.factor(torch.from_numpy(newton_values(s, 0)).to(dev), prec="fp32", target_omega=1e-12,
                   gmres_m=2, max_outer=1, fallback=1)
    v4 = newton_values(s, 4)
    b4 = newton_rhs(s, 4)[0]
    num.set_operator(torch.from_numpy(v4).to(dev))
    x, info = num.solve(torch.from_numpy(b4).to(dev))
    x = x.cpu().numpy()
    om = check.omega(s.to_scipy(v4), x, b4)
    print(f"omega={om:.2e} fallback={info.fp64_fallback}", flush=True)
    assert info.fp64_fallback == 1
    assert om <= 1e-12


def _smooth_stream(s, eps, steps, seed=3):
    """Newton values whose relative change per step is eps N(0,1) (the configured
    stream uses eps = 0.01)."""
    rng = np.random.default_rng(seed)
    v = [s.values.copy()]
    for _ in range(1, steps):
        v.append(v[-1] * (1.0 + eps * rng.standard_normal(s.nnz)))
    return v


@pytest.mark.parametrize("eps,expect_reuse", [(1e-4, True), (1e-2, False)])
def test_reused_factor_newton_sequence(torch_cuda, eps, expect_reuse):
    """Five Newton steps through the reuse policy: every step meets the target on
    its own matrix.  With small changes between steps the kept factors serve every
    later step; with the configured 1% changes a capped reuse fails, the step is
    factored afresh and reuse backs off."""
    from paper_2609_31477_amd.newton import ReusedFactorNewton
    torch = torch_cuda
    dev = torch.device("cuda:0")
    s = build_2d(64, 32, 8)
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    solver = ReusedFactorNewton(S, prec="fp32", target_omega=TARGET, max_inner=10, reuse_m=20, reuse_outer=1)
    vs = _smooth_stream(s, eps, 5)
    for t in range(5):
        bt = newton_rhs(s, t)[0]
        x, info, rec = solver.step(torch.from_numpy(vs[t]).to(dev), torch.from_numpy(bt).to(dev))
        om = check.omega(s.to_scipy(vs[t]), x.cpu().numpy(), bt)
        print(f"eps={eps} step {t}: {rec} omega(cpu)={om:.2e}", flush=True)
        assert om <= TARGET
        if not rec.refactored:
            assert rec.inner_iters <= 20
    h = solver.history
    assert h[0].refactored
    if expect_reuse:
        assert not any(r.refactored for r in h[1:])
    else:
        assert h[1].retried and h[2].refactored and not h[2].retried   # backed off after the failure
    solver.release()
