"""The no-allocation solve entry point (mf_solve_noalloc) against mf_solve.

Two calls in a row through the C ABI on the GPU, the second on a smaller
system, so the shared static scratch holds the first call's contents when the
second starts: each result equals mf_solve's with the same (level-by-level)
sweeps bitwise, and meets the FP64 parity bar against mf_solve's default
result (relative error 1e-8, backward error 1e-12)."""
import numpy as np
import pytest

import paper_2609_31477_amd as mf
from oracle import check
from vivjac import build_2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_noalloc_matches_solve_two_calls(torch_cuda):
    torch = torch_cuda
    dev = torch.device("cuda:0")
    for (nx, ny, seed, nrhs) in [(64, 32, 3, 2), (16, 8, 0, 1)]:
        s = build_2d(nx, ny, seed, nrhs=nrhs)
        S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
        v = torch.from_numpy(s.values).to(dev)
        B = s.b0 if nrhs > 1 else s.b0[0]
        b = torch.from_numpy(np.ascontiguousarray(B)).to(dev)
        ref = S.factor(v, sweep=0)
        x_ref, i_ref = ref.solve(b)
        x_def, _ = S.factor(v).solve(b)
        x_na = torch.full_like(b, float("nan"))
        x_na, i_na = ref.solve_noalloc(b, x_na)
        torch.cuda.synchronize()
        xr, xd, xn = (t.cpu().numpy() for t in (x_ref, x_def, x_na))
        print(f"{nx}x{ny} nrhs={nrhs}: noalloc omega {i_na.omega:.2e} (solve {i_ref.omega:.2e}), "
              f"bitwise equal {np.array_equal(xn, xr)}", flush=True)
        assert np.array_equal(xn, xr)
        assert i_na.omega == i_ref.omega and i_na.outer_iters == i_ref.outer_iters
        A = s.to_scipy()
        for c in range(nrhs):
            xc, dc, bc = np.atleast_2d(xn)[c], np.atleast_2d(xd)[c], np.atleast_2d(B)[c]
            assert np.abs(xc - dc).max() / np.abs(dc).max() <= 1e-8
            assert check.omega(A, xc, bc) <= 1e-12


def test_noalloc_refuses_gmres_ir(torch_cuda):
    torch = torch_cuda
    s = build_2d(16, 8, 0)
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    num = S.factor(torch.from_numpy(s.values).cuda(), prec="fp32")
    b = torch.from_numpy(s.b0[0].copy()).cuda()
    with pytest.raises(mf.MFError) as e:
        num.solve_noalloc(b, torch.empty_like(b))
    assert e.value.status == mf.MF_ERR_ARG
