"""GPU parity of the full ALE Newton system (residual, Jacobian with its
shape-derivative blocks, and the Newton loop) against the CPU oracle.

Bar: residual and Jacobian entries agree with the oracle's to 1e-11 of their
row's largest magnitude (the two sum the same element terms in different
orders; the oracle's derivatives are complex-step exact); Newton iterates agree
to 1e-8 relative and converge quadratically to max |NL| <= 1e-10."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

from oracle import ale
from vivjac.ale2d import build_ale_2d

pytestmark = pytest.mark.gpu

ROW_TOL = 1e-11


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _row_scaled_error(prob, got, want):
    rows = np.repeat(np.arange(prob.n), np.diff(prob.rowptr))
    scale = np.zeros(prob.n)
    np.maximum.at(scale, rows, np.abs(want))
    return float(np.max(np.abs(got - want) / np.maximum(scale[rows], 1e-300)))


@pytest.mark.parametrize("nx,state", [(16, "initial"), (16, "perturbed"), (32, "perturbed"), (40, "perturbed")])
def test_assembly_matches_oracle(torch_cuda, nx, state):
    from paper_2609_31477_amd.ale import Assembly
    torch = torch_cuda
    prob = build_ale_2d(nx, nx // 2, 2)
    U = prob.initial_guess() if state == "initial" else prob.perturbed_state(7)
    A = Assembly(prob)
    Ud = torch.from_numpy(U).cuda()
    R = torch.empty_like(Ud)
    vals = A.jacobian(Ud, R=R)
    R2 = A.residual(Ud)
    torch.cuda.synchronize()
    got_v, got_r, got_r2 = vals.cpu().numpy(), R.cpu().numpy(), R2.cpu().numpy()
    want_v = ale.pattern_values(prob, ale.jacobian(prob, U))
    want_r = ale.residual(prob, U)
    ev = _row_scaled_error(prob, got_v, want_v)
    er = float(np.max(np.abs(got_r - want_r)) / np.abs(want_r).max())
    print(f"{nx} {state}: n={prob.n} nnz={prob.nnz} jacobian row-scaled err={ev:.2e} residual err={er:.2e} "
          f"device bytes={A.device_bytes}", flush=True)
    assert ev <= ROW_TOL
    assert er <= 1e-12
    assert np.array_equal(got_r, got_r2)              # the residual alone sums the same terms in the same order
    A.release()


def test_newton_loop_matches_oracle(torch_cuda):
    """The GPU Newton loop (GPU assembly, libmf factor + solve in FP64) against
    the oracle's (complex-step Jacobian, sparse direct solve)."""
    from paper_2609_31477_amd.ale import newton
    prob = build_ale_2d(24, 12, 4)
    U, norms, infos = newton(prob, iters=5, tol=1e-11)
    Ug = U.cpu().numpy()
    # oracle iterates
    Uo = prob.initial_guess()
    onorms = []
    for _ in range(len(norms)):
        Ro = ale.residual(prob, Uo)
        onorms.append(np.abs(Ro).max())
        if len(onorms) == len(norms):
            break
        Uo = Uo - sla.spsolve(ale.jacobian(prob, Uo).tocsc(), Ro)
    print("gpu", ["%.2e" % v for v in norms], "oracle", ["%.2e" % v for v in onorms], flush=True)
    assert norms[-1] <= 1e-10
    for a, b in zip(norms[1:], norms[2:]):
        if b > 1e-10:
            assert b <= 100.0 * a * a                     # quadratic convergence
    assert np.abs(Ug - Uo).max() <= 1e-8 * np.abs(Uo).max()
    for g, o in zip(norms[:3], onorms[:3]):
        assert g == pytest.approx(o, rel=1e-6, abs=1e-12)


def test_full_size_jacobian_matches_oracle(torch_cuda):
    """256x128 cells (n = 350,270): every Jacobian entry and residual row at a
    moved state against the oracle."""
    from paper_2609_31477_amd.ale import Assembly
    torch = torch_cuda
    prob = build_ale_2d(256, 128, 1)
    U = prob.perturbed_state(9)
    A = Assembly(prob)
    Ud = torch.from_numpy(U).cuda()
    R = torch.empty_like(Ud)
    vals = A.jacobian(Ud, R=R)
    torch.cuda.synchronize()
    want_v = ale.pattern_values(prob, ale.jacobian(prob, U))
    want_r = ale.residual(prob, U)
    ev = _row_scaled_error(prob, vals.cpu().numpy(), want_v)
    er = float(np.max(np.abs(R.cpu().numpy() - want_r)) / np.abs(want_r).max())
    print(f"256x128: jacobian row-scaled err={ev:.2e} residual err={er:.2e}", flush=True)
    assert ev <= ROW_TOL and er <= 1e-12
    A.release()


def test_jacobian_solve_is_the_newton_direction(torch_cuda):
    """One Newton correction from the GPU Jacobian, checked on the CPU: the
    computed dU solves J dU = -NL with omega <= 1e-12 against the oracle's J."""
    from oracle import check
    from paper_2609_31477_amd.ale import Assembly
    import paper_2609_31477_amd as mf
    torch = torch_cuda
    prob = build_ale_2d(32, 16, 5)
    U = prob.perturbed_state(2, scale=0.5)
    A = Assembly(prob)
    Ud = torch.from_numpy(U).cuda()
    R = torch.empty_like(Ud)
    vals = A.jacobian(Ud, R=R)
    S = mf.Symbolic(prob.n, prob.rowptr, prob.colind, prob.root)
    num = S.factor(vals, target_omega=1e-13)
    dU, info = num.solve(-R)
    J = sp.csr_matrix((ale.pattern_values(prob, ale.jacobian(prob, U)), prob.colind, prob.rowptr),
                      shape=(prob.n, prob.n))
    om = check.omega(J, dU.cpu().numpy(), -ale.residual(prob, U))
    print(f"omega against the oracle's J = {om:.2e} (library omega {info.omega:.2e})", flush=True)
    assert om <= 1e-12
    num.release()
    A.release()
