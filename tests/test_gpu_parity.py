"""GPU parity: the HIP multifrontal path (through the C ABI) against the CPU oracle.

Bar (plain FP64 path): relative solution error <= 1e-8 against the oracle and a
componentwise backward error omega <= 1e-12 (computed here on the CPU by the
oracle's own residual), with at most 2 FP64 refinement steps."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2609_31477_amd as mf
from oracle import check, splu, sym as osym
from vivjac import build_2d, newton_rhs, newton_values

pytestmark = pytest.mark.gpu

REL_TOL = 1e-8
OMEGA_TOL = 1e-12


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def oracle_solve(n, rp, ci, vals, root, B):
    S = osym.analyze(n, rp, ci, root)
    F = splu.SparseLU(n, rp, ci, vals, S.perm, tau=0.1 if n > 50000 else 1.0)
    X, om, _ = F.solve(B)
    return X


def gpu_solve(torch, n, rp, ci, vals, root, B, leaf_max=64, **opts):
    dev = torch.device("cuda:0")
    S = mf.Symbolic(n, rp, ci, root, leaf_max=leaf_max)
    num = S.factor(torch.from_numpy(np.ascontiguousarray(vals)).to(dev), **opts)
    x, info = num.solve(torch.from_numpy(np.ascontiguousarray(B)).to(dev))
    torch.cuda.synchronize()
    return x.cpu().numpy(), info, num


def assert_parity(A, X, Xo, B, rel_tol=REL_TOL, omega_tol=OMEGA_TOL):
    X = np.atleast_2d(X)
    Xo = np.atleast_2d(Xo)
    B = np.atleast_2d(B)
    for c in range(X.shape[0]):
        rel = np.abs(X[c] - Xo[c]).max() / np.abs(Xo[c]).max()
        om = check.omega(A, X[c], B[c]) if A.shape[0] <= 20000 else check.omega_fast(A, X[c], B[c])
        print(f"rhs {c}: rel_err={rel:.3e} omega={om:.3e}", flush=True)
        assert rel <= rel_tol
        assert om <= omega_tol


def test_config0_fp64(torch_cuda):
    s = build_2d(16, 8, 0)
    B = s.b0[0]
    X, info, num = gpu_solve(torch_cuda, s.n, s.rowptr, s.colind, s.values, s.root, B)
    fi = num.info()
    print(f"delayed={fi.delayed_pivots} max_front={fi.max_front} root={fi.root_order} "
          f"omega0={info.omega0:.3e} omega={info.omega:.3e} steps={info.outer_iters}", flush=True)
    Xo = oracle_solve(s.n, s.rowptr, s.colind, s.values, s.root, B)
    assert_parity(s.to_scipy(), X, Xo, B)
    assert info.outer_iters <= 2


def random_saddle(rng, n, density=0.1, zero_diag_frac=0.3):
    """Random unsymmetric system with a zero-diagonal block (forces delayed pivots)."""
    A = sp.random(n, n, density=density, random_state=np.random.RandomState(int(rng.integers(1 << 30))), format="csr")
    A = A + sp.eye(n) * 2.0
    A = A.tolil()
    nz = rng.permutation(n)[: int(zero_diag_frac * n)]
    for i in nz:
        A[i, i] = 0.0
        j = int(rng.integers(n))
        if j != i:
            A[i, j] = 1.0 + rng.random()
            A[j, i] = 1.0 + rng.random()
    A = A.tocsr()
    A.sort_indices()
    return A


@pytest.mark.parametrize("seed,n,leaf,nrhs", [(0, 30, 4, 1), (1, 120, 8, 3), (2, 400, 16, 2), (3, 1000, 64, 1),
                                              (4, 257, 1, 1), (5, 777, 32, 5)])
def test_random_forced_delays(torch_cuda, seed, n, leaf, nrhs):
    rng = np.random.default_rng(seed)
    A = random_saddle(rng, n, density=min(0.2, 8.0 / n))
    if abs(np.linalg.det(A.toarray())) < 1e-8:
        pytest.skip("singular draw")
    B = rng.standard_normal((nrhs, n))
    root = [] if seed % 2 else [n - 1]
    X, info, num = gpu_solve(torch_cuda, n, A.indptr, A.indices, A.data, root, B, leaf_max=leaf)
    Xo = np.linalg.solve(A.toarray(), B.T).T
    print(f"n={n} delayed={num.info().delayed_pivots}", flush=True)
    assert_parity(A, X, Xo, B)


def test_multi_rhs_and_determinism(torch_cuda):
    s = build_2d(32, 16, 2, nrhs=8)
    B = s.b0
    X1, i1, _ = gpu_solve(torch_cuda, s.n, s.rowptr, s.colind, s.values, s.root, B)
    X2, i2, _ = gpu_solve(torch_cuda, s.n, s.rowptr, s.colind, s.values, s.root, B)
    assert np.array_equal(X1, X2), "same input must give a bitwise-equal solution"
    Xo = oracle_solve(s.n, s.rowptr, s.colind, s.values, s.root, B)
    assert_parity(s.to_scipy(), X1, Xo, B)


def test_newton_steps_reuse_symbolic(torch_cuda):
    torch = torch_cuda
    s = build_2d(32, 16, 1)
    dev = torch.device("cuda:0")
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    Os = osym.analyze(s.n, s.rowptr, s.colind, s.root)
    num = None
    for t in range(3):
        v = newton_values(s, t)
        b = newton_rhs(s, t)[0]
        num = S.factor(torch.from_numpy(v).to(dev), numeric=num)
        x, info = num.solve(torch.from_numpy(b).to(dev))
        xh = x.cpu().numpy()
        xo, _, _ = splu.SparseLU(s.n, s.rowptr, s.colind, v, Os.perm).solve(b)
        assert_parity(s.to_scipy(v), xh, xo, b)


def test_64x32_fp64(torch_cuda):
    s = build_2d(64, 32, 0)
    B = s.b0[0]
    X, info, num = gpu_solve(torch_cuda, s.n, s.rowptr, s.colind, s.values, s.root, B)
    Xo = oracle_solve(s.n, s.rowptr, s.colind, s.values, s.root, B)
    print(f"64x32: delayed={num.info().delayed_pivots} steps={info.outer_iters}", flush=True)
    assert_parity(s.to_scipy(), X, Xo, B)


def test_singular_reported(torch_cuda):
    torch = torch_cuda
    A = sp.csr_matrix(np.array([[1.0, 2.0, 0.0], [2.0, 4.0, 0.0], [0.0, 0.0, 1.0]]))
    S = mf.Symbolic(3, A.indptr, A.indices, [])
    with pytest.raises(mf.MFError) as e:
        S.factor(torch.from_numpy(A.data.copy()).cuda())
    assert e.value.status == mf.MF_ERR_SINGULAR


def test_empty_system(torch_cuda):
    torch = torch_cuda
    S = mf.Symbolic(0, np.zeros(1, np.int64), np.zeros(0, np.int32), [])
    num = S.factor(torch.zeros(0, dtype=torch.float64, device="cuda"))
    x, info = num.solve(torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert x.numel() == 0


MIXED_OMEGA = 1e-10


@pytest.mark.parametrize("prec,nx,ny,seed,nrhs", [("fp32", 16, 8, 0, 1), ("fp32", 32, 16, 4, 3), ("fp32", 64, 32, 0, 1),
                                                   ("bf16", 16, 8, 0, 1), ("bf16", 32, 16, 4, 2),
                                                   ("bf16", 64, 32, 0, 1)])
def test_mixed_gmres_ir(torch_cuda, prec, nx, ny, seed, nrhs):
    """FP32 non-root fronts (Schur updates in FP32, or BF16 operands with FP32
    accumulation), FP64 root, FP64 GMRES-IR: omega <= 1e-10."""
    s = build_2d(nx, ny, seed, nrhs=nrhs)
    B = s.b0
    X, info, num = gpu_solve(torch_cuda, s.n, s.rowptr, s.colind, s.values, s.root, B,
                             prec=prec, target_omega=MIXED_OMEGA, max_outer=20)
    Xo = oracle_solve(s.n, s.rowptr, s.colind, s.values, s.root, B)
    A = s.to_scipy()
    for c in range(B.shape[0]):
        om = check.omega(A, X[c], B[c])
        rel = np.abs(X[c] - Xo[c]).max() / np.abs(Xo[c]).max()
        print(f"{prec} {nx}x{ny} rhs {c}: omega={om:.2e} rel={rel:.2e} omega0={info.omega0:.2e} "
              f"outer={info.outer_iters} inner={info.inner_iters}", flush=True)
        assert om <= MIXED_OMEGA
        assert rel <= 1e-6
    assert num.info().root_order >= 2


def test_gmres_ir_with_fp64_factors_one_step(torch_cuda):
    """With FP64 factors GMRES-IR needs at most one outer step to reach 1e-12."""
    s = build_2d(32, 16, 7)
    X, info, _ = gpu_solve(torch_cuda, s.n, s.rowptr, s.colind, s.values, s.root, s.b0[0], refine=2)
    assert info.outer_iters <= 1
    assert check.omega(s.to_scipy(), X, s.b0[0]) <= OMEGA_TOL


@pytest.mark.parametrize("prec,nx,ny,seed", [("fp64", 64, 32, 0), ("fp32", 32, 16, 3)])
def test_pivot_rule(torch_cuda, prec, nx, ny, seed):
    """Threshold partial pivoting inside every front (u = 0.01; partial pivoting,
    u = 1, in the FP64 root): each eliminated column's pivot is the largest
    remaining fully summed entry, so its multipliers are at most 1 in magnitude on
    the fully summed rows and at most 1/u on the contribution rows."""
    torch = torch_cuda
    s = build_2d(nx, ny, seed)
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    num = S.factor(torch.from_numpy(s.values).to("cuda:0"), prec=prec)
    torch.cuda.synchronize()
    v = S.export()
    worst_fs = worst_cb = 0.0
    for f in range(v.nfronts):
        meta, F, _ = num.debug_front(f)
        m, P, k = meta["m"], meta["P"], meta["k"]
        root = v.front_parent[f] < 0
        u = 1.0 if root else 0.01
        # multipliers are formed as a * (1/pivot): within a few units in the last
        # place of the front's precision of the exact ratio
        eps = np.finfo(np.float32 if meta["prec"] == 1 else np.float64).eps
        for t in range(k):
            fs = np.abs(F[t + 1:P, t]).max(initial=0.0)
            cb = np.abs(F[P:m, t]).max(initial=0.0)
            worst_fs = max(worst_fs, fs)
            worst_cb = max(worst_cb, cb * u)
            assert fs <= 1.0 + 4 * eps, (f, t, fs)
            assert cb <= (1.0 + 4 * eps) / u, (f, t, cb)
    print(f"{prec} {nx}x{ny}: max FS multiplier {worst_fs:.3f}, max u*CB multiplier {worst_cb:.3f}", flush=True)


@pytest.mark.parametrize("scale", [0, 1, 3])
def test_equilibration_parity(torch_cuda, scale):
    """Ruiz equilibration (power-of-two row and column factors, values only) changes
    the factors but not the solution: every sweep count meets the FP64 bar against the
    oracle on the original system."""
    s = build_2d(32, 16, 5)
    B = s.b0[0]
    X, info, num = gpu_solve(torch_cuda, s.n, s.rowptr, s.colind, s.values, s.root, B, scale=scale)
    Xo = oracle_solve(s.n, s.rowptr, s.colind, s.values, s.root, B)
    print(f"scale={scale}: delayed={num.info().delayed_pivots} omega0={info.omega0:.2e} "
          f"steps={info.outer_iters}", flush=True)
    assert_parity(s.to_scipy(), X, Xo, B)
    assert info.outer_iters <= 2


def _gamma(k):
    u = np.finfo(np.float64).eps / 2
    return k * u / (1 - k * u)


def test_solve_info_eta_and_delays(torch_cuda):
    """The solve reports the normwise backward error eta of its final x (device
    residual with ordinary summation) within the summation error bound of the
    oracle's exact-residual eta, and the delayed-pivot count of its factors."""
    s = build_2d(32, 16, 6)
    X, info, num = gpu_solve(torch_cuda, s.n, s.rowptr, s.colind, s.values, s.root, s.b0[0])
    A = s.to_scipy()
    e = check.eta(A, X, s.b0[0])
    k = int(np.diff(A.indptr).max()) + 1
    print(f"eta device {info.eta:.3e} oracle {e:.3e}; delayed {info.delayed_pivots}", flush=True)
    assert abs(info.eta - e) <= _gamma(k + 1)
    assert info.delayed_pivots == num.info().delayed_pivots


def test_nonfinite_values_refused_up_front(torch_cuda):
    torch = torch_cuda
    s = build_2d(16, 8, 0)
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    for bad in (np.nan, np.inf):
        v = s.values.copy()
        v[100] = bad
        with pytest.raises(mf.MFError) as e:
            S.factor(torch.from_numpy(v).cuda())
        assert e.value.status == mf.MF_ERR_ARG
        assert "values_dev[100]" in str(e.value)


def test_fp64_fallback_when_gmres_ir_stalls(torch_cuda):
    """GMRES-IR on BF16 factors limited to one inner and one outer step cannot
    reach 1e-12; with the fallback on, the handle is refactored in FP64 and the
    solve meets the target (the FP64 bar against the oracle); with it off, the
    solve reports MF_ERR_NOT_CONVERGED."""
    torch = torch_cuda
    s = build_2d(32, 16, 8)
    dev = torch.device("cuda:0")
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    v = torch.from_numpy(s.values).to(dev)
    b = torch.from_numpy(s.b0[0].copy()).to(dev)
    num = S.factor(v, prec="bf16", target_omega=1e-12, gmres_m=1, max_outer=1, fallback=0)
    with pytest.raises(mf.MFError) as e:
        num.solve(b)
    assert e.value.status == mf.MF_ERR_NOT_CONVERGED
    num = S.factor(v, prec="bf16", target_omega=1e-12, gmres_m=1, max_outer=1, fallback=1)
    x, info = num.solve(b)
    torch.cuda.synchronize()
    print(f"fallback={info.fp64_fallback} omega={info.omega:.2e} outer={info.outer_iters}", flush=True)
    assert info.fp64_fallback == 1
    Xo = oracle_solve(s.n, s.rowptr, s.colind, s.values, s.root, s.b0[0])
    assert_parity(s.to_scipy(), x.cpu().numpy(), Xo, s.b0[0])


@pytest.mark.parametrize("prec,nx,ny,seed,nrhs", [("fp64", 16, 8, 0, 1), ("fp64", 32, 16, 3, 3),
                                                   ("fp32", 64, 32, 0, 2), ("fp64", 64, 32, 2, 9)])
def test_persistent_sweeps_match_level_sweeps(torch_cuda, prec, nx, ny, seed, nrhs):
    """The persistent sweeps (one launch per direction over the task list) and
    the level-by-level sweeps apply the same factors: without refinement their
    solutions agree to rounding (relative 1e-10), and each meets the FP64 bar
    against the oracle after refinement (nine right-hand sides span two launch
    chunks of eight)."""
    torch = torch_cuda
    s = build_2d(nx, ny, seed, nrhs=nrhs)
    B = s.b0
    dev = torch.device("cuda:0")
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    v = torch.from_numpy(s.values).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(B)).to(dev)
    raw = {}
    for sw in (0, 1):
        num = S.factor(v, prec=prec, refine=0, sweep=sw)
        x, _ = num.solve(b)
        raw[sw] = x.cpu().numpy()
    d = np.abs(raw[0] - raw[1]).max() / np.abs(raw[0]).max()
    print(f"{prec} {nx}x{ny} nrhs={nrhs}: persistent vs level sweeps {d:.2e}", flush=True)
    assert d <= 1e-10
    Xo = oracle_solve(s.n, s.rowptr, s.colind, s.values, s.root, B)
    target = 1e-12 if prec == "fp64" else 1e-10
    for sw in (0, 1):
        num = S.factor(v, prec=prec, sweep=sw, target_omega=target)
        x, info = num.solve(b)
        assert_parity(s.to_scipy(), x.cpu().numpy(), Xo, B, omega_tol=target,
                      rel_tol=1e-8 if prec == "fp64" else 1e-6)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec,nrhs", [("fp64", 1), ("fp32", 3), ("fp64", 9)])
def test_persistent_sweeps_match_level_sweeps_256x128(torch_cuda, prec, nrhs):
    """At 256x128 the upper tree (levels of at most 64 fronts, fronts up to order
    1,464) runs in the persistent sweeps with its large fronts split over many
    work-groups: without refinement the solution agrees with the level-by-level
    sweeps to rounding (relative 1e-10), and with refinement each meets its
    backward-error target (recomputed on the CPU)."""
    torch = torch_cuda
    s = build_2d(256, 128, 1, nrhs=nrhs)
    dev = torch.device("cuda:0")
    S = mf.Symbolic(s.n, s.rowptr, s.colind, s.root)
    v = torch.from_numpy(s.values).to(dev)
    B = s.b0 if nrhs > 1 else s.b0[0]
    b = torch.from_numpy(np.ascontiguousarray(B)).to(dev)
    raw = {}
    for sw in (0, 1):
        num = S.factor(v, prec=prec, refine=0, sweep=sw)
        x, _ = num.solve(b)
        raw[sw] = x.cpu().numpy()
        num.release()
    d = np.abs(raw[0] - raw[1]).max() / np.abs(raw[0]).max()
    print(f"256x128 {prec} nrhs={nrhs}: persistent vs level sweeps {d:.2e}", flush=True)
    assert d <= 1e-10
    target = 1e-12 if prec == "fp64" else 1e-10
    A = s.to_scipy()
    num = S.factor(v, prec=prec, target_omega=target)
    x, info = num.solve(b)
    X = np.atleast_2d(x.cpu().numpy())
    for c in range(nrhs):
        assert check.omega_fast(A, X[c], np.atleast_2d(B)[c]) <= target
    num.release()


@pytest.mark.parametrize("prec,variant", [
    ("fp64", dict(position="p1")),
    ("fp64", dict(lame="radial")),
    ("fp64", dict(scheme="bdf2", hole="circle")),
    ("fp64", dict(coupling="accumulator")),
    ("fp32", dict(position="p1", lame="radial", scheme="bdf2", hole="circle", coupling="accumulator")),
])
def test_generator_variants(torch_cuda, prec, variant):
    """The paper-faithful generator variants (linear position, radial Lame law,
    BDF2, circular hole, force-accumulator root) against the oracle."""
    s = build_2d(32, 16, 11, **variant)
    B = s.b0[0]
    target = OMEGA_TOL if prec == "fp64" else MIXED_OMEGA
    X, info, num = gpu_solve(torch_cuda, s.n, s.rowptr, s.colind, s.values, s.root, B, prec=prec,
                             target_omega=target)
    fi = num.info()
    print(f"{prec} {variant}: n={s.n} root={fi.root_order} delayed={fi.delayed_pivots} "
          f"omega={info.omega:.2e} outer={info.outer_iters} inner={info.inner_iters}", flush=True)
    Xo = oracle_solve(s.n, s.rowptr, s.colind, s.values, s.root, B)
    assert_parity(s.to_scipy(), X, Xo, B, omega_tol=target, rel_tol=1e-8 if prec == "fp64" else 1e-6)
    assert fi.root_order >= len(s.root)
