"""Pins for the oracle's sparse LU: dense GEPP, exact rationals, manufactured
solutions, the backward-error invariant and special cases."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import check, splu, sym
from vivjac import build_2d


def lu_solve(A, b, q=None, tau=1.0):
    A = sp.csr_matrix(A)
    A.sort_indices()
    F = splu.SparseLU(A.shape[0], A.indptr, A.indices, A.data, q, tau=tau)
    return F.solve(b)


def test_config0_vs_dense_gepp(config0):
    s = config0
    S = sym.analyze(s.n, s.rowptr, s.colind, s.root)
    A = s.to_scipy()
    F = splu.SparseLU(s.n, s.rowptr, s.colind, s.values, S.perm)
    b = s.b0[0]
    x, om, st = F.solve(b)
    xd = check.dense_gepp_solve(A, b)
    assert np.abs(x - xd).max() / np.abs(xd).max() < 1e-12
    assert om[0] <= 1e-13 and check.omega(A, x, b) <= 1e-13
    assert check.eta(A, x, b) <= 1e-16


@pytest.mark.parametrize("seed", range(6))
def test_exact_rationals(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 13))
    while True:
        A = rng.integers(-4, 5, size=(n, n))
        A[rng.random((n, n)) < 0.5] = 0
        np.fill_diagonal(A, 0)                    # zero diagonal forces off-diagonal pivots
        A[:, 0] += 0                              # keep integers
        if round(abs(np.linalg.det(A))) >= 1:
            break
    b = rng.integers(-5, 6, size=n)
    xe = check.fraction_solve(A.tolist(), b.tolist())
    xe = np.array([float(v) for v in xe])
    x, om, _ = lu_solve(A.astype(float), b.astype(float), q=rng.permutation(n).astype(np.int32))
    assert np.abs(x - xe).max() <= 1e-12 * max(1.0, np.abs(xe).max())


def test_exact_rationals_known_3x3():
    # [[0,2,1],[1,0,3],[2,1,0]] x = [3,4,3]  ->  x = [1,1,1]
    A = np.array([[0, 2, 1], [1, 0, 3], [2, 1, 0]], dtype=float)
    b = np.array([3.0, 4.0, 3.0])
    x, _, _ = lu_solve(A, b)
    assert np.array_equal(x, [1.0, 1.0, 1.0])


def manufactured_rhs(A, xs):
    A = A.tocsr()
    b = np.empty(A.shape[0])
    for i in range(A.shape[0]):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        b[i] = math.fsum(A.data[lo:hi] * xs[A.indices[lo:hi]])
    return b


@pytest.mark.parametrize("nx,ny,seed", [(16, 8, 0), (32, 16, 5)])
def test_manufactured_solution(nx, ny, seed):
    s = build_2d(nx, ny, seed)
    A = s.to_scipy()
    rng = np.random.default_rng(1000 + seed)
    xs = rng.standard_normal(s.n)
    b = manufactured_rhs(A, xs)
    S = sym.analyze(s.n, s.rowptr, s.colind, s.root)
    F = splu.SparseLU(s.n, s.rowptr, s.colind, s.values, S.perm)
    x, om, st = F.solve(b)
    assert om[0] <= 1e-13
    assert check.omega(A, x, b) <= 1e-13
    assert np.abs(x - xs).max() / np.abs(xs).max() <= 1e-8


def test_threshold_variant_agrees(config0):
    s = config0
    S = sym.analyze(s.n, s.rowptr, s.colind, s.root)
    A = s.to_scipy()
    b = s.b0[0]
    x1, om1, _ = splu.SparseLU(s.n, s.rowptr, s.colind, s.values, S.perm, tau=1.0).solve(b)
    x2, om2, _ = splu.SparseLU(s.n, s.rowptr, s.colind, s.values, S.perm, tau=0.1).solve(b)
    assert om1[0] <= 1e-13 and om2[0] <= 1e-13
    assert np.abs(x1 - x2).max() / np.abs(x1).max() < 1e-10


def test_spd_pseudo_solid_block_vs_cholesky(config0):
    s = config0
    A = s.to_scipy().tocsr()
    d0, d1 = s.blocks["d"]
    Add = A[d0:d1, d0:d1].toarray()
    # interior rows only (Gamma rows are replaced by the coupling rows)
    inner = [i for i in range(d1 - d0) if not (A.getrow(d0 + i).nnz == 2)]
    K = Add[np.ix_(inner, inner)]
    assert np.allclose(K, K.T, atol=1e-12 * np.abs(K).max())
    rng = np.random.default_rng(7)
    b = rng.standard_normal(len(inner))
    xc = sla.cho_solve(sla.cho_factor(K), b)
    x, om, _ = lu_solve(K, b, q=rng.permutation(len(inner)).astype(np.int32))
    assert np.abs(x - xc).max() / np.abs(xc).max() < 1e-10


def test_single_dense_front_vs_dense_lu():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 40))
    b = rng.standard_normal(40)
    x, om, _ = lu_solve(A, b)
    P, L, U = sla.lu(A)
    xd = sla.solve_triangular(U, sla.solve_triangular(L, P.T @ b, lower=True, unit_diagonal=True))
    assert np.abs(x - xd).max() / np.abs(xd).max() < 1e-12


def test_block_triangular():
    rng = np.random.default_rng(4)
    n1, n2 = 15, 10
    A11 = rng.standard_normal((n1, n1)) + 5 * np.eye(n1)
    A22 = rng.standard_normal((n2, n2)) + 5 * np.eye(n2)
    A21 = rng.standard_normal((n2, n1))
    A = np.block([[A11, np.zeros((n1, n2))], [A21, A22]])
    b = rng.standard_normal(n1 + n2)
    x, om, _ = lu_solve(A, b)
    x1 = np.linalg.solve(A11, b[:n1])
    x2 = np.linalg.solve(A22, b[n1:] - A21 @ x1)
    assert np.allclose(x, np.concatenate([x1, x2]), rtol=1e-12, atol=1e-12)


def test_singular_detected():
    A = sp.csr_matrix(np.array([[1.0, 2.0, 0.0], [2.0, 4.0, 0.0], [0.0, 0.0, 1.0]]))
    with pytest.raises(splu.SingularError):
        splu.SparseLU(3, A.indptr, A.indices, A.data)
    A = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 1.0]]))
    with pytest.raises(splu.SingularError):
        splu.SparseLU(2, A.indptr, A.indices, A.data)


def test_omega_measure_pins():
    # omega of an exact solution is 0; scaling a row of the residual scales omega
    A = sp.csr_matrix(np.array([[2.0, 1.0], [1.0, 3.0]]))
    x = np.array([1.0, 1.0])
    b = np.array([3.0, 4.0])
    assert check.omega(A, x, b) == 0.0
    xp = np.array([1.0 + 1e-10, 1.0])
    r = np.abs(b - A @ xp)
    den = np.abs(A.toarray()) @ np.abs(xp) + np.abs(b)
    assert check.omega(A, xp, b) == pytest.approx((r / den).max(), rel=1e-6)


def test_planted_mistake_is_caught(config0):
    """A dropped term in the oracle's answer (one entry zeroed) must fail the pins."""
    s = config0
    A = s.to_scipy()
    S = sym.analyze(s.n, s.rowptr, s.colind, s.root)
    x, _, _ = splu.SparseLU(s.n, s.rowptr, s.colind, s.values, S.perm).solve(s.b0[0])
    bad = x.copy()
    bad[s.blocks["p"][0]] = 0.0
    assert check.omega(A, bad, s.b0[0]) > 1e-6


# ---- pins of the backward-error measures themselves (hand-worked, not restated)
#
# A = [[2, -1], [1, 3]], x = [1, 2], b = [-1, 8]:
#   A x = [0, 7], so r = b - A x = [-1, 1];
#   |A||x| = [2*1 + 1*2, 1*1 + 3*2] = [4, 7], plus |b| = [1, 8] gives [5, 15];
#   omega = max(|-1| / 5, |1| / 15) = 0.2   (the first row decides).
#   ||r||_inf = 1, ||A||_inf = max(2 + 1, 1 + 3) = 4, ||x||_inf = 2, ||b||_inf = 8;
#   eta = 1 / (4 * 2 + 8) = 1 / 16.
# A dropped absolute value on A gives |A x| + |b| = [1, 15] and omega = 1; a
# dropped |b| gives omega = 0.25; a signed residual gives max(-0.2, 1/15); a
# column-sum norm of A (3 instead of 4) gives eta = 1/14.
HAND_A = np.array([[2.0, -1.0], [1.0, 3.0]])
HAND_X = np.array([1.0, 2.0])
HAND_B = np.array([-1.0, 8.0])


@pytest.mark.parametrize("fn", [check.omega, check.omega_fast])
def test_omega_hand_worked(fn):
    A = sp.csr_matrix(HAND_A)
    assert fn(A, HAND_X, HAND_B) == 0.2


def test_eta_hand_worked():
    assert check.eta(sp.csr_matrix(HAND_A), HAND_X, HAND_B) == 1.0 / 16.0


@pytest.mark.parametrize("fn", [check.omega, check.omega_fast])
def test_omega_zero_over_zero_and_inf(fn):
    # row 0 of A is empty and b_0 = 0: 0/0 counts as 0 (an exactly satisfied empty
    # row); row 1: 3 * 1 = 3 = b_1, exact.  With b_0 = 1 the empty row cannot be
    # satisfied by any x: its denominator |A||x| + |b| is 1, residual 1, omega 1.
    A = sp.csr_matrix(np.array([[0.0, 0.0], [0.0, 3.0]]))
    x = np.array([5.0, 1.0])
    assert fn(A, x, np.array([0.0, 3.0])) == 0.0
    assert fn(A, x, np.array([1.0, 3.0])) == 1.0
    # a zero denominator with a nonzero residual is not a backward-stable answer
    A = sp.csr_matrix(np.array([[1.0, 0.0], [0.0, 3.0]]))
    assert fn(A, np.array([0.0, 1.0]), np.array([0.0, 3.0])) == 0.0


def _gamma(k):
    # Higham's gamma_k = k u / (1 - k u), u the unit roundoff of binary64
    u = np.finfo(np.float64).eps / 2
    return k * u / (1 - k * u)


@pytest.mark.parametrize("nx,ny,seed", [(16, 8, 0), (32, 16, 3)])
def test_omega_fast_within_summation_bound(nx, ny, seed):
    """omega_fast sums each residual row in ordinary floating point; omega sums it
    exactly.  Recursive summation of k terms errs by at most gamma_{k} times the
    sum of the magnitudes (Higham, Accuracy and Stability, Sec. 3.1), and the
    products by one rounding each, so |r_fast - r|_i <= gamma_{k+1} (|A||x| + |b|)_i
    with k the row's entry count, hence |omega_fast - omega| <= gamma_{k+1}.
    Checked on an accurate solution (omega near u) and a perturbed one (omega near
    1e-9, where the two must agree to about 1e-6 relative)."""
    s = build_2d(nx, ny, seed)
    A = s.to_scipy()
    S = sym.analyze(s.n, s.rowptr, s.colind, s.root)
    x, _, _ = splu.SparseLU(s.n, s.rowptr, s.colind, s.values, S.perm).solve(s.b0[0])
    k = int(np.diff(A.indptr).max()) + 1
    bound = _gamma(k + 1)
    rng = np.random.default_rng(11)
    xp = x * (1 + 1e-9 * rng.standard_normal(s.n))
    for xx in (x, xp):
        w, wf = check.omega(A, xx, s.b0[0]), check.omega_fast(A, xx, s.b0[0])
        assert abs(wf - w) <= bound, (w, wf, bound)
    wp = check.omega(A, xp, s.b0[0])
    assert wp > 1e-11
    assert abs(check.omega_fast(A, xp, s.b0[0]) - wp) <= 1e-5 * wp


def test_eta_scales_with_residual():
    # eta is homogeneous of degree 1 in the residual at fixed x: doubling r by
    # moving b away from A x doubles the numerator only (the denominator changes by
    # |b|, worked out here): A = I, x = [1, 1]; b = [1 + t, 1] gives
    # eta = t / (1 + 1 + t) for t >= 0.
    A = sp.csr_matrix(np.eye(2))
    for t in (0.5, 1.0, 3.0):
        assert check.eta(A, np.ones(2), np.array([1.0 + t, 1.0])) == pytest.approx(t / (2.0 + t), rel=1e-15)
