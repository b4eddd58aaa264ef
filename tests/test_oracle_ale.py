"""Pins of the ALE residual/Jacobian oracle (CPU only).

The Jacobian is pinned against finite differences of the residual and by the
quadratic convergence of Newton's method; the residual is pinned by closed
forms on single elements (mass, divergence of an affine field, a uniform
dilation of the pseudo-solid, the multiplier's total force) and by the paper's
worked shape derivative of the continuity integral (Sec. 3.2)."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import ale
from vivjac.ale2d import build_ale_2d


@pytest.fixture(scope="module")
def prob():
    return build_ale_2d(16, 8, 0)


def test_jacobian_matches_central_differences(prob):
    U = prob.perturbed_state(3)
    A = ale.jacobian(prob, U)
    vals = ale.pattern_values(prob, A)          # every entry inside the pattern
    assert vals.size == prob.nnz
    rng = np.random.default_rng(1)
    for _ in range(3):
        d = rng.standard_normal(prob.n)
        h = 1e-6
        fd = (ale.residual(prob, U + h * d) - ale.residual(prob, U - h * d)) / (2 * h)
        Ad = A @ d
        assert np.abs(fd - Ad).max() <= 1e-8 * np.abs(Ad).max()


def test_shape_derivative_blocks_are_present(prob):
    """A_ux, A_px and A_lx (Sec. 3.2) are nonzero at a moved mesh."""
    U = prob.perturbed_state(4)
    A = ale.jacobian(prob, U).tocsr()
    b = prob.blocks
    for r, c in (("u", "x"), ("p", "x"), ("lam", "x")):
        blk = A[b[r][0]:b[r][1], b[c][0]:b[c][1]]
        assert abs(blk).max() > 1e-3, (r, c)
    assert abs(A[b["p"][0]:b["p"][1], b["p"][0]:b["p"][1]]).max() == 0.0   # zero pressure block


def test_newton_converges_quadratically(prob):
    U = prob.initial_guess()
    norms = []
    for _ in range(5):
        R = ale.residual(prob, U)
        norms.append(np.abs(R).max())
        if norms[-1] < 1e-12:
            break
        U = U - sla.spsolve(ale.jacobian(prob, U).tocsc(), R)
    print(["%.2e" % v for v in norms])
    assert norms[-1] < 1e-11
    # e_{m+1} <= C e_m^2 over the steps before rounding takes over
    for a, b in zip(norms[1:], norms[2:]):
        if b > 1e-10:
            assert b <= 100.0 * a * a


def _area(P):
    e1, e2 = P[1] - P[0], P[2] - P[0]
    return 0.5 * abs(e1[0] * e2[1] - e1[1] * e2[0])


def _single(xv):
    return np.asarray(xv, dtype=np.float64)[None]


def test_volume_mass_and_area():
    """u - u_prev = dt e_x with u constant, p = 0, mesh at rest: the u_x rows of a
    triangle sum to its current area (sum of the P2 basis integrals)."""
    xv = _single([[0.3, 0.1], [1.4, 0.2], [0.5, 1.3]])
    area = 0.5 * abs((xv[0, 1, 0] - xv[0, 0, 0]) * (xv[0, 2, 1] - xv[0, 0, 1])
                     - (xv[0, 2, 0] - xv[0, 0, 0]) * (xv[0, 1, 1] - xv[0, 0, 1]))
    dt = 0.01
    un = np.zeros((1, 6, 2))
    u = un + np.array([dt, 0.0])
    Ru, Rp = ale.volume_local(np.zeros((1, 3)), u, un, xv, xv, nu=0.3, dt=dt)
    assert Ru[0, :, 0].sum() == pytest.approx(area, rel=1e-14)
    assert np.abs(Ru[0, :, 1]).max() < 1e-15
    assert np.abs(Ru[0, :3, 0]).max() < 1e-15                # vertex P2 functions integrate to 0
    assert Ru[0, 3:, 0] == pytest.approx(np.full(3, area / 3), rel=1e-13)
    assert np.abs(Rp).max() < 1e-15


def test_divergence_of_affine_field():
    """u = B x (nodal values of an affine field on the current triangle): the
    pressure rows are -div(u) int L_k = -tr(B) |K| / 3."""
    xv = _single([[0.0, 0.0], [1.0, 0.2], [0.1, 0.9]])
    nodes = np.concatenate([xv[0], 0.5 * (xv[0] + np.roll(xv[0], -1, axis=0))])   # vertices, then (0,1),(1,2),(2,0)
    B = np.array([[0.7, -0.3], [0.4, 1.1]])
    u = (nodes @ B.T)[None]
    area = _area(xv[0])
    _, Rp = ale.volume_local(np.zeros((1, 3)), u, u, xv, xv, nu=0.1, dt=1.0)
    assert Rp[0] == pytest.approx(np.full(3, -np.trace(B) * area / 3), rel=1e-13)


def test_paper_continuity_shape_derivative():
    """Sec. 3.2: the variation of int_K q div u under a mesh variation dx is
    int q (-tr(grad u G) + div u tr G) det J, G = grad_x dx (the derivative of
    grad_x u is -grad_x u G, of det J is det J tr G).  The oracle's complex-step
    derivative of its pressure rows matches this closed form."""
    rng = np.random.default_rng(5)
    xv = _single([[0.0, 0.0], [1.1, 0.1], [0.2, 0.8]])
    u = rng.standard_normal((1, 6, 2))
    dx = rng.standard_normal((1, 3, 2))
    h = 1e-30
    _, Rp = ale.volume_local(np.zeros((1, 3)), u.astype(complex), u, xv + 1j * h * dx, xv, nu=0.0, dt=1.0)
    got = Rp.imag[0] / h
    # closed form with its own quadrature (Gauss 6x6 collapsed onto the triangle)
    g, w = np.polynomial.legendre.leggauss(6)
    g, w = 0.5 * (g + 1), 0.5 * w
    want = np.zeros(3)
    dL = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    J = xv[0].T @ dL
    Jinv = np.linalg.inv(J)
    detJ = np.linalg.det(J)
    G = (dx[0].T @ dL) @ Jinv                                  # grad_x dx (constant)
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            xi, eta = a, b * (1 - a)
            wt = wa * wb * (1 - a)
            Lq = np.array([1 - xi - eta, xi, eta])
            grads = [(4 * Lq[v] - 1) * dL[v] for v in range(3)]
            grads += [4 * (Lq[j] * dL[i] + Lq[i] * dL[j]) for i, j in ((0, 1), (1, 2), (2, 0))]
            gu = sum(np.outer(u[0, i], grads[i] @ Jinv) for i in range(6))     # d u_c / d x_a
            div = np.trace(gu)
            want += wt * (-Lq) * (-np.trace(gu @ G) + div * np.trace(G)) * detJ
    assert got == pytest.approx(want, rel=1e-12, abs=1e-14)


def test_pseudo_solid_dilation_and_translation():
    """x = (1 + e) X: eps = e I, sigma = 4 mu e I, so the rows are 4 e mu |K| grad L_v;
    a translation gives no stress."""
    Xv = _single([[0.2, 0.3], [1.0, 0.4], [0.5, 1.2]])
    area = _area(Xv[0])
    lam = np.array([1.0 / area])
    e = 0.01
    R = ale.solid_local((1 + e) * Xv, Xv, lam)[0]
    dL = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    gradL = dL @ np.linalg.inv(Xv[0].T @ dL)
    assert R == pytest.approx(4 * e * gradL, rel=1e-12, abs=1e-15)
    assert np.abs(ale.solid_local(Xv + np.array([0.3, -0.2]), Xv, lam)).max() < 1e-14


def test_multiplier_total_force(prob):
    """lambda = (1, -2) on every Gamma node, mesh at rest: the s rows read
    k s + perimeter * lambda (the force of eq. lambda_coupling)."""
    U = prob.initial_guess()
    U[prob.lam_dof[prob.lam_dof[:, 0] >= 0, 0]] = 1.0
    U[prob.lam_dof[prob.lam_dof[:, 1] >= 0, 1]] = -2.0
    U[prob.s_dof] = [0.003, -0.001]
    gv = np.flatnonzero(prob.gamma_vertex)
    for c in range(2):
        U[prob.x_dof[gv, c]] = prob.vX[gv, c] + U[prob.s_dof[c]]
    R = ale.residual(prob, U)
    perim = 2.0                                                 # 0.5 x 0.5 square hole
    assert R[prob.s_dof[0]] == pytest.approx(prob.k * 0.003 + perim, rel=1e-13)
    assert R[prob.s_dof[1]] == pytest.approx(prob.k * -0.001 - 2 * perim, rel=1e-13)


def test_translation_invariance(prob):
    """Moving the current and previous mesh by the same vector changes no flow
    residual (integrals on K_t depend on positions only through differences)."""
    U = prob.perturbed_state(6)
    P1 = build_ale_2d(16, 8, 0)
    shift = np.array([0.37, -0.21])
    P1.x_prev = prob.x_prev + shift
    U1 = U.copy()
    m = prob.x_dof >= 0
    U1[prob.x_dof[m]] += np.broadcast_to(shift, prob.x_dof.shape)[m]
    u, p, x, lam, s = ale._fields(prob, U)
    Ru0, Rp0 = ale.volume_local(p[prob.vtx], u[prob.tri], prob.u_prev[prob.tri], x[prob.vtx],
                                prob.x_prev[prob.vtx], prob.nu, prob.dt)
    Ru1, Rp1 = ale.volume_local(p[prob.vtx], u[prob.tri], prob.u_prev[prob.tri], x[prob.vtx] + shift,
                                P1.x_prev[prob.vtx], prob.nu, prob.dt)
    assert np.abs(Ru1 - Ru0).max() <= 1e-12 * np.abs(Ru0).max()
    assert np.abs(Rp1 - Rp0).max() <= 1e-12 * np.abs(Rp0).max()
