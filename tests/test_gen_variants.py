"""Pins of the generator's paper-faithful variants (CPU only).

Each variant is checked against something other than its own code: textbook
element entries, an energy identity with an independent quadrature, exact
geometry of the mapped hole, linearity in the time coefficient, and exact
elimination of the force accumulators."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

from vivjac import build_2d
from vivjac.gen2d import p1_elasticity, pseudo_solid_blocks


def test_p1_elasticity_textbook_entries():
    """On the reference triangle (area 1/2) with lambda = mu = 1 the element matrix
    is a(u, v) = int lambda div u div v + 2 mu eps(u):eps(v), entry by entry."""
    A = p1_elasticity(np.eye(2)[None], np.array([0.5]))[0]       # int lambda = 1/2
    grads = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    for i in range(3):
        for a in range(2):
            for j in range(3):
                for b in range(2):
                    Gu = np.zeros((2, 2))       # grad of phi_j e_b: row = component
                    Gu[b] = grads[j]
                    Gv = np.zeros((2, 2))
                    Gv[a] = grads[i]
                    eu, ev = 0.5 * (Gu + Gu.T), 0.5 * (Gv + Gv.T)
                    ref = 0.5 * (np.trace(Gu) * np.trace(Gv) + 2.0 * np.sum(eu * ev))
                    assert A[i, a, j, b] == pytest.approx(ref, abs=1e-15)
    assert A[0, 0, 0, 0] == pytest.approx(2.0)     # hand value: (1 + 2 * 3/2) / 2


def _duffy_rule(n=10):
    """Gauss-Legendre n x n collapsed onto the reference triangle (exact to degree
    2n - 2); independent of the generator's 7-point rule."""
    g, w = np.polynomial.legendre.leggauss(n)
    g, w = 0.5 * (g + 1), 0.5 * w
    u, v = np.meshgrid(g, g, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    x = u.ravel()
    y = (v * (1 - u)).ravel()
    return np.stack([x, y], 1), (wu * wv * (1 - u)).ravel()


def _full_matrix(Ad, nodes, nn):
    E, nl = nodes.shape
    dof = (2 * nodes[:, :, None] + np.arange(2)[None, None, :]).reshape(E, 2 * nl)
    r = np.broadcast_to(dof[:, :, None], (E, 2 * nl, 2 * nl)).ravel()
    c = np.broadcast_to(dof[:, None, :], (E, 2 * nl, 2 * nl)).ravel()
    return sp.coo_matrix((Ad.reshape(E, 2 * nl, 2 * nl).ravel(), (r, c)), shape=(2 * nn, 2 * nn)).tocsr()


@pytest.mark.parametrize("position", ["p1", "p2"])
@pytest.mark.parametrize("lame", ["inv_area", "radial"])
@pytest.mark.parametrize("hole", ["square", "circle"])
def test_pseudo_solid_energy_identity(position, lame, hole):
    """For a linear displacement d(X) = G X the assembled (unconstrained) pseudo-
    solid energy is (tr(eps)^2 + 2 eps:eps) * int_Omega lambda_s, with
    int lambda_s = number of elements for 1/|K| and, for the radial law, the
    integral of (r - (D/2)^2)^-2 by an independent high-order rule; an
    infinitesimal rotation carries no energy."""
    s = build_2d(32, 16, 0, position=position, lame=lame, hole=hole)
    m = s.meta["mesh"]
    X, Y, tri = m["X"], m["Y"], m["tri"]
    c, (ax, by) = s.meta["hole_center"], s.meta["hole_half_widths"]
    Ad = pseudo_solid_blocks(X, Y, tri, position, lame, c, ax + by)
    nodes = tri[:, :3] if position == "p1" else tri
    A = _full_matrix(Ad, nodes, X.size)
    Gm = np.array([[0.3, -0.7], [0.2, 0.5]])
    d = np.zeros(2 * X.size)
    d[0::2] = Gm[0, 0] * X + Gm[0, 1] * Y
    d[1::2] = Gm[1, 0] * X + Gm[1, 1] * Y
    eps = 0.5 * (Gm + Gm.T)
    dens = np.trace(Gm) ** 2 + 2.0 * np.sum(eps * eps)
    if lame == "inv_area":
        lam_int = float(tri.shape[0])
    else:
        pts, w = _duffy_rule(12)
        V = tri[:, :3]
        x0, y0 = X[V[:, 0]], Y[V[:, 0]]
        e1 = np.stack([X[V[:, 1]] - x0, Y[V[:, 1]] - y0], 1)
        e2 = np.stack([X[V[:, 2]] - x0, Y[V[:, 2]] - y0], 1)
        xq = x0[:, None] + pts[None, :, 0] * e1[:, None, 0] + pts[None, :, 1] * e2[:, None, 0]
        yq = y0[:, None] + pts[None, :, 0] * e1[:, None, 1] + pts[None, :, 1] * e2[:, None, 1]
        jac = np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
        r = np.hypot(xq - c[0], yq - c[1])
        D = ax + by
        lam_int = float((jac[:, None] * w[None, :] * (r - (D / 2) ** 2) ** -2.0).sum())
    energy = d @ (A @ d)
    assert energy == pytest.approx(dens * lam_int, rel=2e-5 if lame == "radial" else 1e-12)
    rot = np.zeros(2 * X.size)
    rot[0::2], rot[1::2] = -(Y - c[1]), X - c[0]
    assert np.abs(A @ rot).max() <= 1e-11 * np.abs(A).max() * np.abs(rot).max() * 10


def _gamma_deficits(nx, ny):
    s = build_2d(nx, ny, 0, hole="circle")
    m = s.meta["mesh"]
    c, (ax, by) = s.meta["hole_center"], s.meta["hole_half_widths"]
    g = m["gamma_nodes"]
    R = ax
    # every hole-boundary vertex lies on the circle
    gv = g[m["vertex"][g]]
    assert np.allclose(np.hypot(m["X"][gv] - c[0], m["Y"][gv] - c[1]), R, rtol=0, atol=1e-14)
    # the boundary is the inscribed polygon through those vertices
    ang = np.sort(np.arctan2(m["Y"][gv] - c[1], m["X"][gv] - c[0]))
    dth = np.diff(np.concatenate([ang, ang[:1] + 2 * np.pi]))
    perim = float((2 * R * np.sin(dth / 2)).sum())
    poly_area = float((0.5 * R * R * np.sin(dth)).sum())
    assert s.meta["gamma_length"] == pytest.approx(perim, rel=1e-13)
    assert s.meta["fluid_area"] == pytest.approx(4.0 * 2.0 - poly_area, rel=1e-13)
    return 2 * np.pi * R - perim, np.pi * R * R - poly_area


def test_circle_hole_geometry_converges_second_order():
    """The mapped hole is the polygon inscribed in the circle through its boundary
    vertices (length and enclosed area exact), and its deficits against the circle
    shrink by about 4 when the mesh is refined by 2."""
    assert build_2d(32, 16, 0, hole="circle").meta["hole_half_widths"][0] == pytest.approx(0.25)
    dl1, da1 = _gamma_deficits(32, 16)
    dl2, da2 = _gamma_deficits(64, 32)
    assert dl1 > 0 and da1 > 0
    assert 3.5 < dl1 / dl2 < 4.5 and 3.5 < da1 / da2 < 4.5


def test_radial_lame_reading():
    from vivjac.gen2d import radial_lame
    # D = 0.5: (r - 1/16)^-2 at r = 1 and r = 0.25 (on the square's side midpoints)
    assert radial_lame(np.array([3.0]), np.array([1.0]), (2.0, 1.0), 0.5)[0] == pytest.approx((15 / 16) ** -2)
    assert radial_lame(np.array([2.25]), np.array([1.0]), (2.0, 1.0), 0.5)[0] == pytest.approx((3 / 16) ** -2)


def test_bdf2_scales_only_the_time_derivative():
    """The values are affine in the time coefficient: BDF2 (3/(2 dt)) minus BDF1
    (1/dt) is half of BDF1 minus the coefficient-free matrix, and it touches only
    the velocity-velocity block and the multiplier rows' s columns."""
    s1 = build_2d(16, 8, 2)
    s2 = build_2d(16, 8, 2, scheme="bdf2")
    s0 = build_2d(16, 8, 2, alpha0=0.0)
    A1, A2, A0 = s1.to_scipy(), s2.to_scipy(), s0.to_scipy()
    diff = (A2 - A1).tocoo()
    half = 0.5 * (A1 - A0)
    assert abs(diff - half).max() <= 1e-12 * abs(A1).max()
    u, lam, sb = s1.blocks["u"], s1.blocks["lam"], s1.blocks["s"]
    nz = np.abs(diff.data) > 1e-12 * abs(A1).max()
    r, c = diff.row[nz], diff.col[nz]
    in_uu = (r >= u[0]) & (r < u[1]) & (c >= u[0]) & (c < u[1])
    in_ls = (r >= lam[0]) & (r < lam[1]) & (c >= sb[0]) & (c < sb[1])
    assert (in_uu | in_ls).all() and in_uu.any() and in_ls.any()
    ls1 = A1[lam[0]:lam[1], sb[0]:sb[1]].toarray()
    ls2 = A2[lam[0]:lam[1], sb[0]:sb[1]].toarray()
    assert np.allclose(ls2[ls1 != 0] / ls1[ls1 != 0], 1.5, rtol=1e-15, atol=0)


def test_force_accumulators_eliminate_to_the_master_form():
    """With F_c = sum_j m_j lambda_j,c as extra unknowns and k s_c + F_c = 0, the
    solution restricted to the other unknowns equals the master form's."""
    sm = build_2d(16, 8, 3)
    sa = build_2d(16, 8, 3, coupling="accumulator")
    n0 = sm.n
    assert sa.n == n0 + 2 and list(sa.root) == [n0 - 2, n0 - 1, n0, n0 + 1]
    rng = np.random.default_rng(0)
    b = rng.standard_normal(n0)
    xm = sla.spsolve(sm.to_scipy().tocsc(), b)
    xa = sla.spsolve(sa.to_scipy().tocsc(), np.concatenate([b, [0.0, 0.0]]))
    assert np.abs(xa[:n0] - xm).max() <= 1e-9 * np.abs(xm).max()
    m = sm.meta
    lam0 = sm.blocks["lam"][0]
    # F_c equals the weighted multiplier sum (the spring row then reads k s + F = 0)
    Am = sm.to_scipy()
    for comp in range(2):
        srow = Am[n0 - 2 + comp].toarray().ravel()
        weights = srow[lam0:sm.blocks["lam"][1]]
        assert xa[n0 + comp] == pytest.approx(weights @ xm[lam0:sm.blocks["lam"][1]], rel=1e-9)
        assert m["k"] * xa[n0 - 2 + comp] + xa[n0 + comp] == pytest.approx(b[n0 - 2 + comp], abs=1e-9)


def test_p1_position_dof_counts():
    """Linear position: displacement dofs only on vertices, counted from the
    lattice: all vertices minus those strictly inside the hole, minus both
    components on x = 0 and x = 4 and the normal one on the slip walls; every
    hole-boundary vertex row is replaced by d - s = 0."""
    for nx, ny in [(16, 8), (32, 16), (20, 10)]:
        s = build_2d(nx, ny, 1, position="p1")
        a, b = max(1, nx // 16), max(1, ny // 8)
        verts = (nx + 1) * (ny + 1) - (2 * a - 1) * (2 * b - 1)
        nd = 2 * verts - 4 * (ny + 1) - 2 * (nx - 1)
        d0, d1 = s.blocks["d"]
        assert d1 - d0 == nd
        A = s.to_scipy()
        sx = s.blocks["s"][0]
        rows = [r for r in range(d0, d1) if A[r, sx] != 0 or A[r, sx + 1] != 0]
        assert len(rows) == 2 * 4 * (a + b)
        for r in rows:
            row = A[r].toarray().ravel()
            assert np.count_nonzero(row) == 2 and row[r] == 1.0
