"""3D input-generator invariants: closed forms of the construction, the element
kernels' exactness, and the multiplier reading where Gamma meets the slip walls
(no solver arithmetic)."""
import math

import numpy as np
import pytest

from vivjac import build_3d, newton_rhs, newton_values
from vivjac.gen3d import _tet_rule, p2_tet


@pytest.fixture(scope="module")
def box():
    return build_3d(24, 12, 6, 3)


@pytest.fixture(scope="module")
def small():
    return build_3d(8, 4, 2, 1)


def test_sizes_24x12x6(box):
    s = box
    assert s.n == 84825
    assert {k: v[1] - v[0] for k, v in s.blocks.items()} == {"u": 41339, "p": 2212, "d": 40088, "lam": 1184, "s": 2}
    assert s.nnz == 6675763
    assert list(s.root) == [s.n - 2, s.n - 1]


def test_gamma_area_closed_form(box):
    # sum_j m_j = |Gamma| = lateral area of the 4h x 4h x 1 cylinder = 96 h^2, h = 1/6
    assert math.isclose(box.meta["gamma_area"], 96.0 / 36.0, rel_tol=0, abs_tol=1e-13)


def test_zero_diagonals(box):
    A = box.to_scipy()
    d = A.diagonal()
    p0, p1 = box.blocks["p"]
    l0, l1 = box.blocks["lam"]
    assert int((d == 0).sum()) == (p1 - p0) + (l1 - l0) == 3396
    assert np.abs(A[p0:p1, p0:p1]).sum() == 0 and np.abs(A[l0:l1, l0:l1]).sum() == 0


def test_lambda_z_dropped_on_slip_walls(box):
    # 416 Gamma nodes (32 per lattice layer, 13 layers) carry lambda_x, lambda_y;
    # lambda_z only off the z walls (2 x 32 nodes there): 3 * 416 - 64 = 1184
    assert box.meta["n_gamma_nodes"] == 416
    l0, l1 = box.blocks["lam"]
    assert l1 - l0 == 3 * 416 - 64


def test_spring_rows_and_masters(box):
    A = box.to_scipy().tocsr()
    l0, l1 = box.blocks["lam"]
    for c, srow in enumerate(box.root):
        row = A.getrow(srow)
        assert row[0, srow] == 0.5
        lam = [j for j in row.indices if l0 <= j < l1]
        assert math.isclose(sum(row[0, j] for j in lam), 96.0 / 36.0, abs_tol=1e-13)
        col = A.getcol(srow).toarray().ravel()
        assert math.isclose(col[l0:l1].sum(), 100.0 * 96.0 / 36.0, abs_tol=1e-10)
        # position masters: d_{i,c} - s_c = 0 rows, one per Gamma node
        d0, d1 = box.blocks["d"]
        masters = [r for r in range(d0, d1) if A.indptr[r + 1] - A.indptr[r] == 2 and A[r, srow] == -1.0]
        assert len(masters) == 416


@pytest.mark.parametrize("deg", range(6))
def test_tet_rule_exact_to_degree_5(deg):
    # int over the reference tetrahedron of xi^a eta^b zeta^c = a! b! c! / (a+b+c+3)!
    pts, w = _tet_rule(4)
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            c = deg - a - b
            exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
            got = float((w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c).sum())
            assert math.isclose(got, exact, rel_tol=1e-13), (a, b, c, got, exact)


def test_p2_tet_basis():
    # partition of unity, zero gradient sum, and the P2 integrals: vertex
    # functions integrate to -V/20, edge functions to V/5 (V = 1/6)
    pts, w = _tet_rule(4)
    phi, g, _ = p2_tet(pts)
    assert np.allclose(phi.sum(1), 1.0, atol=1e-14)
    assert np.allclose(g.sum(1), 0.0, atol=1e-13)
    ints = (w[:, None] * phi).sum(0)
    assert np.allclose(ints[:4], -1.0 / 120.0, atol=1e-15)
    assert np.allclose(ints[4:], 1.0 / 30.0, atol=1e-15)
    # nodal interpolation: phi_i(node_j) = delta_ij
    nodes = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
    mids = np.array([(nodes[i] + nodes[j]) / 2 for i, j in [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]])
    P, _, _ = p2_tet(np.vstack([nodes, mids]))
    assert np.allclose(P, np.eye(10), atol=1e-14)


def test_small_box_nonsingular_and_newton_stream(small):
    s = small
    A = s.to_scipy().toarray()
    assert np.isfinite(np.linalg.cond(A)) and np.linalg.matrix_rank(A) == s.n
    v1 = newton_values(s, 1)
    assert v1.shape == s.values.shape and not np.array_equal(v1, s.values)
    assert newton_rhs(s, 0).shape == (1, s.n)


def test_element_blocks_rigid_motions_and_constants():
    """The pseudo-solid element block annihilates rigid motions (translations and
    infinitesimal rotations: eps = 0 and div = 0), the viscous part of the velocity
    block annihilates them too, the convection of a constant field is zero (the
    velocity block on a constant equals alpha0 times the mass on it), and the
    divergence block of a translation vanishes; checked on random tetrahedra."""
    from vivjac.gen3d import element_blocks
    rng = np.random.default_rng(0)
    E = 5
    P = rng.standard_normal((E, 4, 3))
    # the 10 P2 nodes of each tetrahedron: vertices, then edge midpoints
    edges = [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]
    nodes = np.concatenate([P, np.stack([(P[:, i] + P[:, j]) / 2 for i, j in edges], 1)], 1)  # (E,10,3)
    w = rng.uniform(-1, 1, (E, 10, 3))
    Avel, Ad, Bq, vol = element_blocks(P, w, nu=0.01, alpha0=0.0)
    scale = np.abs(Ad).max()
    motions = [np.broadcast_to(np.eye(3)[c], (E, 10, 3)) for c in range(3)]
    for axis in range(3):  # rotation about axis: omega x x
        om = np.eye(3)[axis]
        motions.append(np.cross(om[None, None, :], nodes))
    for u in motions:
        r = np.einsum("eiajb,ejb->eia", Ad, u)
        assert np.abs(r).max() <= 1e-11 * scale
        # alpha0 = 0: the velocity block is convection + viscosity; viscosity kills
        # rigid motions, convection kills only constants
    for u in motions[:3]:
        r = np.einsum("eiajb,ejb->eia", Avel, u)
        assert np.abs(r).max() <= 1e-12 * np.abs(Avel).max()
        assert np.abs(np.einsum("ekjc,ejc->ek", Bq, u)).max() <= 1e-13 * np.abs(Bq).max()
    assert np.all(vol > 0)
