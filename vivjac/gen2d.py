"""2D synthetic Jacobian: rectangle [0,4]x[0,2] with a square hole (the cylinder).

Construction (all readings of the paper's silent points are listed in the
project design notes; each is restated here where it is used):

* Mesh: nx x ny cells, each split along its (i,j)->(i+1,j+1) diagonal.  The
  hole is the cell block [nx/2-a, nx/2+a) x [ny/2-b, ny/2+b) with
  a = max(1, nx//16), b = max(1, ny//8), i.e. the same physical square at every
  refinement.  P2 nodes are exactly the half-cell lattice points of fluid cells.
* Unknowns (Sec. 3.3): Taylor-Hood P2 velocity u and P1 pressure p, P2 mesh
  displacement d, P2 multiplier lambda on the hole boundary Gamma, and the two
  rigid-position dofs s of the global position master (Sec. 4.2, last scheme,
  with a single partition).
* Numbering: u (P2 nodes in lexicographic (ix, iy) lattice order, component
  fastest), p (P1 vertices, same order), d, lambda, s.
* Boundary conditions (eq. flowBC, eq. psBC): inlet x=0 removes both u
  components; the slip walls y=0, y=2 remove u_y; the outflow x=4 is natural.
  d is fixed on x=0 and x=4 and slides (d_y removed) on y=0, y=2.  Dirichlet
  dofs are removed from the system, not kept as identity rows.
* Blocks (eq. weak_system, Jacobian of Sec. 3.2):
    u rows: alpha0 (v,u) + (v,(w.grad)u) + 2 nu (eps(v),eps(u)) - (div v, p)
            - <v, lambda>_Gamma
    p rows: -(q, div u)
    d rows: (lam_s div dhat div d + 2 mu_s eps(dhat):eps(d)), lam_s = mu_s = 1/|K|
    lambda rows: -<mu, u>_Gamma + alpha0 <mu, 1> s   (no-slip u = d/dt x with
            x = X + s on Gamma, BDF1 coefficient alpha0 = 1/dt)
    d rows on Gamma: d_{i,c} - s_c = 0 (position masters, eq. coupling_constraint)
    s rows: k s_c + sum_j m_j lambda_{j,c} = 0 with m_j = int_Gamma phi_j
            (spring balance, eq. solid_balance, F_fluid = -int lambda)
* Quadrature: the 7-point degree-5 Radon rule (exact for every volume term);
  Gamma terms use the exact P2 edge mass matrix.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class System:
    """One coupled Jacobian in CSR form plus its seeded right-hand-side stream."""

    n: int
    rowptr: np.ndarray          # int64[n+1]
    colind: np.ndarray          # int32[nnz]
    values: np.ndarray          # float64[nnz], Newton step 0
    root: np.ndarray            # int32[2]: the rigid-position dofs s
    blocks: dict                # name -> (start, end) dof range
    meta: dict = field(default_factory=dict)
    b0: np.ndarray | None = None  # float64[nrhs0, n]: step-0 right-hand sides

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self, values=None):
        v = self.values if values is None else values
        return sp.csr_matrix((v, self.colind, self.rowptr), shape=(self.n, self.n))


# ---------------------------------------------------------------- quadrature
def radon7():
    """Degree-5, 7-point rule on the reference triangle (area 1/2)."""
    r = np.sqrt(15.0)
    a = (6.0 - r) / 21.0
    b = (6.0 + r) / 21.0
    wa = (155.0 - r) / 1200.0
    wb = (155.0 + r) / 1200.0
    pts = np.array([[1 / 3, 1 / 3],
                    [a, a], [1 - 2 * a, a], [a, 1 - 2 * a],
                    [b, b], [1 - 2 * b, b], [b, 1 - 2 * b]])
    w = np.array([9 / 40, wa, wa, wa, wb, wb, wb]) * 0.5
    return pts, w


def p2_tri(pts):
    """P2 basis values (Q,6) and reference gradients (Q,6,2) on the triangle.

    Local order: vertices 0,1,2 then edge midpoints (0,1), (1,2), (2,0)."""
    xi, eta = pts[:, 0], pts[:, 1]
    L = np.stack([1 - xi - eta, xi, eta], axis=1)
    dL = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    Q = pts.shape[0]
    phi = np.empty((Q, 6))
    g = np.empty((Q, 6, 2))
    for v in range(3):
        phi[:, v] = L[:, v] * (2 * L[:, v] - 1)
        g[:, v, :] = (4 * L[:, v] - 1)[:, None] * dL[v][None, :]
    for e, (a, b) in enumerate([(0, 1), (1, 2), (2, 0)]):
        phi[:, 3 + e] = 4 * L[:, a] * L[:, b]
        g[:, 3 + e, :] = 4 * (L[:, b][:, None] * dL[a][None, :] + L[:, a][:, None] * dL[b][None, :])
    return phi, g, L


# ---------------------------------------------------------------- assembly
class _Triplets:
    """COO triplets; removed dofs carry index -1 and are dropped once at the end."""

    def __init__(self):
        self.r, self.c, self.v = [], [], []

    def add(self, rows, cols, vals):
        rows = np.asarray(rows, dtype=np.int32)
        cols = np.asarray(cols, dtype=np.int32)
        vals = np.asarray(vals, dtype=np.float64)
        shape = np.broadcast_shapes(rows.shape, cols.shape, vals.shape)
        self.r.append(np.broadcast_to(rows, shape).ravel())
        self.c.append(np.broadcast_to(cols, shape).ravel())
        self.v.append(np.broadcast_to(vals, shape).ravel())

    def csr(self, n, drop_rows=None):
        r = np.concatenate(self.r)
        c = np.concatenate(self.c)
        v = np.concatenate(self.v)
        keep = (r >= 0) & (c >= 0)
        if drop_rows is not None:
            keep &= ~drop_rows[np.maximum(r, 0)]
        r, c, v = r[keep], c[keep], v[keep]
        m = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
        m.sort_indices()
        return m


def _vector_block_rows(dofmap, nodes):
    """Global dof index for local vector dof 2*i+c of each element."""
    # dofmap: (Nnodes, 2); nodes: (E, nloc)  -> (E, 2*nloc)
    g = dofmap[nodes]                  # (E, nloc, 2)
    return g.reshape(nodes.shape[0], -1)


def mesh_2d(nx: int, ny: int, Lx: float = 4.0, Ly: float = 2.0) -> dict:
    """The structured triangulation of the 2D construction: nx x ny cells of
    [0,Lx]x[0,Ly] minus the hole cells [nx/2-a, nx/2+a) x [ny/2-b, ny/2+b)
    (a = max(1, nx//16), b = max(1, ny//8)), each cell split along its
    (i,j)->(i+1,j+1) diagonal into T1 = (00, 10, 11) and T2 = (00, 11, 01)
    (counter-clockwise).  P2 nodes are the half-cell lattice points of fluid
    cells, numbered in lexicographic (ix, iy) order; ``tri`` lists each
    triangle's vertices then its edge midpoints (0,1), (1,2), (2,0)."""
    hx, hy = Lx / nx, Ly / ny
    NX, NY = 2 * nx + 1, 2 * ny + 1
    a = max(1, nx // 16)
    b = max(1, ny // 8)
    i0, i1 = nx // 2 - a, nx // 2 + a
    j0, j1 = ny // 2 - b, ny // 2 + b

    # fluid cells and triangles (lattice coordinates)
    ci, cj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    ci, cj = ci.ravel(), cj.ravel()
    fluid = ~((ci >= i0) & (ci < i1) & (cj >= j0) & (cj < j1))
    ci, cj = ci[fluid], cj[fluid]
    I0, J0 = 2 * ci, 2 * cj
    # T1 = (00, 10, 11), T2 = (00, 11, 01)
    vI = np.concatenate([np.stack([I0, I0 + 2, I0 + 2], 1), np.stack([I0, I0 + 2, I0], 1)])
    vJ = np.concatenate([np.stack([J0, J0, J0 + 2], 1), np.stack([J0, J0 + 2, J0 + 2], 1)])
    E = vI.shape[0]
    mI = np.stack([(vI[:, 0] + vI[:, 1]) // 2, (vI[:, 1] + vI[:, 2]) // 2, (vI[:, 2] + vI[:, 0]) // 2], 1)
    mJ = np.stack([(vJ[:, 0] + vJ[:, 1]) // 2, (vJ[:, 1] + vJ[:, 2]) // 2, (vJ[:, 2] + vJ[:, 0]) // 2], 1)
    LI = np.concatenate([vI, mI], 1)
    LJ = np.concatenate([vJ, mJ], 1)

    used = np.zeros(NX * NY, dtype=bool)
    used[(LI * NY + LJ).ravel()] = True
    node_of = -np.ones(NX * NY, dtype=np.int64)
    node_lat = np.flatnonzero(used)                    # lexicographic in (ix, iy)
    node_of[node_lat] = np.arange(node_lat.size)
    nn = node_lat.size
    nI, nJ = node_lat // NY, node_lat % NY
    tri = node_of[LI * NY + LJ]                        # (E, 6)

    vert_mask = (nI % 2 == 0) & (nJ % 2 == 0)
    vert_of = -np.ones(nn, dtype=np.int64)
    vert_of[vert_mask] = np.arange(int(vert_mask.sum()))
    nv = int(vert_mask.sum())
    tri_p = vert_of[tri[:, :3]]

    inlet = nI == 0
    outlet = nI == NX - 1
    wall = (nJ == 0) | (nJ == NY - 1)
    on_gamma = (nI >= 2 * i0) & (nI <= 2 * i1) & (nJ >= 2 * j0) & (nJ <= 2 * j1)

    return dict(hx=hx, hy=hy, NX=NX, NY=NY, a=a, b=b, hole=(i0, i1, j0, j1), E=E, tri=tri, node_of=node_of,
                nn=nn, nI=nI, nJ=nJ, vert_mask=vert_mask, vert_of=vert_of, nv=nv, tri_p=tri_p, inlet=inlet,
                outlet=outlet, wall=wall, on_gamma=on_gamma)


def gamma_edges(m: dict):
    """Edges of the hole boundary as (end node, end node, midpoint node), in the
    order the 2D construction assembles them: bottom/top rows of the hole first,
    then its left/right columns."""
    i0, i1, j0, j1 = m["hole"]
    NY, node_of = m["NY"], m["node_of"]
    out = []
    for i in range(i0, i1):
        for jj in (j0, j1):
            out.append((node_of[2 * i * NY + 2 * jj], node_of[(2 * i + 2) * NY + 2 * jj],
                        node_of[(2 * i + 1) * NY + 2 * jj]))
    for j in range(j0, j1):
        for ii in (i0, i1):
            out.append((node_of[2 * ii * NY + 2 * j], node_of[2 * ii * NY + 2 * j + 2],
                        node_of[2 * ii * NY + 2 * j + 1]))
    return np.array(out, dtype=np.int64)


def p1_elasticity(invT, lam_int):
    """Pseudo-solid element matrices of affine P1 triangles, (E, 3, 2, 3, 2) in
    (node i, component a, node j, component b): lam_int * (d_a phi_i d_b phi_j +
    delta_ab grad phi_i . grad phi_j + d_b phi_i d_a phi_j), the bilinear form of
    lambda_s div div + 2 mu_s eps:eps with lambda_s = mu_s, whose integral over the
    element is lam_int (the gradients are constant)."""
    gref = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    G = np.einsum("eab,ib->eia", invT, gref)                   # (E,3,2)
    D = G[:, :, :, None, None] * G[:, None, None, :, :]        # d_a phi_i d_b phi_j
    K = np.einsum("eia,eja->eij", G, G)
    eye2 = np.eye(2)
    A = D + K[:, :, None, :, None] * eye2[None, None, :, None, :] + np.transpose(D, (0, 1, 4, 3, 2))
    return lam_int[:, None, None, None, None] * A


def circle_map(X, Y, xc, yc, ax, by, blend=2.0):
    """Move the lattice nodes around the rectangular hole [xc-ax, xc+ax] x [yc-by,
    yc+by] so that its boundary lies on the ellipse of half-axes (ax, by) (a circle
    when ax = by).  In normalised coordinates q = ((X-xc)/ax, (Y-yc)/by), the square
    of radius s = max|q_i| is pulled toward the circle of radius s by the weight
    w = (blend - s) / (blend - 1) on 1 <= s <= blend; nodes with s >= blend stay."""
    qx, qy = (X - xc) / ax, (Y - yc) / by
    s = np.maximum(np.abs(qx), np.abs(qy))
    r = np.hypot(qx, qy)
    w = np.clip((blend - s) / (blend - 1.0), 0.0, 1.0)
    f = np.where(r > 0, (1.0 - w) + w * s / np.where(r > 0, r, 1.0), 1.0)
    return xc + ax * qx * f, yc + by * qy * f


def radial_lame(x, y, center, diameter):
    """The paper's radial Lame distribution lambda_s = mu_s (Sec. 6, "Lame
    coefficients"), read as printed: (r - (D/2)^2)^-2, r = distance to the centre."""
    return (np.hypot(x - center[0], y - center[1]) - (diameter / 2) ** 2) ** -2.0


def pseudo_solid_blocks(X, Y, tri, position, lame, center, diameter):
    """Element matrices of the pseudo-solid block, (E, nl, 2, nl, 2) with nl = 3
    (P1 position) or 6 (P2): lambda_s div div + 2 mu_s eps:eps with lambda_s = mu_s
    equal to 1/|K| ("inv_area") or radial_lame ("radial"), integrated with the
    7-point rule.  The P2 / inv_area combination is assembled inline by build_2d
    (same matrices; kept there so the configured construction stays bitwise)."""
    V = tri[:, :3]
    x0, y0 = X[V[:, 0]], Y[V[:, 0]]
    Jm = np.empty((tri.shape[0], 2, 2))
    Jm[:, 0, 0] = X[V[:, 1]] - x0
    Jm[:, 0, 1] = X[V[:, 2]] - x0
    Jm[:, 1, 0] = Y[V[:, 1]] - y0
    Jm[:, 1, 1] = Y[V[:, 2]] - y0
    det = Jm[:, 0, 0] * Jm[:, 1, 1] - Jm[:, 0, 1] * Jm[:, 1, 0]
    invT = np.empty_like(Jm)
    invT[:, 0, 0] = Jm[:, 1, 1] / det
    invT[:, 0, 1] = -Jm[:, 1, 0] / det
    invT[:, 1, 0] = -Jm[:, 0, 1] / det
    invT[:, 1, 1] = Jm[:, 0, 0] / det
    qp, qw = radon7()
    phi, gref, Lq = p2_tri(qp)
    W = qw[None, :] * np.abs(det)[:, None]
    if lame == "radial":
        lamW = W * radial_lame(Lq @ X[V].T, Lq @ Y[V].T, center, diameter).T   # (E,Q)
    else:
        lamW = W / (0.5 * np.abs(det))[:, None]
    if position == "p1":
        return p1_elasticity(invT, lamW.sum(1))
    G = np.einsum("eab,qib->eqia", invT, gref)
    Dl = np.einsum("eq,eqia,eqjb->eiajb", lamW, G, G)
    Kl = np.einsum("eq,eqia,eqja->eij", lamW, G, G)
    eye2 = np.eye(2)
    return Dl + Kl[:, :, None, :, None] * eye2[None, None, :, None, :] + np.transpose(Dl, (0, 1, 4, 3, 2))


VARIANTS = {"position": ("p2", "p1"), "lame": ("inv_area", "radial"), "scheme": ("bdf1", "bdf2"),
            "hole": ("square", "circle"), "coupling": ("master", "accumulator")}


def build_2d(nx: int, ny: int, seed: int, *, k: float = 0.5, nu: float = 0.01,
             alpha0: float = 100.0, nrhs: int = 1, Lx: float = 4.0, Ly: float = 2.0,
             position: str = "p2", lame: str = "inv_area", scheme: str = "bdf1", hole: str = "square",
             coupling: str = "master") -> System:
    """Assemble the coupled Jacobian on an nx x ny mesh (nx, ny even).

    Variants (defaults first; the defaults are the configured construction):
      position  "p2" | "p1": mesh displacement on the P2 nodes, or linear on the
                vertices as the paper discretizes the position (Sec. 3.3)
      lame      "inv_area" | "radial": lambda_s = mu_s = 1/|K| per element, or the
                paper's radial distribution of Sec. 6 ("Lame coefficients"), read
                as printed, (r - (D/2)^2)^-2 with r the distance to the hole's
                centre, evaluated at the quadrature points
      scheme    "bdf1" | "bdf2": alpha0 is 1/dt; BDF2 scales the time-derivative
                coefficient (mass block and the multiplier rows' s term) by 3/2
      hole      "square" | "circle": the cell-aligned square hole, or the same
                lattice mapped so that the hole boundary is a circle (circle_map)
      coupling  "master" | "accumulator": s rows k s_c + sum_j m_j lambda_j,c = 0,
                or two force-accumulator dofs F_c = sum_j m_j lambda_j,c with
                k s_c + F_c = 0 (Sec. 4.2, global position master to global force
                accumulator); the root then holds s and F."""
    if nx < 4 or ny < 4 or nx % 2 or ny % 2:
        raise ValueError("nx, ny must be even and >= 4")
    for key, val in (("position", position), ("lame", lame), ("scheme", scheme), ("hole", hole),
                     ("coupling", coupling)):
        if val not in VARIANTS[key]:
            raise ValueError(f"{key} must be one of {VARIANTS[key]}")
    a_t = alpha0 * (1.5 if scheme == "bdf2" else 1.0)     # time-derivative coefficient
    m = mesh_2d(nx, ny, Lx, Ly)
    hx, hy, NX, NY, a, b = m["hx"], m["hy"], m["NX"], m["NY"], m["a"], m["b"]
    i0, i1, j0, j1 = m["hole"]
    E, tri, node_of, nn, nI, nJ = m["E"], m["tri"], m["node_of"], m["nn"], m["nI"], m["nJ"]
    vert_mask, vert_of, nv, tri_p = m["vert_mask"], m["vert_of"], m["nv"], m["tri_p"]
    inlet, outlet, wall, on_gamma = m["inlet"], m["outlet"], m["wall"], m["on_gamma"]

    # ---- dof numbering
    nxt = 0
    u_keep = np.ones((nn, 2), dtype=bool)
    u_keep[inlet, :] = False
    u_keep[wall, 1] = False
    u_dof = -np.ones((nn, 2), dtype=np.int64)
    u_dof[u_keep] = np.arange(int(u_keep.sum()))       # node-major, component fastest
    nxt = int(u_keep.sum())
    blocks = {"u": (0, nxt)}
    p_dof = np.arange(nv) + nxt
    blocks["p"] = (nxt, nxt + nv)
    nxt += nv
    d_keep = np.ones((nn, 2), dtype=bool)
    d_keep[inlet | outlet, :] = False
    d_keep[wall, 1] = False
    if position == "p1":
        d_keep[~vert_mask, :] = False                  # linear position: vertices only
    d_dof = -np.ones((nn, 2), dtype=np.int64)
    d_dof[d_keep] = np.arange(int(d_keep.sum())) + nxt
    blocks["d"] = (nxt, nxt + int(d_keep.sum()))
    nxt += int(d_keep.sum())
    g_nodes = np.flatnonzero(on_gamma)
    lam_dof = -np.ones((nn, 2), dtype=np.int64)
    lam_dof[g_nodes, :] = (np.arange(2 * g_nodes.size) + nxt).reshape(-1, 2)
    blocks["lam"] = (nxt, nxt + 2 * g_nodes.size)
    nxt += 2 * g_nodes.size
    s_dof = np.array([nxt, nxt + 1])
    blocks["s"] = (nxt, nxt + 2)
    nxt += 2
    f_dof = None
    if coupling == "accumulator":
        f_dof = np.array([nxt, nxt + 1])
        blocks["F"] = (nxt, nxt + 2)
        nxt += 2
    n = nxt

    # ---- geometry (affine triangles)
    X = nI * (hx / 2)
    Y = nJ * (hy / 2)
    xc, yc, ax, by = 0.5 * (i0 + i1) * hx, 0.5 * (j0 + j1) * hy, a * hx, b * hy
    if hole == "circle":
        X, Y = circle_map(X, Y, xc, yc, ax, by)
        # affine P2 elements: the edge nodes sit at the straight edges' midpoints
        for e, (va, vb) in enumerate([(0, 1), (1, 2), (2, 0)]):
            X[tri[:, 3 + e]] = 0.5 * (X[tri[:, va]] + X[tri[:, vb]])
            Y[tri[:, 3 + e]] = 0.5 * (Y[tri[:, va]] + Y[tri[:, vb]])
    x0, y0 = X[tri[:, 0]], Y[tri[:, 0]]
    Jm = np.empty((E, 2, 2))
    Jm[:, 0, 0] = X[tri[:, 1]] - x0
    Jm[:, 0, 1] = X[tri[:, 2]] - x0
    Jm[:, 1, 0] = Y[tri[:, 1]] - y0
    Jm[:, 1, 1] = Y[tri[:, 2]] - y0
    det = Jm[:, 0, 0] * Jm[:, 1, 1] - Jm[:, 0, 1] * Jm[:, 1, 0]
    if not (det > 0).all():
        raise AssertionError("inverted or degenerate triangle")
    area = 0.5 * np.abs(det)
    invT = np.empty((E, 2, 2))                          # J^{-T}
    invT[:, 0, 0] = Jm[:, 1, 1] / det
    invT[:, 0, 1] = -Jm[:, 1, 0] / det
    invT[:, 1, 0] = -Jm[:, 0, 1] / det
    invT[:, 1, 1] = Jm[:, 0, 0] / det

    qp, qw = radon7()
    phi, gref, Lq = p2_tri(qp)                          # (Q,6), (Q,6,2), (Q,3)
    W = qw[None, :] * np.abs(det)[:, None]              # (E,Q)
    G = np.einsum("eab,qib->eqia", invT, gref)          # physical grads (E,Q,6,2)

    # seeded convecting velocity (nodal P2, U[-1,1] per component), then RHS
    rng = np.random.default_rng(seed)
    wnod = rng.uniform(-1.0, 1.0, size=(nn, 2))
    b0 = rng.standard_normal((nrhs, n))

    M = np.einsum("eq,qi,qj->eij", W, phi, phi)
    K = np.einsum("eq,eqia,eqja->eij", W, G, G)
    D = np.einsum("eq,eqia,eqjb->eiajb", W, G, G)       # int d_a phi_i d_b phi_j
    wq = np.einsum("qk,ekd->eqd", phi, wnod[tri])        # w at quadrature points
    C = np.einsum("eq,qi,eqd,eqjd->eij", W, phi, wq, G)  # int phi_i (w.grad) phi_j
    Bq = -np.einsum("eq,qk,eqjc->ekjc", W, Lq, G)       # -int psi_k d_c phi_j  (E,3,6,2)

    eye2 = np.eye(2)
    # velocity block, local (i,c),(j,c'):
    Avel = (a_t * M + C)[:, :, None, :, None] * eye2[None, None, :, None, :]
    Avel = Avel + nu * (K[:, :, None, :, None] * eye2[None, None, :, None, :]
                        + np.transpose(D, (0, 1, 4, 3, 2)))
    # pseudo-solid
    if position == "p2" and lame == "inv_area":
        # lam_s = mu_s = 1/|K|
        lam_s = (1.0 / area)[:, None, None, None, None]
        Ad = lam_s * (D + K[:, :, None, :, None] * eye2[None, None, :, None, :]
                      + np.transpose(D, (0, 1, 4, 3, 2)))
    else:
        Ad = pseudo_solid_blocks(X, Y, tri, position, lame, (xc, yc), ax + by)

    T = _Triplets()
    ur = _vector_block_rows(u_dof, tri)                 # (E,12)
    dloc = tri[:, :3] if position == "p1" else tri
    dr = _vector_block_rows(d_dof, dloc)
    T.add(ur[:, :, None], ur[:, None, :], Avel.reshape(E, 12, 12))
    pr = p_dof[tri_p]                                   # (E,3)
    Bflat = Bq.reshape(E, 3, 12)
    T.add(pr[:, :, None], ur[:, None, :], Bflat)                     # p rows
    T.add(ur[:, :, None], pr[:, None, :], np.transpose(Bflat, (0, 2, 1)))  # u rows
    nd = 2 * dloc.shape[1]
    T.add(dr[:, :, None], dr[:, None, :], Ad.reshape(E, nd, nd))

    # ---- Gamma edges (hole perimeter), nodes (end, end, mid)
    edges = []
    for i in range(i0, i1):
        for jj in (j0, j1):
            edges.append(((2 * i, 2 * jj), (2 * i + 2, 2 * jj), (2 * i + 1, 2 * jj), hx))
    for j in range(j0, j1):
        for ii in (i0, i1):
            edges.append(((2 * ii, 2 * j), (2 * ii, 2 * j + 2), (2 * ii, 2 * j + 1), hy))
    Me_ref = np.array([[4.0, -1.0, 2.0], [-1.0, 4.0, 2.0], [2.0, 2.0, 16.0]]) / 30.0
    m_int = np.zeros(nn)
    for (pa, pb, pm, Le) in edges:
        en = np.array([node_of[pa[0] * NY + pa[1]], node_of[pb[0] * NY + pb[1]], node_of[pm[0] * NY + pm[1]]])
        if hole == "circle":                            # straight edge between the mapped ends
            Le = float(np.hypot(X[en[1]] - X[en[0]], Y[en[1]] - Y[en[0]]))
        Me = Le * Me_ref
        m_int[en] += Le * np.array([1 / 6, 1 / 6, 2 / 3])
        for c in range(2):
            uu = u_dof[en, c]
            ll = lam_dof[en, c]
            T.add(uu[:, None], ll[None, :], -Me)        # -<v, lambda>
            T.add(ll[:, None], uu[None, :], -Me)        # -<mu, u>
    gl = g_nodes
    gd = gl[d_dof[gl, 0] >= 0]                          # Gamma nodes carrying position dofs
    R = _Triplets()                                     # rows that replace the Gamma d rows
    for c in range(2):
        T.add(lam_dof[gl, c], s_dof[c], a_t * m_int[gl])      # +alpha0 <mu,1> s_c
        T.add(s_dof[c], s_dof[c], k)
        if f_dof is None:
            T.add(s_dof[c], lam_dof[gl, c], m_int[gl])        # spring row: sum m_j lambda_j
        else:
            T.add(s_dof[c], f_dof[c], 1.0)                    # spring row: k s_c + F_c
            T.add(f_dof[c], f_dof[c], 1.0)                    # accumulator: F_c - sum m_j lambda_j
            T.add(f_dof[c], lam_dof[gl, c], -m_int[gl])
        # position masters: d_{i,c} - s_c = 0 replaces the Gamma displacement rows
        R.add(d_dof[gd, c], d_dof[gd, c], 1.0)
        R.add(d_dof[gd, c], s_dof[c], -1.0)

    drop = np.zeros(n, dtype=bool)
    drop[d_dof[gd].ravel()] = True
    rr = np.concatenate(T.r)
    T.r, T.c, T.v = [np.where(drop[np.maximum(rr, 0)], -1, rr).astype(np.int32)] + R.r, \
        [np.concatenate(T.c)] + R.c, [np.concatenate(T.v)] + R.v
    del rr
    A = T.csr(n)

    meta = dict(dim=2, nx=nx, ny=ny, seed=seed, k=k, nu=nu, alpha0=alpha0,
                hole=(i0, i1, j0, j1), n_nodes=nn, n_vertices=nv, n_gamma_nodes=int(gl.size),
                gamma_length=float(m_int.sum()), fluid_area=float(area.sum()),
                variant=dict(position=position, lame=lame, scheme=scheme, hole=hole, coupling=coupling),
                time_coefficient=a_t, hole_center=(xc, yc), hole_half_widths=(ax, by),
                mesh=dict(X=X, Y=Y, tri=tri, gamma_nodes=gl, vertex=vert_mask))
    root = s_dof if f_dof is None else np.concatenate([s_dof, f_dof])
    return System(n=n, rowptr=A.indptr.astype(np.int64), colind=A.indices.astype(np.int32),
                  values=A.data.astype(np.float64), root=root.astype(np.int32),
                  blocks=blocks, meta=meta, b0=b0)


# ---------------------------------------------------------------- Newton stream
def newton_values(system: System, step: int) -> np.ndarray:
    """Values at Newton step t: a_t = a_{t-1} * (1 + 0.01 xi_t), xi_t ~ N(0,1).

    Step 0 is unperturbed; step t draws xi_t first from default_rng([seed, t])."""
    v = system.values.copy()
    for t in range(1, step + 1):
        rng = np.random.default_rng([system.meta["seed"], t])
        v *= 1.0 + 0.01 * rng.standard_normal(v.size)
    return v


def newton_rhs(system: System, step: int, nrhs: int = 1) -> np.ndarray:
    """Right-hand sides (nrhs, n) at Newton step t (fresh N(0,1) each step)."""
    if step == 0:
        if system.b0 is not None and system.b0.shape[0] >= nrhs:
            return system.b0[:nrhs].copy()
        rng = np.random.default_rng(system.meta["seed"])
        rng.uniform(-1.0, 1.0, size=(system.meta["n_nodes"], system.meta["dim"]))
        return rng.standard_normal((nrhs, system.n))
    rng = np.random.default_rng([system.meta["seed"], step])
    rng.standard_normal(system.nnz)
    return rng.standard_normal((nrhs, system.n))
