"""3D synthetic Jacobian: box [0,4]x[0,2]x[0,1] with a square-section cylinder.

Construction (the 3D configuration of the serving workload; the paper's 3D
runs, Sec. 6 "Three-dimensional results", use the same unknowns and coupling):

* Mesh: nx x ny x nz hexahedra (default 24 x 12 x 6, h = 1/6), each split into
  the six Kuhn tetrahedra that share its (0,0,0)->(1,1,1) diagonal, so every
  face of every hexahedron is split along the diagonal through its lowest
  corner and neighbouring hexahedra conform.  P2 nodes are exactly the
  half-cell lattice points of fluid hexahedra (all 27 per hexahedron).  The
  cylinder is the hexahedra [nx/2-a, nx/2+a) x [ny/2-b, ny/2+b) x all z, with
  a = max(1, nx//12), b = max(1, ny//6): cells 10..13 x 4..7 at 24 x 12.
* Unknowns (Sec. 3.3): Taylor-Hood P2 velocity u (3 components) and P1
  pressure p, P2 mesh displacement d, P2 multiplier lambda on the four lateral
  faces Gamma of the cylinder, and the two in-plane rigid-position dofs s (the
  cylinder moves in x and y only and is fixed in z).
* Numbering: u (P2 nodes in lexicographic (ix, iy, iz) lattice order, component
  fastest), p (P1 vertices, same order), d, lambda, s.
* Boundary conditions: inlet x=0 removes all u components; the slip walls
  y=0, y=2 remove u_y and z=0, z=1 remove u_z; the outflow x=4 is natural.  d is
  fixed on x=0 and x=4 and slides on the walls (d_y removed on y walls, d_z on z
  walls); on Gamma d_z = 0 (removed) and d_x, d_y follow the cylinder.
* Where Gamma meets the z walls the no-slip trace of u_z is already prescribed,
  and a multiplier lambda_z there would make the coupled matrix singular: those
  lambda_z are not unknowns (the paper notes that such intersections disturb the
  multiplier, Sec. 3.3).
* Blocks: as in 2D (eq. weak_system, Jacobian of Sec. 3.2): Oseen
  alpha0 (v,u) + (v,(w.grad)u) + 2 nu (eps(v),eps(u)) - (div v, p), divergence
  -(q, div u), pseudo-solid lam_s div dhat div d + 2 mu_s eps(dhat):eps(d) with
  lam_s = mu_s = 1/|K|, multiplier rows -<mu,u> + alpha0 <mu,1> s_c (c = x, y),
  Gamma rows of d replaced by d_c - s_c = 0, spring rows k s_c + sum_j m_j
  lambda_{j,c} = 0.
* Quadrature: volume terms by the collapsed-coordinate Gauss rule with 4 Gauss-
  Legendre points per direction (exact for degree 5 on a tetrahedron: the
  convection term is the highest); Gamma terms by the 7-point degree-5 triangle
  rule.
"""
from __future__ import annotations

import numpy as np

from .gen2d import System, _Triplets, p2_tri, radon7


def _tet_rule(q=4):
    """Points (Q,3) and weights (Q,) on the reference tetrahedron (volume 1/6):
    Gauss-Legendre in each collapsed coordinate, xi = a, eta = b (1 - a),
    zeta = c (1 - a)(1 - b), Jacobian (1 - a)^2 (1 - b)."""
    x, w = np.polynomial.legendre.leggauss(q)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    a, b, c = np.meshgrid(x, x, x, indexing="ij")
    wa, wb, wc = np.meshgrid(w, w, w, indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()
    W = (wa * wb * wc).ravel() * (1 - a) ** 2 * (1 - b)
    pts = np.stack([a, b * (1 - a), c * (1 - a) * (1 - b)], axis=1)
    return pts, W


_TET_EDGES = [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]


def p2_tet(pts):
    """P2 basis values (Q,10) and reference gradients (Q,10,3) on the tetrahedron.

    Local order: vertices 0..3 then edge midpoints (0,1), (1,2), (0,2), (0,3),
    (1,3), (2,3)."""
    xi, eta, zeta = pts[:, 0], pts[:, 1], pts[:, 2]
    L = np.stack([1 - xi - eta - zeta, xi, eta, zeta], axis=1)
    dL = np.array([[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    Q = pts.shape[0]
    phi = np.empty((Q, 10))
    g = np.empty((Q, 10, 3))
    for v in range(4):
        phi[:, v] = L[:, v] * (2 * L[:, v] - 1)
        g[:, v, :] = (4 * L[:, v] - 1)[:, None] * dL[v][None, :]
    for e, (i, j) in enumerate(_TET_EDGES):
        phi[:, 4 + e] = 4 * L[:, i] * L[:, j]
        g[:, 4 + e, :] = 4 * (L[:, j][:, None] * dL[i][None, :] + L[:, i][:, None] * dL[j][None, :])
    return phi, g, L


def _kuhn_tets():
    """The six tetrahedra of the unit cube along its (0,0,0)->(1,1,1) diagonal,
    as lists of corner offsets: (0, e_a, e_a + e_b, 1) over the axis orders."""
    out = []
    for order in [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]:
        p = np.zeros(3, dtype=np.int64)
        verts = [p.copy()]
        for ax in order:
            p[ax] += 1
            verts.append(p.copy())
        out.append(np.array(verts))
    return out  # each (4, 3) with coordinates in {0, 1}


def element_blocks(P, wnodal, nu, alpha0):
    """Local matrices of a batch of affine P2 tetrahedra with vertex coordinates
    P (E, 4, 3) and nodal convecting velocity wnodal (E, 10, 3): the velocity
    block (E, 10, 3, 10, 3), the pseudo-solid block with lam_s = mu_s = 1/|K|
    (same layout), the divergence block -int psi_k d_c phi_j (E, 4, 10, 3), and
    the element volumes."""
    Jm = np.transpose(P[:, 1:, :] - P[:, :1, :], (0, 2, 1))               # columns: edges from vertex 0
    det = np.linalg.det(Jm)
    vol = np.abs(det) / 6.0
    invT = np.transpose(np.linalg.inv(Jm), (0, 2, 1))                     # J^{-T}
    qp, qw = _tet_rule(4)
    phi, gref, _ = p2_tet(qp)                                # (Q,10), (Q,10,3)
    Lq = np.stack([1 - qp.sum(1), qp[:, 0], qp[:, 1], qp[:, 2]], axis=1)  # P1 basis (Q,4)
    W = qw[None, :] * np.abs(det)[:, None]                   # (E,Q)
    G = np.einsum("eab,qib->eqia", invT, gref, optimize=True)             # (E,Q,10,3)
    M = np.einsum("eq,qi,qj->eij", W, phi, phi, optimize=True)
    K = np.einsum("eq,eqia,eqja->eij", W, G, G, optimize=True)
    D = np.einsum("eq,eqia,eqjb->eiajb", W, G, G, optimize=True)          # int d_a phi_i d_b phi_j
    wq = np.einsum("qk,ekd->eqd", phi, wnodal, optimize=True)
    C = np.einsum("eq,qi,eqd,eqjd->eij", W, phi, wq, G, optimize=True)
    Bq = -np.einsum("eq,qk,eqjc->ekjc", W, Lq, G, optimize=True)           # (E,4,10,3)
    del G
    eye3 = np.eye(3)
    Avel = (alpha0 * M + C)[:, :, None, :, None] * eye3[None, None, :, None, :]
    Avel = Avel + nu * (K[:, :, None, :, None] * eye3[None, None, :, None, :] + np.transpose(D, (0, 1, 4, 3, 2)))
    lam_s = (1.0 / vol)[:, None, None, None, None]
    Ad = lam_s * (D + K[:, :, None, :, None] * eye3[None, None, :, None, :] + np.transpose(D, (0, 1, 4, 3, 2)))
    return Avel, Ad, Bq, vol


def _vector_rows(dofmap, nodes):
    g = dofmap[nodes]                  # (E, nloc, 3)
    return g.reshape(nodes.shape[0], -1)


def build_3d(nx: int = 24, ny: int = 12, nz: int = 6, seed: int = 0, *, k: float = 0.5, nu: float = 0.01,
             alpha0: float = 100.0, nrhs: int = 1, Lx: float = 4.0, Ly: float = 2.0, Lz: float = 1.0) -> System:
    """Assemble the coupled 3D Jacobian on an nx x ny x nz hexahedral mesh (nx, ny even)."""
    if nx < 4 or ny < 4 or nz < 1 or nx % 2 or ny % 2:
        raise ValueError("nx, ny must be even and >= 4; nz >= 1")
    hx, hy, hz = Lx / nx, Ly / ny, Lz / nz
    NX, NY, NZ = 2 * nx + 1, 2 * ny + 1, 2 * nz + 1
    a = max(1, nx // 12)
    b = max(1, ny // 6)
    i0, i1 = nx // 2 - a, nx // 2 + a
    j0, j1 = ny // 2 - b, ny // 2 + b

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    fluid = ~((ci >= i0) & (ci < i1) & (cj >= j0) & (cj < j1))
    ci, cj, ck = ci[fluid], cj[fluid], ck[fluid]
    base = np.stack([2 * ci, 2 * cj, 2 * ck], axis=1)       # lattice corner of each hexahedron

    # tetrahedra: 4 vertices + 6 edge midpoints in the half-cell lattice
    loc = []
    for tv in _kuhn_tets():
        v = 2 * tv                                           # (4, 3) lattice offsets
        mids = np.array([(v[i] + v[j]) // 2 for i, j in _TET_EDGES])
        loc.append(np.concatenate([v, mids], axis=0))        # (10, 3)
    loc = np.stack(loc)                                      # (6, 10, 3)
    LAT = (base[:, None, None, :] + loc[None, :, :, :]).reshape(-1, 10, 3)   # (E, 10, 3)
    E = LAT.shape[0]
    lin = (LAT[..., 0] * NY + LAT[..., 1]) * NZ + LAT[..., 2]

    used = np.zeros(NX * NY * NZ, dtype=bool)
    used[lin.ravel()] = True
    node_of = -np.ones(NX * NY * NZ, dtype=np.int64)
    node_lat = np.flatnonzero(used)                          # lexicographic in (ix, iy, iz)
    node_of[node_lat] = np.arange(node_lat.size)
    nn = node_lat.size
    nI = node_lat // (NY * NZ)
    nJ = (node_lat // NZ) % NY
    nK = node_lat % NZ
    tet = node_of[lin]                                       # (E, 10)

    vert_mask = (nI % 2 == 0) & (nJ % 2 == 0) & (nK % 2 == 0)
    vert_of = -np.ones(nn, dtype=np.int64)
    vert_of[vert_mask] = np.arange(int(vert_mask.sum()))
    nv = int(vert_mask.sum())
    tet_p = vert_of[tet[:, :4]]

    inlet = nI == 0
    outlet = nI == NX - 1
    ywall = (nJ == 0) | (nJ == NY - 1)
    zwall = (nK == 0) | (nK == NZ - 1)
    on_gamma = (nI >= 2 * i0) & (nI <= 2 * i1) & (nJ >= 2 * j0) & (nJ <= 2 * j1)

    # ---- dof numbering
    u_keep = np.ones((nn, 3), dtype=bool)
    u_keep[inlet, :] = False
    u_keep[ywall, 1] = False
    u_keep[zwall, 2] = False
    u_dof = -np.ones((nn, 3), dtype=np.int64)
    u_dof[u_keep] = np.arange(int(u_keep.sum()))
    nxt = int(u_keep.sum())
    blocks = {"u": (0, nxt)}
    p_dof = np.arange(nv) + nxt
    blocks["p"] = (nxt, nxt + nv)
    nxt += nv
    d_keep = np.ones((nn, 3), dtype=bool)
    d_keep[inlet | outlet, :] = False
    d_keep[ywall, 1] = False
    d_keep[zwall, 2] = False
    d_keep[on_gamma, 2] = False                              # cylinder fixed in z
    d_dof = -np.ones((nn, 3), dtype=np.int64)
    d_dof[d_keep] = np.arange(int(d_keep.sum())) + nxt
    blocks["d"] = (nxt, nxt + int(d_keep.sum()))
    nxt += int(d_keep.sum())
    g_nodes = np.flatnonzero(on_gamma)
    l_keep = np.ones((g_nodes.size, 3), dtype=bool)
    l_keep[zwall[g_nodes], 2] = False                        # no lambda_z where u_z is prescribed
    lam_dof = -np.ones((nn, 3), dtype=np.int64)
    lam_dof[g_nodes[:, None].repeat(3, 1)[l_keep], np.nonzero(l_keep)[1]] = np.arange(int(l_keep.sum())) + nxt
    blocks["lam"] = (nxt, nxt + int(l_keep.sum()))
    nxt += int(l_keep.sum())
    s_dof = np.array([nxt, nxt + 1])
    blocks["s"] = (nxt, nxt + 2)
    n = nxt + 2

    # ---- geometry (affine tetrahedra) and local matrices
    X = nI * (hx / 2)
    Y = nJ * (hy / 2)
    Z = nK * (hz / 2)
    P = np.stack([X[tet[:, :4]], Y[tet[:, :4]], Z[tet[:, :4]]], axis=-1)   # (E, 4, 3)
    rng = np.random.default_rng(seed)
    wnod = rng.uniform(-1.0, 1.0, size=(nn, 3))
    b0 = rng.standard_normal((nrhs, n))
    Avel, Ad, Bq, vol = element_blocks(P, wnod[tet], nu, alpha0)

    T = _Triplets()
    ur = _vector_rows(u_dof, tet)                            # (E,30)
    dr = _vector_rows(d_dof, tet)
    T.add(ur[:, :, None], ur[:, None, :], Avel.reshape(E, 30, 30))
    pr = p_dof[tet_p]                                        # (E,4)
    Bflat = Bq.reshape(E, 4, 30)
    T.add(pr[:, :, None], ur[:, None, :], Bflat)
    T.add(ur[:, :, None], pr[:, None, :], np.transpose(Bflat, (0, 2, 1)))
    T.add(dr[:, :, None], dr[:, None, :], Ad.reshape(E, 30, 30))
    del Avel, Ad, Bq

    # ---- Gamma: lateral faces of the cylinder, each square split along the
    # diagonal through its lowest corner (as the Kuhn tetrahedra split it)
    tq, tw = radon7()
    tphi, _, _ = p2_tri(tq)
    Mref = np.einsum("q,qi,qj->ij", tw, tphi, tphi) * 2.0    # times the triangle's area
    mref = (tw[:, None] * tphi).sum(0) * 2.0
    faces = []                                               # (corner, axis u, axis v) in the lattice
    for k2 in range(nz):
        for j in range(j0, j1):
            for ii in (i0, i1):
                faces.append(((2 * ii, 2 * j, 2 * k2), 1, 2))
        for i in range(i0, i1):
            for jj in (j0, j1):
                faces.append(((2 * i, 2 * jj, 2 * k2), 0, 2))
    step = {0: np.array([2, 0, 0]), 1: np.array([0, 2, 0]), 2: np.array([0, 0, 2])}
    m_int = np.zeros(nn)

    def nid(p):
        return node_of[(p[0] * NY + p[1]) * NZ + p[2]]

    for corner, au, av in faces:
        c0 = np.array(corner)
        cmax = c0 + step[au] + step[av]
        for third in (c0 + step[au], c0 + step[av]):
            v3 = [c0, third, cmax]
            lat = v3 + [(v3[0] + v3[1]) // 2, (v3[1] + v3[2]) // 2, (v3[2] + v3[0]) // 2]
            en = np.array([nid(p) for p in lat])
            pts = np.array([[X[e], Y[e], Z[e]] for e in en[:3]])
            area = 0.5 * np.linalg.norm(np.cross(pts[1] - pts[0], pts[2] - pts[0]))
            Me = area * Mref
            m_int[en] += area * mref
            for c in range(3):
                uu = u_dof[en, c]
                ll = lam_dof[en, c]
                T.add(uu[:, None], ll[None, :], -Me)         # -<v, lambda>
                T.add(ll[:, None], uu[None, :], -Me)         # -<mu, u>
    gl = g_nodes
    R = _Triplets()
    for c in range(2):
        T.add(lam_dof[gl, c], s_dof[c], alpha0 * m_int[gl])  # +alpha0 <mu,1> s_c
        T.add(s_dof[c], lam_dof[gl, c], m_int[gl])           # spring row: sum m_j lambda_j
        T.add(s_dof[c], s_dof[c], k)
        R.add(d_dof[gl, c], d_dof[gl, c], 1.0)              # d_c - s_c = 0 on Gamma
        R.add(d_dof[gl, c], s_dof[c], -1.0)

    drop = np.zeros(n, dtype=bool)
    drop[d_dof[gl, :2].ravel()] = True
    rr = np.concatenate(T.r)
    T.r, T.c, T.v = [np.where(drop[np.maximum(rr, 0)], -1, rr).astype(np.int32)] + R.r, \
        [np.concatenate(T.c)] + R.c, [np.concatenate(T.v)] + R.v
    del rr
    A = T.csr(n)

    meta = dict(dim=3, nx=nx, ny=ny, nz=nz, seed=seed, k=k, nu=nu, alpha0=alpha0,
                hole=(i0, i1, j0, j1), n_nodes=nn, n_vertices=nv, n_gamma_nodes=int(gl.size),
                gamma_area=float(m_int.sum()))
    return System(n=n, rowptr=A.indptr.astype(np.int64), colind=A.indices.astype(np.int32),
                  values=A.data.astype(np.float64), root=s_dof.astype(np.int32),
                  blocks=blocks, meta=meta, b0=b0)
