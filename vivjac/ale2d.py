"""The full ALE Newton problem in 2D: what a Newton iteration of the paper's
monolithic solver sees (Sec. 3.1-3.4), on the structured 2D construction.

Input generation only: the mesh, the unknowns' numbering, the boundary data, a
seeded previous time level and the Jacobian's sparsity pattern.  The residual
NL(U) and its Jacobian (with the shape-derivative blocks A_ux, A_px, A_lx) are
computed elsewhere: by the CPU oracle and by the GPU assembly, independently.

Discretization (the paper's choices where it makes them):
* Taylor-Hood P2 velocity u and P1 pressure p on the current mesh, the mesh
  position x linear (P1 on the vertices, Sec. 3.3), a P2 multiplier lambda on
  the hole boundary Gamma, and the two position dofs s of the global position
  master (Sec. 4.2).
* Time: BDF1 with step dt from the previous level (u_prev, x_prev): d_t u =
  (u - u_prev)/dt at fixed reference position, mesh velocity w = (x - x_prev)/dt.
* Boundary data: inlet x = 0 fixes u = (1, 0); the slip walls y = 0, 2 fix
  u_y = 0; the outflow is natural.  The position is fixed (x = X) on the inlet
  and the outlet and slides (x_y = Y) on the walls.  The Gamma vertex rows of the
  pseudo-solid are replaced by x - X - s = 0.
* Pseudo-solid Lame coefficients lambda_s = mu_s = 1/|K_0|.
* Numbering: u (P2 nodes, lexicographic, component fastest), p (vertices), x
  (vertices, component fastest), lambda (Gamma nodes, component fastest), s.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .gen2d import gamma_edges, mesh_2d


@dataclass
class AleProblem:
    n: int
    nx: int
    ny: int
    X: np.ndarray            # (nn, 2) reference coordinates of the P2 nodes
    tri: np.ndarray          # (E, 6) P2 nodes of each triangle (vertices first)
    vtx: np.ndarray          # (E, 3) vertex numbers (0..nv-1) of each triangle
    vX: np.ndarray           # (nv, 2) reference vertex coordinates
    gedge: np.ndarray        # (nG, 3) Gamma edges: end node, end node, midpoint node
    gvtx: np.ndarray         # (nG, 2) vertex numbers of the edge ends
    u_dof: np.ndarray        # (nn, 2) unknown number or -1 (Dirichlet)
    p_dof: np.ndarray        # (nv,)
    x_dof: np.ndarray        # (nv, 2) unknown number or -1 (fixed)
    lam_dof: np.ndarray      # (nn, 2) unknown number on Gamma nodes, else -1
    s_dof: np.ndarray        # (2,)
    gamma_vertex: np.ndarray  # (nv,) bool: pseudo-solid rows replaced by x - X - s = 0
    u_bc: np.ndarray         # (nn, 2) Dirichlet velocity values (where u_dof = -1)
    u_prev: np.ndarray       # (nn, 2) previous time level (Dirichlet entries equal u_bc)
    x_prev: np.ndarray       # (nv, 2)
    lam_s: np.ndarray        # (E,) pseudo-solid Lame coefficient (lambda_s = mu_s)
    nu: float
    dt: float
    k: float
    rowptr: np.ndarray       # CSR pattern of the Jacobian
    colind: np.ndarray
    blocks: dict

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    @property
    def root(self) -> np.ndarray:
        return self.s_dof.astype(np.int32)

    def initial_guess(self) -> np.ndarray:
        """U_0: the previous velocity, zero pressure, the reference mesh, zero
        multiplier, zero cylinder displacement."""
        U = np.zeros(self.n)
        m = self.u_dof >= 0
        U[self.u_dof[m]] = self.u_prev[m]
        m = self.x_dof >= 0
        U[self.x_dof[m]] = self.vX[m]
        return U

    def perturbed_state(self, seed: int, scale: float = 1.0) -> np.ndarray:
        """A generic state for Jacobian checks: U_0 plus seeded perturbations
        (velocity, pressure, multiplier and s of order scale; free vertices moved
        by up to 0.1 scale of a cell)."""
        rng = np.random.default_rng(seed)
        U = self.initial_guess()
        b = self.blocks
        U[b["u"][0]:b["u"][1]] += 0.3 * scale * rng.uniform(-1, 1, b["u"][1] - b["u"][0])
        U[b["p"][0]:b["p"][1]] = scale * rng.uniform(-1, 1, b["p"][1] - b["p"][0])
        h = min(4.0 / self.nx, 2.0 / self.ny)
        U[b["x"][0]:b["x"][1]] += 0.1 * scale * h * rng.uniform(-1, 1, b["x"][1] - b["x"][0])
        U[b["lam"][0]:b["lam"][1]] = scale * rng.uniform(-1, 1, b["lam"][1] - b["lam"][0])
        U[b["s"][0]:b["s"][1]] = 0.01 * scale * rng.uniform(-1, 1, 2)
        # keep the Gamma vertices on the rigid motion x = X + s
        gv = np.flatnonzero(self.gamma_vertex)
        for c in range(2):
            U[self.x_dof[gv, c]] = self.vX[gv, c] + U[self.s_dof[c]]
        return U


def build_ale_2d(nx: int, ny: int, seed: int, *, nu: float = 0.01, dt: float = 0.01, k: float = 0.5,
                 Lx: float = 4.0, Ly: float = 2.0) -> AleProblem:
    m = mesh_2d(nx, ny, Lx, Ly)
    nn, nv, tri = m["nn"], m["nv"], m["tri"]
    X = np.stack([m["nI"] * (m["hx"] / 2), m["nJ"] * (m["hy"] / 2)], 1)
    vert_nodes = np.flatnonzero(m["vert_mask"])         # vertex number -> node
    vX = X[vert_nodes]
    vtx = m["vert_of"][tri[:, :3]]
    ge = gamma_edges(m)
    gvtx = m["vert_of"][ge[:, :2]]
    inlet, outlet, wall, on_gamma = m["inlet"], m["outlet"], m["wall"], m["on_gamma"]

    u_keep = np.ones((nn, 2), dtype=bool)
    u_keep[inlet, :] = False
    u_keep[wall, 1] = False
    u_dof = -np.ones((nn, 2), dtype=np.int64)
    u_dof[u_keep] = np.arange(int(u_keep.sum()))
    nxt = int(u_keep.sum())
    blocks = {"u": (0, nxt)}
    p_dof = np.arange(nv) + nxt
    blocks["p"] = (nxt, nxt + nv)
    nxt += nv
    vin, vout, vwall = inlet[vert_nodes], outlet[vert_nodes], wall[vert_nodes]
    x_keep = np.ones((nv, 2), dtype=bool)
    x_keep[vin | vout, :] = False
    x_keep[vwall, 1] = False
    x_dof = -np.ones((nv, 2), dtype=np.int64)
    x_dof[x_keep] = np.arange(int(x_keep.sum())) + nxt
    blocks["x"] = (nxt, nxt + int(x_keep.sum()))
    nxt += int(x_keep.sum())
    g_nodes = np.flatnonzero(on_gamma)
    lam_dof = -np.ones((nn, 2), dtype=np.int64)
    lam_dof[g_nodes, :] = (np.arange(2 * g_nodes.size) + nxt).reshape(-1, 2)
    blocks["lam"] = (nxt, nxt + 2 * g_nodes.size)
    nxt += 2 * g_nodes.size
    s_dof = np.array([nxt, nxt + 1])
    blocks["s"] = (nxt, nxt + 2)
    n = nxt + 2
    gamma_vertex = on_gamma[vert_nodes]

    u_bc = np.zeros((nn, 2))
    u_bc[inlet, 0] = 1.0
    rng = np.random.default_rng(seed)
    u_prev = np.stack([1.0 + 0.3 * rng.uniform(-1, 1, nn), 0.3 * rng.uniform(-1, 1, nn)], 1)
    u_prev[~u_keep] = u_bc[~u_keep]
    x_prev = vX.copy()
    P = vX[vtx]
    area0 = 0.5 * np.abs((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
                         - (P[:, 2, 0] - P[:, 0, 0]) * (P[:, 1, 1] - P[:, 0, 1]))
    lam_s = 1.0 / area0

    # ---- sparsity pattern (the couplings of the weak form, Sec. 3.2 block structure)
    rows, cols = [], []

    def couple(r, c):
        r = np.asarray(r).reshape(r.shape[0], -1)
        c = np.asarray(c).reshape(c.shape[0], -1)
        rr = np.broadcast_to(r[:, :, None], (r.shape[0], r.shape[1], c.shape[1]))
        cc = np.broadcast_to(c[:, None, :], (c.shape[0], r.shape[1], c.shape[1]))
        ok = (rr >= 0) & (cc >= 0)
        rows.append(rr[ok])
        cols.append(cc[ok])

    ue = u_dof[tri].reshape(-1, 12)
    pe = p_dof[vtx]
    xe = x_dof[vtx].reshape(-1, 6)
    flow_cols = np.concatenate([ue, pe, xe], 1)
    couple(ue, flow_cols)                                    # A_uu, A_up, A_ux
    couple(pe, np.concatenate([ue, xe], 1))                  # A_pu, A_px
    xe_rows = np.where(gamma_vertex[vtx][:, :, None], -1, x_dof[vtx]).reshape(-1, 6)
    couple(xe_rows, xe)                                      # A_xx (pseudo-solid)
    gv = np.flatnonzero(gamma_vertex)
    for c in range(2):                                       # x - X - s = 0 on Gamma vertices
        couple(x_dof[gv, c][:, None], np.stack([x_dof[gv, c], np.full(gv.size, s_dof[c])], 1))
    eu = u_dof[ge].reshape(-1, 6)
    el = lam_dof[ge].reshape(-1, 6)
    ex = x_dof[gvtx].reshape(-1, 4)
    couple(eu, np.concatenate([el, ex], 1))                  # A_ul and its x-dependence
    couple(el, np.concatenate([eu, ex], 1))                  # A_lu, A_lx
    for c in range(2):                                       # s rows: k s_c + int lambda_c
        couple(np.full((ge.shape[0], 1), s_dof[c]), np.concatenate([el[:, c::2], ex], 1))
        couple(np.array([[s_dof[c]]]), np.array([[s_dof[c]]]))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    A = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()

    return AleProblem(n=n, nx=nx, ny=ny, X=X, tri=tri, vtx=vtx, vX=vX, gedge=ge, gvtx=gvtx, u_dof=u_dof,
                      p_dof=p_dof, x_dof=x_dof, lam_dof=lam_dof, s_dof=s_dof, gamma_vertex=gamma_vertex,
                      u_bc=u_bc, u_prev=u_prev, x_prev=x_prev, lam_s=lam_s, nu=nu, dt=dt, k=k,
                      rowptr=A.indptr.astype(np.int64), colind=A.indices.astype(np.int32), blocks=blocks)
