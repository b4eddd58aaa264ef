"""Oracle for the full ALE Newton system: the residual NL(U) and its Jacobian.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The residual is the paper's nonlinear functional (Sec. 3.2, eq.
nonlinear_functional, from the weak form eq. weak_system of Sec. 3.1) with rho = 1
and mu_f = nu, discretized as described in ``vivjac.ale2d`` (P2-P1 flow on the
current mesh, P1 position, P2 multiplier on Gamma, BDF1):

  u rows   (phi_i e_c):  int_{K_t} phi_i [(u - u_prev)/dt + ((u - w).grad) u]_c
                          + grad phi_i . sigma_f(p, u)_c            - int_{Gamma_t} phi_i lambda_c
  p rows   (L_k):        - int_{K_t} L_k div u
  x rows   (L_v e_c):    int_{K_0} grad_X L_v . sigma_s(x)_c   (Gamma vertices: x - X - s)
  lambda rows (psi_j e_c): - int_{Gamma_t} psi_j (u - w)_c
  s rows:                k s_c + int_{Gamma_t} lambda_c        (eq. lambda_coupling)

with sigma_f = -p I + nu (grad u + grad u^T), w = (x - x_prev)/dt interpolated
linearly, sigma_s = lam_s tr(eps) I + 2 mu_s eps, eps = sym(grad_X x) - I
(Sec. 2), and integrals over the current configuration mapped to the reference
triangle (Sec. 3.2: dx = det J dxi, grad_x = J^{-T} grad_xi).

The Jacobian is the Frechet derivative of this residual, which the paper
assembles from Gateaux derivatives (Sec. 3.2).  Here every element's local
Jacobian is obtained by complex-step differentiation of that element's local
residual, column by column: J[:, j] = Im R(U + i h e_j) / h with h = 1e-30,
exact to rounding because the residual is analytic in U (a rational function of
the positions).  No derivative formula is written out, so the shape-derivative
blocks A_ux, A_px, A_lx come from the definition itself.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

H = 1e-30


# ---------------------------------------------------------------- reference element
def quad_triangle():
    """7-point degree-5 rule on the reference triangle (weights sum to 1/2)."""
    r = np.sqrt(15.0)
    a, b = (6.0 - r) / 21.0, (6.0 + r) / 21.0
    wa, wb = (155.0 - r) / 1200.0, (155.0 + r) / 1200.0
    pts = np.array([[1 / 3, 1 / 3], [a, a], [1 - 2 * a, a], [a, 1 - 2 * a], [b, b], [1 - 2 * b, b], [b, 1 - 2 * b]])
    return pts, np.array([9 / 40, wa, wa, wa, wb, wb, wb]) * 0.5


def basis(pts):
    """P1 values (Q,3), P1 reference gradients (3,2), P2 values (Q,6) and P2
    reference gradients (Q,6,2); P2 order: vertices, then midpoints of edges
    (0,1), (1,2), (2,0)."""
    xi, eta = pts[:, 0], pts[:, 1]
    L = np.stack([1 - xi - eta, xi, eta], 1)
    dL = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    phi = np.zeros((len(pts), 6))
    dphi = np.zeros((len(pts), 6, 2))
    for v in range(3):
        phi[:, v] = L[:, v] * (2 * L[:, v] - 1)
        dphi[:, v] = (4 * L[:, v] - 1)[:, None] * dL[v]
    for e, (a, b) in enumerate([(0, 1), (1, 2), (2, 0)]):
        phi[:, 3 + e] = 4 * L[:, a] * L[:, b]
        dphi[:, 3 + e] = 4 * (L[:, b][:, None] * dL[a] + L[:, a][:, None] * dL[b])
    return L, dL, phi, dphi


def quad_edge():
    """3-point Gauss-Legendre on [0, 1] (weights sum to 1)."""
    g = np.sqrt(0.6)
    return np.array([0.5 - 0.5 * g, 0.5, 0.5 + 0.5 * g]), np.array([5 / 18, 8 / 18, 5 / 18])


# ---------------------------------------------------------------- local residuals
def volume_local(P, u, un, xv, xnv, nu, dt):
    """Flow residual of each triangle.  u, un (E,6,2) nodal velocities; P (E,3)
    vertex pressures; xv, xnv (E,3,2) current and previous vertex positions.
    Returns (Ru (E,6,2), Rp (E,3))."""
    pts, wts = quad_triangle()
    L, dL, phi, dphi = basis(pts)
    J = np.einsum("eva,vb->eab", xv, dL)                          # d x_a / d xi_b
    det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    Jinv = np.empty_like(J)
    Jinv[:, 0, 0] = J[:, 1, 1] / det
    Jinv[:, 0, 1] = -J[:, 0, 1] / det
    Jinv[:, 1, 0] = -J[:, 1, 0] / det
    Jinv[:, 1, 1] = J[:, 0, 0] / det
    gphi = np.einsum("eba,qib->eqia", Jinv, dphi)                 # grad_x phi_i
    uq = np.einsum("qi,eic->eqc", phi, u)
    unq = np.einsum("qi,eic->eqc", phi, un)
    G = np.einsum("eic,eqia->eqca", u, gphi)                      # d u_c / d x_a
    wq = np.einsum("qv,evc->eqc", L, (xv - xnv) / dt)
    pq = np.einsum("qv,ev->eq", L, P)
    conv = np.einsum("eqa,eqca->eqc", uq - wq, G)
    eye = np.eye(2)
    sig = -pq[:, :, None, None] * eye + nu * (G + np.swapaxes(G, 2, 3))
    Wd = wts[None, :] * det[:, None]                              # (E,Q)
    Ru = np.einsum("eq,qi,eqc->eic", Wd, phi, (uq - unq) / dt + conv) \
        + np.einsum("eq,eqia,eqca->eic", Wd, gphi, sig)
    Rp = -np.einsum("eq,qv,eq->ev", Wd, L, G[:, :, 0, 0] + G[:, :, 1, 1])
    return Ru, Rp


def solid_local(xv, Xv, lam_s):
    """Pseudo-solid residual of each triangle on the reference mesh (E,3,2)."""
    dL = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    J0 = np.einsum("eva,vb->eab", Xv, dL)
    det0 = J0[:, 0, 0] * J0[:, 1, 1] - J0[:, 0, 1] * J0[:, 1, 0]
    J0inv = np.stack([np.stack([J0[:, 1, 1], -J0[:, 0, 1]], 1), np.stack([-J0[:, 1, 0], J0[:, 0, 0]], 1)], 1) \
        / det0[:, None, None]
    gL = np.einsum("eba,vb->eva", J0inv, dL)                      # grad_X L_v (E,3,2)
    F = np.einsum("evc,eva->eca", xv, gL)                         # d x_c / d X_a
    eps = 0.5 * (F + np.swapaxes(F, 1, 2)) - np.eye(2)
    tr = eps[:, 0, 0] + eps[:, 1, 1]
    sig = lam_s[:, None, None] * (tr[:, None, None] * np.eye(2) + 2.0 * eps)
    return 0.5 * np.abs(det0)[:, None, None] * np.einsum("eva,eca->evc", gL, sig)


def edge_local(u, lam, xv, xnv, dt):
    """Gamma edge terms.  u, lam (G,3,2) at (end, end, midpoint); xv, xnv (G,2,2)
    end positions.  Returns (Ru (G,3,2), Rl (G,3,2), Rs (G,2))."""
    t, w = quad_edge()
    psi = np.stack([(1 - t) * (1 - 2 * t), t * (2 * t - 1), 4 * t * (1 - t)], 1)   # (Q,3)
    lin = np.stack([1 - t, t], 1)                                                   # (Q,2)
    d = xv[:, 1] - xv[:, 0]
    Lt = np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2)
    uq = np.einsum("qj,gjc->gqc", psi, u)
    lq = np.einsum("qj,gjc->gqc", psi, lam)
    wq = np.einsum("qv,gvc->gqc", lin, (xv - xnv) / dt)
    Wl = w[None, :] * Lt[:, None]
    Ru = -np.einsum("gq,qj,gqc->gjc", Wl, psi, lq)
    Rl = -np.einsum("gq,qj,gqc->gjc", Wl, psi, uq - wq)
    Rs = np.einsum("gq,gqc->gc", Wl, lq)
    return Ru, Rl, Rs


# ---------------------------------------------------------------- global residual
def _fields(prob, U):
    dt = np.result_type(U, np.float64)
    u = prob.u_bc.astype(dt)
    m = prob.u_dof >= 0
    u[m] = U[prob.u_dof[m]]
    x = prob.vX.astype(dt)
    m = prob.x_dof >= 0
    x[m] = U[prob.x_dof[m]]
    lam = np.zeros(prob.u_dof.shape, dtype=dt)
    m = prob.lam_dof >= 0
    lam[m] = U[prob.lam_dof[m]]
    return u, U[prob.p_dof], x, lam, U[prob.s_dof]


def _add(R, dof, vals):
    ok = dof >= 0
    np.add.at(R, dof[ok], vals[ok])


def residual(prob, U):
    """NL(U) as a vector over the unknowns (real or complex U)."""
    U = np.asarray(U)
    u, p, x, lam, s = _fields(prob, U)
    R = np.zeros(prob.n, dtype=U.dtype)
    Ru, Rp = volume_local(p[prob.vtx], u[prob.tri], prob.u_prev[prob.tri], x[prob.vtx], prob.x_prev[prob.vtx],
                          prob.nu, prob.dt)
    _add(R, prob.u_dof[prob.tri], Ru)
    _add(R, prob.p_dof[prob.vtx], Rp)
    Rx = solid_local(x[prob.vtx], prob.vX[prob.vtx], prob.lam_s)
    rows = np.where(prob.gamma_vertex[prob.vtx][:, :, None], -1, prob.x_dof[prob.vtx])
    _add(R, rows, Rx)
    gv = np.flatnonzero(prob.gamma_vertex)
    for c in range(2):
        R[prob.x_dof[gv, c]] = x[gv, c] - prob.vX[gv, c] - s[c]
    ge = prob.gedge
    Eu, El, Es = edge_local(u[ge], lam[ge], x[prob.gvtx], prob.x_prev[prob.gvtx], prob.dt)
    _add(R, prob.u_dof[ge], Eu)
    _add(R, prob.lam_dof[ge], El)
    for c in range(2):
        R[prob.s_dof[c]] += prob.k * s[c] + Es[:, c].sum()
    return R


# ---------------------------------------------------------------- Jacobian
def _complex_step_columns(fn, inputs, ncol_list):
    """Columns of the local Jacobian of fn by complex steps on each local input.
    inputs: list of real arrays (E, ...); ncol_list: their flattened sizes per
    element.  Returns a list over inputs of arrays (E, out, ncols) per output."""
    base = [np.asarray(a, dtype=np.complex128) for a in inputs]
    cols = []
    for which, a in enumerate(base):
        E = a.shape[0]
        flat = a.reshape(E, -1)
        per_out = None
        for j in range(flat.shape[1]):
            pert = flat.copy()
            pert[:, j] += 1j * H
            args = list(base)
            args[which] = pert.reshape(a.shape)
            outs = fn(*args)
            if per_out is None:
                per_out = [np.zeros((E, o.reshape(E, -1).shape[1], flat.shape[1])) for o in outs]
            for k, o in enumerate(outs):
                per_out[k][:, :, j] = o.reshape(E, -1).imag / H
        cols.append(per_out)
    return cols


def jacobian(prob, U):
    """The Jacobian at U as a scipy CSR matrix (n x n), assembled from local
    complex-step Jacobians; its entries lie in the problem's pattern."""
    U = np.asarray(U, dtype=np.float64)
    u, p, x, lam, s = _fields(prob, U)
    tri, vtx = prob.tri, prob.vtx
    rr, cc, vv = [], [], []

    def emit(row_dofs, col_dofs, block):
        E = block.shape[0]
        r = np.broadcast_to(row_dofs.reshape(E, -1, 1), block.shape)
        c = np.broadcast_to(col_dofs.reshape(E, 1, -1), block.shape)
        ok = (r >= 0) & (c >= 0)
        rr.append(r[ok])
        cc.append(c[ok])
        vv.append(block[ok])

    # volume terms: inputs (P, u, x) -> outputs (Ru, Rp)
    un, xnv = prob.u_prev[tri], prob.x_prev[vtx]
    cols = _complex_step_columns(lambda P_, u_, x_: volume_local(P_, u_, un, x_, xnv, prob.nu, prob.dt),
                                 [p[vtx], u[tri], x[vtx]], None)
    row_u, row_p = prob.u_dof[tri], prob.p_dof[vtx]
    for (blk_u, blk_p), col_d in zip(cols, [prob.p_dof[vtx], prob.u_dof[tri], prob.x_dof[vtx]]):
        emit(row_u, col_d, blk_u)
        emit(row_p, col_d, blk_p)
    # pseudo-solid (rows of non-Gamma vertices)
    (blk,), = _complex_step_columns(lambda x_: (solid_local(x_, prob.vX[vtx], prob.lam_s),), [x[vtx]], None)
    rows = np.where(prob.gamma_vertex[vtx][:, :, None], -1, prob.x_dof[vtx])
    emit(rows, prob.x_dof[vtx], blk)
    # Gamma vertex rows x - X - s
    gv = np.flatnonzero(prob.gamma_vertex)
    for c in range(2):
        d = prob.x_dof[gv, c]
        rr += [d, d]
        cc += [d, np.full(gv.size, prob.s_dof[c])]
        vv += [np.ones(gv.size), -np.ones(gv.size)]
    # Gamma edges: inputs (u, lam, x) -> outputs (Ru, Rl, Rs)
    ge, gvt = prob.gedge, prob.gvtx
    xn = prob.x_prev[gvt]
    cols = _complex_step_columns(lambda u_, l_, x_: edge_local(u_, l_, x_, xn, prob.dt),
                                 [u[ge], lam[ge], x[gvt]], None)
    srow = np.broadcast_to(prob.s_dof[None, :], (ge.shape[0], 2))
    for (bu, bl, bs), col_d in zip(cols, [prob.u_dof[ge], prob.lam_dof[ge], prob.x_dof[gvt]]):
        emit(prob.u_dof[ge], col_d, bu)
        emit(prob.lam_dof[ge], col_d, bl)
        emit(srow, col_d, bs)
    for c in range(2):
        rr.append(np.array([prob.s_dof[c]]))
        cc.append(np.array([prob.s_dof[c]]))
        vv.append(np.array([prob.k]))
    A = sp.coo_matrix((np.concatenate(vv), (np.concatenate(rr), np.concatenate(cc))), shape=(prob.n, prob.n))
    return A.tocsr()


def pattern_values(prob, A):
    """The values of A in the problem's CSR pattern order; raises if A has a
    nonzero outside the pattern."""
    A = A.tocoo()
    n = np.int64(prob.n)
    prow = np.repeat(np.arange(prob.n, dtype=np.int64), np.diff(prob.rowptr))
    pkeys = prow * n + prob.colind
    akeys = A.row.astype(np.int64) * n + A.col
    j = np.minimum(np.searchsorted(pkeys, akeys), pkeys.size - 1)
    inside = pkeys[j] == akeys
    if np.any(A.data[~inside] != 0.0):
        raise AssertionError(f"{int(np.count_nonzero(A.data[~inside]))} Jacobian entries outside the pattern")
    out = np.zeros(prob.nnz)
    np.add.at(out, j[inside], A.data[inside])
    return out
