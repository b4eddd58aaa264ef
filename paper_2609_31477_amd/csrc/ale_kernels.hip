// Element kernels of the ALE Newton system: residual and Jacobian of every
// triangle, pseudo-solid triangle and Gamma edge, written once over a scalar
// type and evaluated either in plain doubles or in forward-mode dual numbers
// (value + one directional derivative).  One thread evaluates one element in
// one derivative direction, so the Jacobian's column j of an element comes
// from the thread seeded on its local input j; the residual is the value part.
// The terms are those of the weak form (Sec. 3.1, eq. weak_system) as the
// nonlinear functional of Sec. 3.2 collects them; the shape-derivative blocks
// come out of differentiating det J and J^{-T} (Jacobi's formula, Sec. 3.2).
#include "ale_internal.h"

namespace ale {
namespace {

struct Dual {
    double v, d;
};
__device__ inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ inline Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ inline Dual operator*(Dual a, double s) { return {s * a.v, s * a.d}; }
__device__ inline Dual operator/(Dual a, Dual b) {
    const double r = 1.0 / b.v;
    const double q = a.v * r;
    return {q, (a.d - q * b.d) * r};
}
__device__ inline Dual operator/(Dual a, double s) { return {a.v / s, a.d / s}; }
__device__ inline Dual operator+(Dual a, double s) { return {a.v + s, a.d}; }
__device__ inline Dual operator-(Dual a, double s) { return {a.v - s, a.d}; }
__device__ inline Dual dsqrt(Dual a) {
    const double r = sqrt(a.v);
    return {r, a.d / (2.0 * r)};
}
__device__ inline Dual cst(double v) { return {v, 0.0}; }

// Flow terms of one triangle on its current position (ALE, BDF1).
__device__ void triangle(const Dual (&u)[6][2], const double (&un)[6][2], const Dual (&p)[3], const Dual (&x)[3][2],
                         const double (&xn)[3][2], double nu, double dt, const Tables& T, Dual (&Ru)[6][2],
                         Dual (&Rp)[3]) {
    // J = dx/dxi (columns: edges from vertex 0), its determinant and inverse
    const Dual J00 = x[1][0] - x[0][0], J01 = x[2][0] - x[0][0];
    const Dual J10 = x[1][1] - x[0][1], J11 = x[2][1] - x[0][1];
    const Dual det = J00 * J11 - J01 * J10;
    const Dual i00 = J11 / det, i01 = -J01 / det, i10 = -J10 / det, i11 = J00 / det;
    Dual w[3][2];  // mesh velocity at the vertices
#pragma unroll
    for (int v = 0; v < 3; v++)
#pragma unroll
        for (int c = 0; c < 2; c++) w[v][c] = (x[v][c] - xn[v][c]) / dt;
#pragma unroll
    for (int i = 0; i < 6; i++) Ru[i][0] = Ru[i][1] = cst(0.0);
#pragma unroll
    for (int v = 0; v < 3; v++) Rp[v] = cst(0.0);
    for (int q = 0; q < kVolQ; q++) {
        Dual g[6][2];  // grad_x phi_i = J^{-T} grad_xi phi_i
#pragma unroll
        for (int i = 0; i < 6; i++) {
            const double a = T.dphi[q][i][0], b = T.dphi[q][i][1];
            g[i][0] = i00 * a + i10 * b;
            g[i][1] = i01 * a + i11 * b;
        }
        Dual uq[2] = {cst(0.0), cst(0.0)};
        double unq[2] = {0.0, 0.0};
        Dual G[2][2] = {{cst(0.0), cst(0.0)}, {cst(0.0), cst(0.0)}};  // G[c][a] = d u_c / d x_a
#pragma unroll
        for (int i = 0; i < 6; i++)
#pragma unroll
            for (int c = 0; c < 2; c++) {
                uq[c] = uq[c] + T.phi[q][i] * u[i][c];
                unq[c] += T.phi[q][i] * un[i][c];
                G[c][0] = G[c][0] + u[i][c] * g[i][0];
                G[c][1] = G[c][1] + u[i][c] * g[i][1];
            }
        Dual wq[2] = {cst(0.0), cst(0.0)};
        Dual pq = cst(0.0);
#pragma unroll
        for (int v = 0; v < 3; v++) {
            wq[0] = wq[0] + T.L[q][v] * w[v][0];
            wq[1] = wq[1] + T.L[q][v] * w[v][1];
            pq = pq + T.L[q][v] * p[v];
        }
        const Dual r0 = uq[0] - wq[0], r1 = uq[1] - wq[1];  // relative (convective) velocity
        Dual acc[2], sig[2][2];
#pragma unroll
        for (int c = 0; c < 2; c++) acc[c] = (uq[c] - unq[c]) / dt + r0 * G[c][0] + r1 * G[c][1];
        const Dual off = nu * (G[0][1] + G[1][0]);
        sig[0][0] = 2.0 * nu * G[0][0] - pq;
        sig[1][1] = 2.0 * nu * G[1][1] - pq;
        sig[0][1] = off;
        sig[1][0] = off;
        const Dual W = T.vw[q] * det;
#pragma unroll
        for (int i = 0; i < 6; i++)
#pragma unroll
            for (int c = 0; c < 2; c++)
                Ru[i][c] = Ru[i][c] + W * (T.phi[q][i] * acc[c] + g[i][0] * sig[c][0] + g[i][1] * sig[c][1]);
        const Dual div = G[0][0] + G[1][1];
#pragma unroll
        for (int v = 0; v < 3; v++) Rp[v] = Rp[v] - W * (T.L[q][v] * div);
    }
}

// Pseudo-solid terms of one triangle on the reference mesh (linear in x).
__device__ void solid(const Dual (&x)[3][2], const double (&X)[3][2], double lam, Dual (&R)[3][2]) {
    const double J00 = X[1][0] - X[0][0], J01 = X[2][0] - X[0][0];
    const double J10 = X[1][1] - X[0][1], J11 = X[2][1] - X[0][1];
    const double det = J00 * J11 - J01 * J10;
    const double i00 = J11 / det, i01 = -J01 / det, i10 = -J10 / det, i11 = J00 / det;
    const double dL[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
    double gL[3][2];
#pragma unroll
    for (int v = 0; v < 3; v++) {
        gL[v][0] = i00 * dL[v][0] + i10 * dL[v][1];
        gL[v][1] = i01 * dL[v][0] + i11 * dL[v][1];
    }
    Dual F[2][2];  // F[c][a] = d x_c / d X_a
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
        for (int a = 0; a < 2; a++) F[c][a] = x[0][c] * gL[0][a] + x[1][c] * gL[1][a] + x[2][c] * gL[2][a];
    const Dual e00 = F[0][0] - 1.0, e11 = F[1][1] - 1.0, e01 = 0.5 * (F[0][1] + F[1][0]);
    const Dual tr = e00 + e11;
    const Dual s00 = lam * (tr + 2.0 * e00), s11 = lam * (tr + 2.0 * e11), s01 = lam * (2.0 * e01);
    const double area = 0.5 * fabs(det);
#pragma unroll
    for (int v = 0; v < 3; v++) {
        R[v][0] = area * (gL[v][0] * s00 + gL[v][1] * s01);
        R[v][1] = area * (gL[v][0] * s01 + gL[v][1] * s11);
    }
}

// Gamma edge terms: the multiplier's work in the momentum rows, the no-slip
// constraint rows and the force in the s rows, on the current edge.
__device__ void edge(const Dual (&u)[3][2], const Dual (&lam)[3][2], const Dual (&x)[2][2], const double (&xn)[2][2],
                     double dt, const Tables& T, Dual (&Ru)[3][2], Dual (&Rl)[3][2], Dual (&Rs)[2]) {
    const Dual dx = x[1][0] - x[0][0], dy = x[1][1] - x[0][1];
    const Dual len = dsqrt(dx * dx + dy * dy);
    Dual w[2][2];
#pragma unroll
    for (int v = 0; v < 2; v++)
#pragma unroll
        for (int c = 0; c < 2; c++) w[v][c] = (x[v][c] - xn[v][c]) / dt;
#pragma unroll
    for (int j = 0; j < 3; j++) Ru[j][0] = Ru[j][1] = Rl[j][0] = Rl[j][1] = cst(0.0);
    Rs[0] = Rs[1] = cst(0.0);
#pragma unroll
    for (int q = 0; q < kEdgQ; q++) {
        const Dual W = T.ew[q] * len;
#pragma unroll
        for (int c = 0; c < 2; c++) {
            Dual uq = cst(0.0), lq = cst(0.0);
#pragma unroll
            for (int j = 0; j < 3; j++) {
                uq = uq + T.psi[q][j] * u[j][c];
                lq = lq + T.psi[q][j] * lam[j][c];
            }
            const Dual wq = T.lin[q][0] * w[0][c] + T.lin[q][1] * w[1][c];
            const Dual slip = uq - wq;
#pragma unroll
            for (int j = 0; j < 3; j++) {
                Ru[j][c] = Ru[j][c] - W * (T.psi[q][j] * lq);
                Rl[j][c] = Rl[j][c] - W * (T.psi[q][j] * slip);
            }
            Rs[c] = Rs[c] + W * lq;
        }
    }
}

__device__ inline double vel(const Dev& D, const double* U, int node, int c) {
    const int d = D.u_dof[2 * node + c];
    return d >= 0 ? U[d] : D.u_bc[2 * node + c];
}
__device__ inline double pos(const Dev& D, const double* U, int v, int c) {
    const int d = D.x_dof[2 * v + c];
    return d >= 0 ? U[d] : D.x_ref[2 * v + c];
}

// One thread per (triangle, direction); ndir = kVolIn for the Jacobian, 1 for the
// residual alone.  Direction 0 also writes the residual.
__global__ void __launch_bounds__(128) k_ale_triangle(Dev D, Tables T, const double* __restrict__ U, int ndir) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t e = t / ndir;
    const int j = (int)(t % ndir);
    if (e >= D.nelem) return;
    const int* tri = D.tri + 6 * e;
    const int* vt = D.vtx + 3 * e;
    int cdof = 0;
    if (ndir > 1) {
        cdof = j < 12 ? D.u_dof[2 * tri[j >> 1] + (j & 1)]
                      : (j < 15 ? D.p_dof[vt[j - 12]] : D.x_dof[2 * vt[(j - 15) >> 1] + ((j - 15) & 1)]);
        if (cdof < 0 && j != 0) return;  // a prescribed value has no column
    }
    const bool deriv = ndir > 1 && cdof >= 0;
    Dual u[6][2], p[3], x[3][2];
    double un[6][2], xn[3][2];
#pragma unroll
    for (int i = 0; i < 6; i++)
#pragma unroll
        for (int c = 0; c < 2; c++) {
            u[i][c] = cst(vel(D, U, tri[i], c));
            un[i][c] = D.u_prev[2 * tri[i] + c];
        }
#pragma unroll
    for (int v = 0; v < 3; v++) {
        p[v] = cst(U[D.p_dof[vt[v]]]);
#pragma unroll
        for (int c = 0; c < 2; c++) {
            x[v][c] = cst(pos(D, U, vt[v], c));
            xn[v][c] = D.x_prev[2 * vt[v] + c];
        }
    }
    if (deriv) {
#pragma unroll
        for (int i = 0; i < 12; i++)
            if (j == i) u[i >> 1][i & 1].d = 1.0;
#pragma unroll
        for (int v = 0; v < 3; v++)
            if (j == 12 + v) p[v].d = 1.0;
#pragma unroll
        for (int i = 0; i < 6; i++)
            if (j == 15 + i) x[i >> 1][i & 1].d = 1.0;
    }
    Dual Ru[6][2], Rp[3];
    triangle(u, un, p, x, xn, D.nu, D.dt, T, Ru, Rp);
    if (j == 0) {
        double* r = D.loc + D.off_volR + kVolOut * e;
#pragma unroll
        for (int i = 0; i < 12; i++) r[i] = Ru[i >> 1][i & 1].v;
#pragma unroll
        for (int v = 0; v < 3; v++) r[12 + v] = Rp[v].v;
    }
    if (deriv) {
        double* o = D.loc + D.off_volJ + (int64_t)kVolOut * (kVolIn * e + j);
#pragma unroll
        for (int i = 0; i < 12; i++) o[i] = Ru[i >> 1][i & 1].d;
#pragma unroll
        for (int v = 0; v < 3; v++) o[12 + v] = Rp[v].d;
    }
}

// One thread per triangle: the pseudo-solid residual and, when asked, its six
// columns (the block is linear, so every direction is exact).
__global__ void __launch_bounds__(128) k_ale_solid(Dev D, const double* __restrict__ U, int jacobian) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= D.nelem) return;
    const int* vt = D.vtx + 3 * e;
    double X[3][2], xv[3][2];
#pragma unroll
    for (int v = 0; v < 3; v++)
#pragma unroll
        for (int c = 0; c < 2; c++) {
            X[v][c] = D.x_ref[2 * vt[v] + c];
            xv[v][c] = pos(D, U, vt[v], c);
        }
    const double lam = D.lam_s[e];
    for (int j = 0; j < (jacobian ? kSolIn : 1); j++) {
        Dual x[3][2];
#pragma unroll
        for (int i = 0; i < 6; i++) x[i >> 1][i & 1] = {xv[i >> 1][i & 1], (jacobian && i == j) ? 1.0 : 0.0};
        Dual R[3][2];
        solid(x, X, lam, R);
        if (j == 0) {
            double* r = D.loc + D.off_solR + kSolOut * e;
#pragma unroll
            for (int i = 0; i < 6; i++) r[i] = R[i >> 1][i & 1].v;
        }
        if (jacobian) {
            double* o = D.loc + D.off_solJ + (int64_t)kSolOut * (kSolIn * e + j);
#pragma unroll
            for (int i = 0; i < 6; i++) o[i] = R[i >> 1][i & 1].d;
        }
    }
}

__global__ void __launch_bounds__(128) k_ale_edge(Dev D, Tables T, const double* __restrict__ U, int ndir) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t g = t / ndir;
    const int j = (int)(t % ndir);
    if (g >= D.nedge) return;
    const int* ge = D.gedge + 3 * g;
    const int* gv = D.gvtx + 2 * g;
    int cdof = 0;
    if (ndir > 1) {
        cdof = j < 6 ? D.u_dof[2 * ge[j >> 1] + (j & 1)]
                     : (j < 12 ? D.lam_dof[2 * ge[(j - 6) >> 1] + (j & 1)]
                               : D.x_dof[2 * gv[(j - 12) >> 1] + (j & 1)]);
        if (cdof < 0 && j != 0) return;
    }
    const bool deriv = ndir > 1 && cdof >= 0;
    Dual u[3][2], lam[3][2], x[2][2];
    double xn[2][2];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int c = 0; c < 2; c++) {
            u[i][c] = cst(vel(D, U, ge[i], c));
            const int l = D.lam_dof[2 * ge[i] + c];
            lam[i][c] = cst(l >= 0 ? U[l] : 0.0);
        }
#pragma unroll
    for (int v = 0; v < 2; v++)
#pragma unroll
        for (int c = 0; c < 2; c++) {
            x[v][c] = cst(pos(D, U, gv[v], c));
            xn[v][c] = D.x_prev[2 * gv[v] + c];
        }
    if (deriv) {
#pragma unroll
        for (int i = 0; i < 6; i++) {
            if (j == i) u[i >> 1][i & 1].d = 1.0;
            if (j == 6 + i) lam[i >> 1][i & 1].d = 1.0;
        }
#pragma unroll
        for (int i = 0; i < 4; i++)
            if (j == 12 + i) x[i >> 1][i & 1].d = 1.0;
    }
    Dual Ru[3][2], Rl[3][2], Rs[2];
    edge(u, lam, x, xn, D.dt, T, Ru, Rl, Rs);
    if (j == 0) {
        double* r = D.loc + D.off_edgR + kEdgOut * g;
#pragma unroll
        for (int i = 0; i < 6; i++) {
            r[i] = Ru[i >> 1][i & 1].v;
            r[6 + i] = Rl[i >> 1][i & 1].v;
        }
        r[12] = Rs[0].v;
        r[13] = Rs[1].v;
    }
    if (deriv) {
        double* o = D.loc + D.off_edgJ + (int64_t)kEdgOut * (kEdgIn * g + j);
#pragma unroll
        for (int i = 0; i < 6; i++) {
            o[i] = Ru[i >> 1][i & 1].d;
            o[6 + i] = Rl[i >> 1][i & 1].d;
        }
        o[12] = Rs[0].d;
        o[13] = Rs[1].d;
    }
}

// out[p] = cst[p] + the listed element values of entry p, in list order.
__global__ void __launch_bounds__(256) k_ale_sum(int64_t m, const int64_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ idx, const double* __restrict__ cstv,
                                                 const double* __restrict__ loc, double* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    double v = cstv ? cstv[p] : 0.0;
    const int64_t a = ptr[p], b = ptr[p + 1];
    for (int64_t t = a; t < b; t++) v += loc[idx[t]];
    out[p] = v;
}

// Rows that no element assembles: x - X - s on the Gamma vertices, and the
// spring term k s added to the s rows.
__global__ void __launch_bounds__(256) k_ale_fixup(Dev D, const int32_t* __restrict__ gv, int32_t ngv,
                                                   const double* __restrict__ U, double* __restrict__ R) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 2 * ngv) {
        const int v = gv[t >> 1], c = t & 1;
        const int d = D.x_dof[2 * v + c];
        R[d] = U[d] - D.x_ref[2 * v + c] - U[D.s_dof[c]];
    } else if (t < 2 * ngv + 2) {
        const int c = t - 2 * ngv;
        R[D.s_dof[c]] += D.k * U[D.s_dof[c]];
    }
}

inline unsigned blocks_for(int64_t threads, int bs) { return (unsigned)((threads + bs - 1) / bs); }

}  // namespace

hipError_t launch_elements(const Dev& D, const Tables& T, const double* U, bool jacobian, hipStream_t st) {
    const int nv = jacobian ? kVolIn : 1, ne = jacobian ? kEdgIn : 1;
    if (D.nelem > 0) {
        hipLaunchKernelGGL(k_ale_triangle, dim3(blocks_for((int64_t)D.nelem * nv, 128)), dim3(128), 0, st, D, T,
                           U, nv);
        hipLaunchKernelGGL(k_ale_solid, dim3(blocks_for(D.nelem, 128)), dim3(128), 0, st, D, U, jacobian ? 1 : 0);
    }
    if (D.nedge > 0)
        hipLaunchKernelGGL(k_ale_edge, dim3(blocks_for((int64_t)D.nedge * ne, 128)), dim3(128), 0, st, D, T, U, ne);
    return hipGetLastError();
}

hipError_t launch_sum(int64_t m, const int64_t* ptr, const int32_t* idx, const double* cstv, const double* loc,
                      double* out, hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL(k_ale_sum, dim3(blocks_for(m, 256)), dim3(256), 0, st, m, ptr, idx, cstv, loc, out);
    return hipGetLastError();
}

hipError_t launch_fixup(const Dev& D, const int32_t* gv, int32_t ngv, const double* U, double* R, hipStream_t st) {
    hipLaunchKernelGGL(k_ale_fixup, dim3(blocks_for(2 * (int64_t)ngv + 2, 256)), dim3(256), 0, st, D, gv, ngv, U, R);
    return hipGetLastError();
}

}  // namespace ale
