/*
 * ale.h -- GPU assembly of the full ALE Newton system (residual and Jacobian).
 *
 * Each Newton iteration of the paper's monolithic solver solves
 *     J(U_m) dU_m = -NL(U_m)                  (Sec. 3.4, eq. NR_iteration)
 * where NL is the nonlinear functional of Sec. 3.2 (eq. nonlinear_functional)
 * built from the weak form of Sec. 3.1 (eq. weak_system) and J its Frechet
 * derivative.  Because the flow integrals live on the current mesh, J contains
 * the shape-derivative blocks A_ux, A_px and A_lambda-x that follow from Jacobi's
 * formula (Sec. 3.2).  These entry points evaluate NL(U) and J(U) on the GPU for
 * the 2D discretization of the paper (Sec. 3.3): Taylor-Hood P2-P1 flow on the
 * current mesh, the mesh position linear on the vertices, a P2 multiplier on the
 * obstacle boundary Gamma, the global position master of Sec. 4.2 (two
 * unknowns s), BDF1 in time, rho = 1 and mu_f = nu.
 *
 * Residual rows (phi_i, L_k, psi_j: P2, P1, P2-on-Gamma test functions):
 *   u rows      int_{K_t} phi_i [(u - u_prev)/dt + ((u - w).grad) u]_c
 *               + grad phi_i . sigma_f(p, u)_c  -  int_{Gamma_t} phi_i lambda_c
 *   p rows      - int_{K_t} L_k div u
 *   x rows      int_{K_0} grad_X L_v . sigma_s(x)_c; on Gamma vertices x - X - s
 *   lambda rows - int_{Gamma_t} psi_j (u - w)_c
 *   s rows      k s_c + int_{Gamma_t} lambda_c                 (eq. lambda_coupling)
 * with sigma_f = -p I + nu (grad u + grad u^T), w = (x - x_prev)/dt,
 * sigma_s = lambda_s tr(eps) I + 2 mu_s eps, eps = sym(grad_X x) - I
 * (lambda_s = mu_s per element).  Quadrature: 7-point degree-5 rule on
 * triangles, 3-point Gauss on Gamma edges.
 *
 * The element Jacobians are computed by forward-mode differentiation of the
 * element residuals (one derivative direction per thread) and summed into the
 * CSR values in a fixed order (deterministic, no atomics).
 *
 * Status codes are those of mf.h; mf_last_error() describes the last failure.
 */
#ifndef ALE_H
#define ALE_H

#include <stdint.h>

#include "mf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ale_problem* ale_t;

/* Problem description: host arrays, copied by ale_create (the caller keeps
 * ownership).  Unknown numbers are 0-based in [0, n); -1 marks a prescribed
 * value (Dirichlet velocity from u_bc, fixed position from x_ref).
 * Triangles are counter-clockwise; tri lists the three vertex nodes, then the
 * midpoints of edges (0,1), (1,2), (2,0).  Gamma edges list (end, end, midpoint)
 * nodes and the vertex numbers of their ends.  rowptr / colind is the Jacobian's
 * CSR pattern (sorted columns); it must contain every coupling of the element
 * terms, else MF_ERR_PATTERN. */
typedef struct {
    int64_t n;                  /* unknowns */
    int32_t nnodes;             /* P2 nodes */
    int32_t nvert;              /* vertices */
    int32_t nelem;              /* triangles */
    int32_t nedge;              /* Gamma edges */
    const int32_t* tri;         /* nelem x 6 node numbers */
    const int32_t* vtx;         /* nelem x 3 vertex numbers */
    const int32_t* gedge;       /* nedge x 3 node numbers */
    const int32_t* gvtx;        /* nedge x 2 vertex numbers */
    const int64_t* u_dof;       /* nnodes x 2 */
    const int64_t* p_dof;       /* nvert */
    const int64_t* x_dof;       /* nvert x 2 */
    const int64_t* lam_dof;     /* nnodes x 2 (-1 off Gamma) */
    const int64_t* s_dof;       /* 2 */
    const uint8_t* gamma_vertex; /* nvert: 1 where the x rows are x - X - s */
    const double* u_bc;         /* nnodes x 2 prescribed velocity */
    const double* u_prev;       /* nnodes x 2 previous time level */
    const double* x_ref;        /* nvert x 2 reference positions X */
    const double* x_prev;       /* nvert x 2 previous positions */
    const double* lam_s;        /* nelem pseudo-solid Lame coefficient */
    double nu, dt, k;
    const int64_t* rowptr;      /* n + 1 */
    const int32_t* colind;      /* nnz */
} ale_desc;

/* Build the device data and the fixed-order summation lists (host work plus
 * uploads, once per problem, on the current device).  The description's arrays
 * are host memory owned by the caller and copied here; they may be freed on
 * return.  Errors: MF_ERR_ARG (bad sizes or indices), MF_ERR_PATTERN (a
 * coupling missing from the pattern), MF_ERR_OOM, MF_ERR_DEVICE.
 *
 * The assembly calls below are enqueued on `stream` and return before they
 * finish.  They share the handle's element scratch, so calls on one handle must
 * be ordered (one stream, or synchronized between streams); different handles
 * are independent.  A handle is used on the device it was created on
 * (MF_ERR_ARG otherwise). */
mf_status ale_create(const ale_desc* desc, ale_t* out);

/* NL(U): U_dev and R_dev are device FP64 vectors of n entries, on `stream`. */
mf_status ale_residual(ale_t p, const double* U_dev, double* R_dev, void* stream);

/* J(U) into values_dev (device FP64, nnz entries in the pattern's order) and,
 * if R_dev is not NULL, NL(U) as well (one pass over the elements). */
mf_status ale_jacobian(ale_t p, const double* U_dev, double* values_dev, double* R_dev, void* stream);

/* Device bytes held by the problem (element scratch and summation lists). */
int64_t ale_device_bytes(ale_t p);

/* Free the handle's device data (the frees wait for the device's work).
 * NULL is ignored. */
void ale_release(ale_t p);

#ifdef __cplusplus
}
#endif
#endif
