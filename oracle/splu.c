/*
 * Oracle sparse LU: plain left-looking LU with partial pivoting (Gilbert and
 * Peierls, 1988) and fixed-precision FP64 iterative refinement (Skeel, 1980).
 *
 * TEST INFRASTRUCTURE ONLY: linked by nothing in the solver library; loaded
 * through ctypes by oracle/splu.py for the tests, the smoke check and the
 * benchmark's CPU baseline.
 *
 * It solves the Newton system J dU = -NL(U) of the paper's Newton-Raphson
 * iteration (Sec. 3.4, eq. NR_iteration), which the paper hands to a parallel
 * direct solver (Sec. 4.3).  The matrix is first permuted symmetrically,
 * B = Q^T A Q (Q: any fill-reducing order, e.g. the oracle's nested
 * dissection), then each column k of B is computed as
 *     x = L \ B(:,k)            (sparse triangular solve, reach by DFS)
 *     pivot = argmax |x_i| over rows not yet pivotal (lowest row on ties);
 *             with a threshold tau < 1 the diagonal row k of B is kept instead
 *             whenever |x_k| >= tau * max |x_i| (threshold partial pivoting)
 *     U(:,k) = x on pivotal rows and the pivot;  L(:,k) = x / pivot elsewhere
 * so that P B = L U with unit-diagonal L.  Everything is FP64, single-threaded,
 * without blocking or BLAS.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n;
    /* L: unit diagonal not stored; row indices in B numbering until finalize,
       then in pivot numbering. */
    int64_t *Lp; int64_t *Li; double *Lx; int64_t Lcap;
    /* U: the diagonal is stored last in each column; row indices in pivot
       numbering (row k of U = the k-th pivot row). */
    int64_t *Up; int64_t *Ui; double *Ux; int64_t Ucap;
    int64_t *pinv;   /* B row -> pivot step */
    int32_t *q;      /* new -> old symmetric permutation */
    /* original matrix (for the residual) */
    const int64_t *Arp; const int32_t *Aci; double *Av;
    int64_t *Arp_copy; int32_t *Aci_copy;
} splu_t;

static int grow(void **p, int64_t *cap, int64_t need, size_t elt, void **p2, size_t elt2) {
    if (need <= *cap) return 0;
    int64_t nc = *cap ? *cap : 1024;
    while (nc < need) nc *= 2;
    void *a = realloc(*p, (size_t)nc * elt);
    if (!a) return -1;
    *p = a;
    if (p2) {
        void *b = realloc(*p2, (size_t)nc * elt2);
        if (!b) return -1;
        *p2 = b;
    }
    *cap = nc;
    return 0;
}

void splu_free(splu_t *F) {
    if (!F) return;
    free(F->Lp); free(F->Li); free(F->Lx);
    free(F->Up); free(F->Ui); free(F->Ux);
    free(F->pinv); free(F->q);
    free(F->Av); free(F->Arp_copy); free(F->Aci_copy);
    free(F);
}

/* returns 0 ok, -1 oom, -2 bad input, -4 singular (zero pivot column) */
int splu_factor(int64_t n, const int64_t *rowptr, const int32_t *colind, const double *val,
                const int32_t *q_in, double tau, splu_t **out, int64_t *fail_col) {
    *out = NULL;
    if (n < 0) return -2;
    splu_t *F = (splu_t *)calloc(1, sizeof(splu_t));
    if (!F) return -1;
    F->n = n;
    int64_t nnzA = rowptr[n];
    F->Arp_copy = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    F->Aci_copy = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnzA ? nnzA : 1));
    F->Av = (double *)malloc(sizeof(double) * (size_t)(nnzA ? nnzA : 1));
    F->q = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    F->pinv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    F->Lp = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    F->Up = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    if (!F->Arp_copy || !F->Aci_copy || !F->Av || !F->q || !F->pinv || !F->Lp || !F->Up) {
        splu_free(F); return -1;
    }
    memcpy(F->Arp_copy, rowptr, sizeof(int64_t) * (size_t)(n + 1));
    if (nnzA) {
        memcpy(F->Aci_copy, colind, sizeof(int32_t) * (size_t)nnzA);
        memcpy(F->Av, val, sizeof(double) * (size_t)nnzA);
    }
    F->Arp = F->Arp_copy; F->Aci = F->Aci_copy;
    for (int64_t i = 0; i < n; i++) F->q[i] = q_in ? q_in[i] : (int32_t)i;
    int64_t *qinv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; i++) qinv[i] = -1;
    for (int64_t i = 0; i < n; i++) {
        int32_t o = F->q[i];
        if (o < 0 || o >= n || qinv[o] >= 0) { free(qinv); splu_free(F); return -2; }
        qinv[o] = i;
    }
    /* CSC of B = Q^T A Q: column j of B = column q[j] of A with rows renumbered. */
    int64_t *Bp = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t *Bi = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnzA ? nnzA : 1));
    double *Bx = (double *)malloc(sizeof(double) * (size_t)(nnzA ? nnzA : 1));
    for (int64_t r = 0; r < n; r++)
        for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) {
            if (colind[t] < 0 || colind[t] >= n) { free(qinv); free(Bp); free(Bi); free(Bx); splu_free(F); return -2; }
            Bp[qinv[colind[t]] + 1]++;
        }
    for (int64_t j = 0; j < n; j++) Bp[j + 1] += Bp[j];
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    for (int64_t j = 0; j < n; j++) next[j] = Bp[j];
    for (int64_t r = 0; r < n; r++)
        for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) {
            int64_t j = qinv[colind[t]];
            Bi[next[j]] = qinv[r];
            Bx[next[j]] = val[t];
            next[j]++;
        }
    free(next);

    /* workspaces */
    double *x = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    int64_t *xi = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * n + 1));  /* reach stack + dfs stack */
    int64_t *pstack = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    char *mark = (char *)calloc((size_t)(n ? n : 1), 1);
    int rc = 0;
    for (int64_t i = 0; i < n; i++) F->pinv[i] = -1;

    for (int64_t k = 0; k < n; k++) {
        /* reach: DFS over L's graph from the rows of B(:,k); topological order
           is returned in xi[top..n) */
        int64_t top = n;
        for (int64_t t = Bp[k]; t < Bp[k + 1]; t++) {
            int64_t i0 = Bi[t];
            if (mark[i0]) continue;
            /* iterative DFS */
            int64_t head = 0;                 /* DFS stack lives in xi[0..head] */
            xi[0] = i0;
            while (head >= 0) {
                int64_t j = xi[head];
                int64_t jcol = F->pinv[j];
                if (!mark[j]) {
                    mark[j] = 1;
                    pstack[head] = (jcol < 0) ? 0 : F->Lp[jcol];
                }
                int done = 1;
                if (jcol >= 0) {
                    int64_t pend = F->Lp[jcol + 1];
                    for (int64_t p = pstack[head]; p < pend; p++) {
                        int64_t i = F->Li[p];
                        if (mark[i]) continue;
                        pstack[head] = p + 1;
                        xi[++head] = i;
                        done = 0;
                        break;
                    }
                }
                if (done) {
                    head--;
                    xi[--top] = j;
                }
            }
        }
        /* numeric: scatter B(:,k), then eliminate in topological order */
        for (int64_t p = top; p < n; p++) x[xi[p]] = 0.0;
        for (int64_t t = Bp[k]; t < Bp[k + 1]; t++) x[Bi[t]] += Bx[t];
        for (int64_t p = top; p < n; p++) {
            int64_t j = xi[p];
            int64_t jcol = F->pinv[j];
            if (jcol < 0) continue;
            double xj = x[j];
            for (int64_t q = F->Lp[jcol]; q < F->Lp[jcol + 1]; q++) x[F->Li[q]] -= F->Lx[q] * xj;
        }
        /* pivot: largest magnitude among non-pivotal rows, lowest row on ties */
        int64_t ipiv = -1;
        double amax = -1.0;
        for (int64_t p = top; p < n; p++) {
            int64_t i = xi[p];
            if (F->pinv[i] >= 0) continue;
            double a = fabs(x[i]);
            if (a > amax || (a == amax && i < ipiv)) { amax = a; ipiv = i; }
        }
        if (ipiv < 0 || amax == 0.0 || !isfinite(amax)) { rc = -4; if (fail_col) *fail_col = k; break; }
        /* threshold variant (tau < 1): keep the symmetric diagonal row k of B when
           it is still free and within tau of the column maximum */
        if (tau < 1.0 && F->pinv[k] < 0 && mark[k] && fabs(x[k]) >= tau * amax && x[k] != 0.0) ipiv = k;
        double piv = x[ipiv];
        int64_t cnt = n - top;
        if (grow((void **)&F->Ui, &F->Ucap, F->Up[k] + cnt + 1, sizeof(int64_t), (void **)&F->Ux, sizeof(double)) ||
            grow((void **)&F->Li, &F->Lcap, F->Lp[k] + cnt + 1, sizeof(int64_t), (void **)&F->Lx, sizeof(double))) {
            rc = -1; break;
        }
        int64_t up = F->Up[k], lp = F->Lp[k];
        for (int64_t p = top; p < n; p++) {
            int64_t i = xi[p];
            if (F->pinv[i] >= 0) {           /* U entry (row = pivot step of i) */
                F->Ui[up] = F->pinv[i]; F->Ux[up] = x[i]; up++;
            } else if (i != ipiv) {
                F->Li[lp] = i; F->Lx[lp] = x[i] / piv; lp++;
            }
            x[i] = 0.0;
            mark[i] = 0;
        }
        F->Ui[up] = k; F->Ux[up] = piv; up++;
        F->Up[k + 1] = up; F->Lp[k + 1] = lp;
        F->pinv[ipiv] = k;
    }
    if (rc == 0)   /* L row indices: B row -> pivot step */
        for (int64_t p = 0; p < F->Lp[n]; p++) F->Li[p] = F->pinv[F->Li[p]];
    free(x); free(xi); free(pstack); free(mark); free(Bp); free(Bi); free(Bx); free(qinv);
    if (rc) { splu_free(F); return rc; }
    *out = F;
    return 0;
}

int64_t splu_nnz_l(const splu_t *F) { return F->Lp[F->n]; }
int64_t splu_nnz_u(const splu_t *F) { return F->Up[F->n]; }

/* x = A^{-1} b for one right-hand side, using P Q^T A Q = L U. */
static void lu_solve1(const splu_t *F, const double *b, double *x, double *w) {
    int64_t n = F->n;
    /* w = P Q^T b : w[pinv[i]] = b[q[i]] */
    for (int64_t i = 0; i < n; i++) w[F->pinv[i]] = b[F->q[i]];
    for (int64_t j = 0; j < n; j++) {             /* L w = w (unit lower, by columns) */
        double wj = w[j];
        for (int64_t p = F->Lp[j]; p < F->Lp[j + 1]; p++) w[F->Li[p]] -= F->Lx[p] * wj;
    }
    for (int64_t j = n - 1; j >= 0; j--) {        /* U w = w (diagonal last in column) */
        int64_t pd = F->Up[j + 1] - 1;
        w[j] /= F->Ux[pd];
        double wj = w[j];
        for (int64_t p = F->Up[j]; p < pd; p++) w[F->Ui[p]] -= F->Ux[p] * wj;
    }
    for (int64_t i = 0; i < n; i++) x[F->q[i]] = w[i];   /* x = Q y */
}

/* componentwise backward error omega = max_i |b - A x|_i / (|A||x| + |b|)_i,
   with 0/0 taken as 0 (Oettli-Prager). */
static double omega_of(const splu_t *F, const double *b, const double *x, double *r) {
    double om = 0.0;
    for (int64_t i = 0; i < F->n; i++) {
        double s = b[i], d = fabs(b[i]);
        for (int64_t t = F->Arp[i]; t < F->Arp[i + 1]; t++) {
            double a = F->Av[t];
            s -= a * x[F->Aci[t]];
            d += fabs(a) * fabs(x[F->Aci[t]]);
        }
        r[i] = s;
        double w = (d > 0.0) ? fabs(s) / d : (s == 0.0 ? 0.0 : INFINITY);
        if (w > om || isnan(w)) om = w;
    }
    return om;
}

/* Solve with refinement: x0 = LU\b; while omega > tol and steps < max: x += LU\r.
   b, x: n x nrhs column-major with leading dimension n.  omega_out[c] gets the
   final backward error of column c and steps_out[c] the refinement count. */
int splu_solve(const splu_t *F, const double *b, double *x, int32_t nrhs, double tol, int32_t max_steps,
               double *omega_out, int32_t *steps_out) {
    int64_t n = F->n;
    double *w = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    double *r = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    double *d = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    if (!w || !r || !d) { free(w); free(r); free(d); return -1; }
    for (int32_t c = 0; c < nrhs; c++) {
        const double *bc = b + (int64_t)c * n;
        double *xc = x + (int64_t)c * n;
        lu_solve1(F, bc, xc, w);
        double om = omega_of(F, bc, xc, r);
        int32_t s = 0;
        while (om > tol && s < max_steps) {
            lu_solve1(F, r, d, w);
            for (int64_t i = 0; i < n; i++) xc[i] += d[i];
            om = omega_of(F, bc, xc, r);
            s++;
        }
        if (omega_out) omega_out[c] = om;
        if (steps_out) steps_out[c] = s;
    }
    free(w); free(r); free(d);
    return 0;
}
