/*
 * mf.h -- C ABI of libmf, a multifrontal LU solver for the coupled Newton
 * Jacobian of the monolithic ALE fluid / pseudo-solid / rigid-cylinder system.
 *
 * The paper solves, at every Newton-Raphson iteration, the linear system
 * J(U_m) dU_m = -NL(U_m) (Sec. 3.4, eq. NR_iteration) with a parallel sparse
 * direct solver (Sec. 4.3).  Because the mesh, and so the sparsity pattern,
 * never changes, the analysis (ordering) is done once and every later solve is
 * a numerical factorization plus a solve (Sec. 6, "Scaling").  This library
 * follows that split:
 *
 *     mf_analyze(pattern)  -> symbolic handle (ordering, front tree, maps)
 *     mf_factor(values)    -> numeric handle (front LU factors, resident on the GPU)
 *     mf_solve(rhs, nrhs)  -> solution, with FP64 refinement to a backward-error target
 *     mf_release(handle)
 *
 * Conventions (all entry points):
 *   - Every function returns an mf_status; no exception crosses the ABI.
 *     mf_last_error() returns a thread-local message for the last failure.
 *   - Indices are 0-based.  Host arrays are read during the call only; the
 *     library copies what it keeps.
 *   - "Device" pointers are HIP device allocations (e.g. torch tensors on
 *     cuda:0); they are read or written only on the stream passed in.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Handles are not thread-safe: one call at a time per handle.
 *   - Values at the boundary are always FP64; reduced precision is internal.
 *   - Device buffers are plain pointers: the library cannot check their sizes.
 *     A buffer shorter than documented is read or written out of range, so the
 *     caller (e.g. the Python binding) checks lengths before the call.
 *
 * Hard limits (MF_ERR_ARG when exceeded, before any kernel runs on the level):
 *   - front order (nominal rows plus delayed-in columns) <= 4096: the tile work
 *     lists hold 64-row tile indices in 6 bits;
 *   - fully summed variables per front <= 8192 (the panel's row maps in 64 KB of
 *     LDS);
 *   - fronts per tree level <= 65535 (16 bits of the extend-add task code); a
 *     batch of many systems adds their levels' front counts, so batches are
 *     sized to stay below it (the serving loop splits cohorts for this).
 */
#ifndef MF_H
#define MF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MF_OK = 0,
    MF_ERR_ARG = -1,            /* bad argument (null pointer, size, index out of range) */
    MF_ERR_PATTERN = -2,        /* values/pattern do not match the symbolic handle */
    MF_ERR_OOM = -3,            /* host or device allocation failed */
    MF_ERR_SINGULAR = -4,       /* a root front column has no nonzero pivot (or NaN/Inf) */
    MF_ERR_DEVICE = -5,         /* a HIP call failed */
    MF_ERR_NOT_CONVERGED = -6,  /* refinement stopped above the target; x is still written */
    MF_ERR_STATE = -7           /* call out of order (e.g. solve before factor) */
} mf_status;

typedef enum {
    MF_FP64 = 0,  /* all fronts FP64 */
    MF_FP32 = 1,  /* non-root fronts FP32 (FP32 MFMA Schur updates); root front FP64 */
    MF_BF16 = 2   /* as MF_FP32, but Schur-update operands rounded to BF16, FP32 accumulate */
} mf_precision;

typedef struct {
    int32_t prec;          /* mf_precision of the non-root fronts (default MF_FP64) */
    double pivot_u;        /* threshold u of partial pivoting inside fronts (default 0.01) */
    int32_t leaf_max;      /* nested-dissection leaf size; part of the symbolic (default 64) */
    double target_omega;   /* componentwise backward-error target of mf_solve (default 1e-12) */
    int32_t max_outer;     /* max refinement steps (default 10) */
    int32_t gmres_m;       /* GMRES restart length / max inner iterations (default 30) */
    double gmres_tol;      /* inner relative tolerance on the preconditioned residual
                              (default 1e-12).  The inner iteration also stops as
                              soon as the refined iterate meets target_omega (its
                              true FP64 residual is checked after every inner step),
                              which normally ends it first */
    int32_t refine;        /* 0 = none, 1 = classical FP64 refinement, 2 = GMRES-IR,
                              3 = classical steps while each cuts omega at least tenfold,
                              then GMRES-IR (default -1: 1 for MF_FP64, 3 otherwise) */
    int32_t panel_nb;      /* reserved (the panel width is chosen per front from its order) */
    int32_t profile;       /* 1 = time the factorization phases with HIP events on the
                              caller's stream (reported in mf_factor_info; default 0) */
    int32_t scale;         /* Ruiz equilibration sweeps applied to the values before each
                              factorization (Ruiz 2001: rows and columns divided by the
                              square roots of their largest magnitudes, rounded to powers
                              of two so that scaling is exact); the factors are of
                              Dr J Dc and mf_solve undoes the scaling around every use of
                              them, while residuals and omega are of J itself.
                              With power-of-two factors one sweep already reaches the
                              fixed point on the Jacobians here. 0 = none; default 1 */
    int32_t plan;          /* 1 = planned schedule: after a factorization that synchronizes
                              once per tree level, the handle keeps every front's
                              delayed-in count plus slack as a capacity that fixes its
                              storage, tile lists and launch shapes, and the following
                              factorizations on the handle enqueue all levels at once with
                              a single synchronization at the end; a front that outgrows
                              its capacity makes that call factor the levels from that
                              front's level on with per-level synchronization, on top of
                              the planned levels below it (same result), and enlarges the
                              plan.  On the
                              256x128 Jacobians it is no faster: the extra empty panel
                              rounds that capacities add cost about what the per-level
                              synchronizations do.  2 = the same, with the planned
                              launches captured once into a HIP graph (on a private
                              stream) and replayed on `stream`; recaptured when the
                              plan, the pivot threshold or the scaling mode changes.
                              0 = synchronize per level; default 0 */
    int32_t tune;          /* 1 = launch-shape tuner: the first 4 factorizations on a handle
                              (level by level, not profiled) each run one combination of
                              panel block (4 or 8 waves, for fronts of order <= 512) and
                              swap tile width (16 or 64 columns) on every tree level and
                              time each level; later ones use each level's fastest.  The
                              shapes never change a result.  0 = fixed heuristics; default 0 */
    int32_t fallback;      /* 1 = when GMRES-IR on FP32/BF16 factors stops above target_omega,
                              mf_solve factors the handle again in FP64 (from its own copy of
                              the values) and solves with FP64 refinement; the handle then
                              holds FP64 factors and mf_solve_info.fp64_fallback is 1.
                              0 = return MF_ERR_NOT_CONVERGED.  Default 1 */
    int32_t sweep;         /* triangular sweeps of mf_solve: 1 = one persistent launch per direction
                              over a device task list (fronts in dependency order, tickets
                              from one counter, per-front ready counts with bounded waits;
                              large fronts split into 64-row blocks run by many work-groups);
                              0 = two launches per tree level and direction.  The two give
                              different rounding; each is deterministic.  Default 1 */
} mf_options;

/* Fill *opt with the defaults above. */
void mf_default_options(mf_options* opt);

typedef struct mf_sym* mf_sym_t;
typedef struct mf_num* mf_num_t;

/*
 * Symbolic analysis, host only.  The pattern is the paper's fixed Jacobian
 * pattern (Sec. 3.2 block structure); the analysis is a specified nested
 * dissection (George-Liu pseudo-peripheral roots, level-set separators, leaves
 * of at most leaf_max variables) whose output is bit-exactly reproducible, so
 * that it can be compared against an independent implementation.
 *
 *   n                 matrix order (>= 0)
 *   rowptr, colind    host CSR pattern, rowptr[n+1] (int64), colind[rowptr[n]]
 *                     (int32).  Column order within a row is free; duplicate
 *                     (row, col) entries are summed at factor time; explicitly
 *                     stored zeros are structural.
 *   nroot, root_idx   variables forced into the single root front, in the
 *                     order given (the two rigid-position dofs of the global
 *                     position master, Sec. 4.2).  nroot = 0 is allowed.
 *   opt               may be NULL (defaults); copied into the handle.
 *   out               receives the handle; owns copies of everything it needs.
 * Errors: MF_ERR_ARG (bad sizes or indices), MF_ERR_OOM.
 * Device memory is not touched until the first mf_factor.
 */
mf_status mf_analyze(int64_t n, const int64_t* rowptr, const int32_t* colind,
                     int32_t nroot, const int32_t* root_idx,
                     const mf_options* opt, mf_sym_t* out);

/* Read-only view of the symbolic result; arrays are owned by the handle and
 * valid until it is released.  Fronts are numbered in completion (post)order.
 * This is the analysis the paper computes once per mesh and reuses for every
 * factorization of the run (Sec. 6, "Scaling"); exporting it lets an
 * independent implementation of the same specification be compared bit for bit.
 *   perm[n]            new position -> original variable
 *   front_ptr[nf+1]    pivot ranges of each front in the new numbering
 *   front_parent[nf]   parent front, -1 for a root
 *   rows_ptr[nf+1]     ranges into rows
 *   rows[]             rows of each front as original variables: the pivots in
 *                      pivot order, then the remaining rows by ascending new index
 *   var_etree[n]       elimination tree of the permuted A + A^T (new numbering, -1 roots) */
typedef struct {
    int64_t n;
    int32_t nfronts;
    int32_t leaf_max;
    int32_t spec_version;
    int32_t nlevels;            /* height of the front tree + 1 */
    const int32_t* perm;
    const int32_t* front_ptr;
    const int32_t* front_parent;
    const int64_t* rows_ptr;
    const int32_t* rows;
    const int32_t* var_etree;
    double nominal_flops;       /* sum over fronts of sum_{i=m-p}^{m-1} (i + 2 i^2) */
    double nominal_nnz_lu;      /* sum over fronts of 2 m p - p^2 */
} mf_symbolic_view;

mf_status mf_symbolic_export(mf_sym_t sym, mf_symbolic_view* out);

/*
 * Numeric multifrontal LU of the matrix with the analyzed pattern.
 *   values_dev   device FP64 values in the CSR order given to mf_analyze
 *                (rowptr[n] entries); copied, so it may be reused after return.
 *   opt          NULL = the options given to mf_analyze; otherwise overrides the
 *                numeric options (prec, pivot_u, refinement, panel_nb).
 *   inout        if *inout is a numeric handle of the same symbolic handle its
 *                device memory is reused; if NULL a new handle is created.
 * Pivoting: threshold partial pivoting inside each front; a fully summed column
 * with no acceptable pivot among the fully summed rows is delayed to the parent
 * front (the zero pressure and multiplier diagonals of Sec. 3.2 make this
 * common).  The root front always factors in FP64 with partial pivoting.
 * Front sizes depend on the delays, so a call synchronizes with `stream` once
 * per tree level, except under options.plan once the handle has a plan: then
 * it synchronizes once.  Factors stay resident on the device.
 * Errors: MF_ERR_SINGULAR (a root column without a pivot; message names the
 * front and column), MF_ERR_DEVICE, MF_ERR_OOM, MF_ERR_ARG.
 */
mf_status mf_factor(mf_sym_t sym, const double* values_dev, const mf_options* opt,
                    void* stream, mf_num_t* inout);

typedef struct {
    int64_t delayed_pivots;     /* total delayed columns over all fronts */
    int32_t max_front;          /* largest actual front order */
    int32_t root_order;         /* actual order of the root front */
    double factor_flops;        /* nominal algorithmic flops of the factorization */
    double actual_flops;        /* flops of the actual (delay-grown) fronts */
    int64_t factor_bytes;       /* device bytes held by the fronts */
    /* filled when options.profile = 1 (milliseconds of device time, summed over levels) */
    double t_assemble_ms;       /* extend-add gather + original-entry scatter */
    double t_panel_ms;          /* panel factorization, row swaps + U12 solves, eager updates */
    double t_schur_ms;          /* deferred contribution-block (Schur) GEMMs */
    double t_finalize_ms;       /* column bookkeeping */
    double schur_flops;         /* algorithmic flops of the Schur GEMMs: sum 2 (m-P)^2 k */
    int32_t schur_launches;     /* Schur GEMM launches timed */
    int32_t levels;             /* tree levels (one host synchronization each) */
    double t_panel_kernel_ms;   /* the panel kernel alone (sum over its launches) */
    double panel_flops;         /* nominal panel flops (no delays): per window pivot, scaling + rank-1 update */
    int32_t panel_launches;     /* panel kernel launches timed */
    int32_t planned;            /* 1 if this factorization ran on the planned schedule, 2 as a graph replay */
    int32_t plan_fallbacks;     /* planned runs on this handle finished level by level (overflow) */
    int32_t tuned;              /* 1 if this factorization used the tuner's chosen shapes */
} mf_factor_info;

mf_status mf_get_factor_info(mf_num_t num, mf_factor_info* info);

/*
 * Solve J X = B with the factors: the Newton correction of eq. NR_iteration
 * (Sec. 3.4), which the paper obtains from a direct solver (Sec. 4.3).  The
 * solution is refined in FP64 until the componentwise backward error
 *     omega = max_i |B - J X|_i / (|J||X| + |B|)_i  <=  target_omega.
 *   b_dev, x_dev   device FP64, n x nrhs column-major with leading dimension ld >= n
 *                  (b_dev == x_dev is not allowed); read / written on `stream`
 *   info           may be NULL
 * Refinement: classical (x += M^{-1} r) for FP64 factors; for reduced-precision
 * factors classical steps while each cuts omega at least tenfold, then GMRES-IR
 * (left-preconditioned GMRES on M^{-1} J d = M^{-1} r, FP64 vectors, all
 * right-hand sides in lockstep), with the FP64 fallback of mf_options.fallback.  MF_ERR_NOT_CONVERGED leaves the best x
 * written.  Errors: MF_ERR_STATE (no successful mf_factor), MF_ERR_ARG,
 * MF_ERR_DEVICE, MF_ERR_OOM.
 */
typedef struct {
    double omega;               /* max over right-hand sides of the final omega */
    double omega0;              /* omega of the unrefined solution */
    int32_t outer_iters;        /* refinement steps (max over right-hand sides) */
    int32_t inner_iters;        /* total GMRES iterations */
    double eta;                 /* normwise backward error of the final x, max over right-hand
                                   sides: ||B - J X||_inf / (||J||_inf ||X||_inf + ||B||_inf) */
    int64_t delayed_pivots;     /* delayed columns of the factorization the solve used */
    int32_t fp64_fallback;      /* 1 if the solve refactored in FP64 (mf_options.fallback) */
} mf_solve_info;

mf_status mf_solve(mf_num_t num, const double* b_dev, double* x_dev, int32_t nrhs, int64_t ld,
                   void* stream, mf_solve_info* info);

/*
 * Replace the operator of a factored handle without factoring it again: later
 * solves (mf_solve, mf_solve_batched) solve J' X = B for the new values J' (same
 * pattern and CSR order as the factored values) by GMRES-IR, with the existing
 * factors, of the earlier values and in their own precision, kept only as the
 * preconditioner.  This is the iterative solver with a multifrontal
 * preconditioner that the paper names as the way past its direct solver (Sec.
 * 4.3, Sec. 7): here the preconditioner is a reduced-precision factorization
 * reused across the Newton iterations of eq. NR_iteration (Sec. 3.4), whose
 * Jacobian changes from one iteration to the next.
 *   values_dev   device FP64, nnz entries (mf_set_operator) or one array per
 *                system of a batch handle (mf_set_operator_batched); copied on
 *                `stream`, which the call synchronizes
 *   opt          NULL keeps the factorization's refinement settings; otherwise
 *                its target_omega, max_outer, gmres_m, gmres_tol, fallback and
 *                (if >= 0) refine replace them for the following solves (a cap
 *                on the iterations a reuse may spend); other fields are ignored
 * The refinement of a replaced operator is always the Krylov one (refine 1 is
 * taken as GMRES-IR; refine 0 returns the preconditioner applied once): when
 * GMRES-IR stops above the target, the fallback (if enabled) factors the new
 * values in FP64.  The next mf_factor ends the reuse and restores its own
 * options.  mf_solve_noalloc refuses a replaced operator.
 * Errors: MF_ERR_STATE (no successful factorization), MF_ERR_ARG (null values,
 * bad options, the wrong call for the handle's kind, or NaN / Inf in the values: the handle
 * must then be factored again before it solves), MF_ERR_DEVICE, MF_ERR_OOM.
 */
mf_status mf_set_operator(mf_num_t num, const double* values_dev, const mf_options* opt, void* stream);
mf_status mf_set_operator_batched(mf_num_t num, const double* const* values_dev, const mf_options* opt,
                                  void* stream);

/*
 * mf_solve without any device or pinned-host allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, layout and result as mf_solve with the
 * handle's refinement (refine 0 or 1 only: GMRES-IR's Krylov basis does not fit),
 * level-by-level sweeps, and no FP64 fallback.  Its scratch (the front vector
 * blocks, residual and correction vectors, residual maxima) comes from one
 * statically sized device array per GPU, 64 MiB, held until the process ends;
 * about 8 (sum of front orders + 3 n) bytes per right-hand side must fit, else
 * MF_ERR_ARG.  Every call on a GPU uses that GPU's one array: calls that overlap
 * on one GPU (other threads, other streams) race.
 */
mf_status mf_solve_noalloc(mf_num_t num, const double* b_dev, double* x_dev, int32_t nrhs, int64_t ld,
                           void* stream, mf_solve_info* info);

/*
 * Batches of independent systems (many uneven small Newton systems, or
 * concurrent requests of a serving loop) factor and solve in the same launches.
 * Batching is this library's extension for many concurrent parametric solves;
 * the paper factors one system at a time (its method per system is unchanged).
 *
 * mf_batch_analyze merges already-analyzed systems into one block-diagonal plan
 * (a symbolic handle of its own; the inputs may be released afterwards).  With
 * a device present, each system's pattern maps go to the current device once
 * (kept with the system's handle and shared with every batch it joins) and the
 * batch's maps are concatenated there at its first factorization; the host then
 * merges only per-front data.  Such a batch is factored on the device it was
 * analyzed on (MF_ERR_ARG otherwise).  Each
 * system keeps its own fronts, tree heights, panel shapes and root front, and
 * every reduction of the solve and of the refinement is done per system, so a
 * system's factors and solution are bitwise the same alone and in any batch.
 *   count     number of systems (>= 1)
 *   syms      count symbolic handles (from mf_analyze)
 * Errors: MF_ERR_ARG (null or foreign handles), MF_ERR_OOM.
 */
mf_status mf_batch_analyze(int32_t count, const mf_sym_t* syms, mf_sym_t* out);

/* Factor every system of a batch plan: values_dev[i] are system i's device FP64
 * values (its own CSR order).  Same semantics as mf_factor otherwise. */
mf_status mf_factor_batched(mf_sym_t batch, const double* const* values_dev, const mf_options* opt,
                            void* stream, mf_num_t* inout);

/* Solve every system of a factored batch: b_dev[i], x_dev[i] are n_i x nrhs[i]
 * column-major with leading dimension n_i (nrhs[i] >= 0; nrhs == NULL means one
 * right-hand side each).  Systems with fewer right-hand sides than the batch's
 * largest count are padded with zero columns internally (their solution is 0 and
 * needs no refinement), so every system's columns are solved exactly as alone.
 * info (may be NULL) receives one mf_solve_info per system.  MF_ERR_NOT_CONVERGED
 * if any system stopped above the target (all x are written). */
mf_status mf_solve_batched(mf_num_t num, const double* const* b_dev, double* const* x_dev, const int32_t* nrhs,
                           void* stream, mf_solve_info* info);

/* Device bytes a factorization of this pattern needs at nominal front sizes,
 * times (1 + margin) for delayed-pivot growth: the admission estimate of the
 * serving loop (a library extension; the paper's direct solver is instead given
 * a fixed relative workspace increase, 200 % in its Appendix A job settings). */
int64_t mf_footprint_bytes(mf_sym_t sym, const mf_options* opt, double margin);

/* Introspection of one factored front (for tests and debugging): copies the
 * front's state to host memory.  meta[8] = {m, P, din, k, npiv, mnom, prec, slot};
 * F_host (may be NULL) receives the m x m column-major front as FP64 (L\U, L21,
 * U12 and the contribution block); iv_host (may be NULL) receives
 * rowpiv[P], colperm[P], rowperm[P], colvar[m].  Synchronizes the device. */
mf_status mf_debug_front(mf_num_t num, int32_t front, int32_t* meta, double* F_host, int32_t* iv_host);

/* Release a symbolic or numeric handle (synchronizes its device work first).
 * NULL is ignored.  A symbolic handle must outlive its numeric handles. */
void mf_release(void* handle);

/* Thread-local message describing the last error (never NULL). */
const char* mf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MF_H */
