/*
 * opf.h -- C ABI of the MI355X condensed-space interior-point method for
 * polar AC optimal power flow (Shin, Anitescu, Pacaud, "Accelerating Optimal
 * Power Flow with GPUs: SIMD Abstraction of Nonlinear Programs and
 * Condensed-Space Interior-Point Methods", PSCC 2024).
 *
 * Conventions shared by every call:
 *  - All arithmetic is IEEE FP64; indices are int32, counts of nonzeros int64.
 *  - "host" pointers are ordinary CPU memory owned by the caller; the library
 *    copies what it needs before returning.  "device" pointers are HBM
 *    buffers owned by the caller (for example torch tensors); the library
 *    never frees them.  Every device allocation made by the library belongs to
 *    the handle that made it and is released by the matching *_destroy call.
 *  - ``stream`` is a hipStream_t passed as void* (NULL = default stream).
 *    Calls that only enqueue work return before it completes; calls that
 *    return a host-visible numeric status synchronise the stream first.
 *  - Every call returns an opf_status.  Nothing throws or aborts across the
 *    ABI; opf_last_error() returns a thread-local message for the last
 *    failure in the calling thread.
 *  - A handle is not thread-safe: use one handle per thread/stream.
 */
#ifndef OPF_H
#define OPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OPF_OK = 0,
    OPF_E_INVALID = -1,    /* bad argument, index or size */
    OPF_E_NOMEM = -2,      /* host or HBM allocation failed */
    OPF_E_DEVICE = -3,     /* HIP runtime error */
    OPF_E_STATE = -4,      /* call out of order (e.g. solve before factor) */
    OPF_E_NOT_PD = -5,     /* non-positive pivot in the Cholesky factorization */
    OPF_E_MAXITER = -6,    /* IPM iteration limit reached */
    OPF_E_LINESEARCH = -7, /* filter line search could not find an acceptable step */
    OPF_E_NUMERIC = -8,    /* NaN/Inf in an iterate or a residual */
    OPF_E_BUDGET = -9      /* a served request needs more HBM than the server's whole pool */
} opf_status;

const char* opf_last_error(void);

/* ------------------------------------------------------------------------
 * Problem data.  The polar ACOPF model the paper solves with ExaModels
 * (Section III-B lists its 15 computational patterns; Section V-A names the
 * rosetta-opf / PowerModels polar form): variables, in order,
 *   x = [va(N), vm(N), pg(G), qg(G), p(2E), q(2E)]        (n = 2N+2G+4E)
 * where arc a < E is branch a oriented from->to and arc E+l is branch l
 * oriented to->from; constraint rows, in order,
 *   reference angle (1), active flow definitions p_a - phi_p(a) (2E),
 *   reactive flow definitions (2E), angle differences va_f - va_t (E),
 *   thermal limits p_a^2 + q_a^2 (2E), active balances (N), reactive
 *   balances (N)                                             (m = 2N+1+7E).
 * Branches have tap 1, zero shift, and half the line charging at each end.
 * Per-unit data, base_mva used to convert costs given per MW.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t nbus, nbranch, ngen, ref_bus;
    double base_mva;
    /* buses [nbus]: loads, shunts, voltage-magnitude bounds (host) */
    const double *pd, *qd, *gs, *bs, *vmin, *vmax;
    /* branches [nbranch]: endpoints, series r, x, total charging b, rating, angle limits (host) */
    const int32_t *f, *t;
    const double *r, *x, *b, *rate, *angmin, *angmax;
    /* generators [ngen]: bus, cost c2 ($/MW^2h), c1 ($/MWh), c0, P/Q limits (host) */
    const int32_t* gbus;
    const double *c2, *c1, *c0, *pmin, *pmax, *qmin, *qmax;
} opf_grid;

typedef struct opf_model opf_model;

/* Options of a model.  assembly selects how the condensed matrix and the
 * sparse products J x, J^T v, W x are gathered: 0 (default) term lists sorted
 * by output and reduced by segmented wave scans, whenever the packed term
 * codes fit (nnz_jac < 2^22, n < 2^22, m < 2^20 - 2), else per-entry lists;
 * 1 always per-entry lists (one work-item per output walking its own list). */
typedef struct {
    int32_t assembly;
} opf_options;

void opf_default_options(opf_options* o);

/* Build the model templates, the fixed Jacobian/Hessian COO structure, the
 * condensed-matrix pattern and the assembly maps (host), and record their
 * upload to HBM, which runs on `stream` at the model's first device use.
 * opts NULL = defaults.  Validates sizes and bus indices (OPF_E_INVALID).
 * The grid arrays are copied; the caller may free them after the call. */
int opf_create(const opf_grid* grid, const opf_options* opts, void* stream, opf_model** out);
int opf_destroy(opf_model* model);

/* Sizes: variables, constraints, Jacobian nonzeros, Hessian (lower, with
 * duplicates) nonzeros, condensed-matrix (lower) nonzeros. */
int opf_dims(const opf_model* model, int32_t* n, int32_t* m, int64_t* nnz_jac, int64_t* nnz_hess,
             int64_t* nnz_kkt);

/* Fixed COO structure of the Jacobian (jrow/jcol [nnz_jac]) and of the lower
 * triangle of the Lagrangian Hessian (hrow >= hcol, [nnz_hess]; duplicates add)
 * in the order opf_eval_derivs writes values (host outputs). */
int opf_structure(const opf_model* model, int32_t* jrow, int32_t* jcol, int32_t* hrow, int32_t* hcol);

/* Variable bounds xl/xu [n] and constraint bounds gl/gu [m] (host; +-INFINITY
 * marks an absent bound) and the flat starting point x0 [n] (va = 0, vm = 1,
 * pg = pmax/2, qg = 0, arc flows equal to the flow functions there). */
int opf_bounds(const opf_model* model, double* xl, double* xu, double* gl, double* gu);
int opf_initial_point(const opf_model* model, double* x0);

/* Derivative evaluation over the bus, branch and generator templates
 * (Section III; Patterns 1-3 of Section II-C), one work-item per template
 * instance.  ``what`` is a bitwise OR of the OPF_EVAL_* flags; outputs whose
 * flag is clear may be NULL.  All pointers are device pointers:
 *   x [n], y [m] (multipliers, needed for OPF_EVAL_HESS),
 *   f [1]   objective value,            c [m] constraint values,
 *   grad [n] objective gradient,        jac [nnz_jac] Jacobian values,
 *   hess [nnz_hess] values of obj_weight * grad^2 f - sum_i y_i grad^2 c_i
 * (the Lagrangian L = f - y^T g of Section II-A).  Asynchronous on stream.
 * OPF_EVAL_JAC_VAR (only together with OPF_EVAL_JAC) writes just the Jacobian
 * entries that depend on x and leaves the constant ones (the unit coefficients
 * of the flow variables, the angle-difference rows, the generator and arc
 * columns of the balance rows, the reference row) as an earlier OPF_EVAL_JAC
 * call without it wrote them into the same buffer. */
enum { OPF_EVAL_F = 1, OPF_EVAL_C = 2, OPF_EVAL_GRAD = 4, OPF_EVAL_JAC = 8, OPF_EVAL_HESS = 16,
       OPF_EVAL_JAC_VAR = 32 };
int opf_eval_derivs(opf_model* model, unsigned what, const double* x, const double* y, double obj_weight,
                    double* f, double* c, double* grad, double* jac, double* hess, void* stream);

/* ------------------------------------------------------------------------
 * Condensed KKT system (Section IV-C):
 *     K = W + delta_w I + Sigma_x + J^T D J,   rhs = q_x + J^T v
 * on the fixed lower pattern returned by kkt_pattern (CSC: column pointers
 * colptr [n+1], row indices rowind [nnz_kkt], rows ascending; host outputs).
 * Pattern: the diagonal, the Hessian pattern, and every column pair of each
 * Jacobian row.  kkt_condense reads device arrays hess [nnz_hess], jac
 * [nnz_jac], sigx [n], dvec [m] and writes kval [nnz_kkt] in pattern order
 * without atomics (each entry gathers its own contributions).  If qx, v and
 * rhs are all non-NULL it also writes rhs [n] = qx [n] + J^T v [m].
 * Asynchronous on stream.
 * ---------------------------------------------------------------------- */
int kkt_pattern(const opf_model* model, int32_t* colptr, int32_t* rowind);
int kkt_condense(opf_model* model, const double* hess, const double* jac, const double* sigx, const double* dvec,
                 double delta_w, double* kval, const double* qx, const double* v, double* rhs, void* stream);

/* ------------------------------------------------------------------------
 * Pivot-free sparse Cholesky of the condensed matrix (Section IV-C: the
 * condensed matrix is positive definite exactly when the augmented system has
 * the correct inertia, so a fixed pivot sequence is valid).
 * Analysis (host, once per pattern): exact minimum degree ordering (ties to
 * the smallest index; the remaining vertices are ordered by index once the
 * minimum degree reaches dense_frac*(remaining-1) or dense_abs), elimination
 * tree, postorder (children ascending), fundamental supernodes and relaxed
 * amalgamation of a supernode into its parent when its columns directly
 * precede the parent's, the merged width is <= max_width and the explicit
 * zeros are <= zero_abs or <= zero_rel of the merged supernode's entries.
 * ---------------------------------------------------------------------- */
typedef struct {
    double dense_frac; /* default 0.5 */
    int32_t dense_abs; /* default INT32_MAX */
    int32_t max_width; /* default INT32_MAX */
    int64_t zero_abs;  /* default 64 */
    double zero_rel;   /* default 0.05 */
    /* numeric: a pivot is accepted when it exceeds pivot_tol * |K_jj| (the
     * assembled diagonal entry); default 0, i.e. when it is positive */
    double pivot_tol;
    /* fronts with at least tile_min pivots are factored by one
     * dependency-driven tile launch instead of blocked steps; 0 (default)
     * disables it: experimental, its first device run did not complete */
    int32_t tile_min;
    /* a level whose only blocked front has at least pair_min pivots pairs
     * its leading 64-column panels, as long as a pair leaves at least
     * pair_min rows below it: the first panel of a pair updates only the
     * second one's columns, the second applies both to the rest of the front
     * as one rank-128 update (half the passes over the trailing matrix);
     * default 2048, 0: never */
    int32_t pair_min;
    /* panels per group when pairing (2..8, default 2): the group's last
     * step applies all of them to the rest of the front as one update of
     * rank 64 * pair_panels */
    int32_t pair_panels;
    /* 0 (default): Cholesky, P K P^T = L L^T.  1: the LU factorization with
     * this fixed pivot sequence (the refactorization alternative of Section
     * VI), held in its symmetric form P K P^T = L D L^T (U = D L^T): L unit
     * lower, D diagonal.  A pivot is then rejected when |d| <= pivot_tol *
     * |K_jj| (pivot_tol 0: when it is zero or not finite); negative pivots
     * are accepted, so an indefinite K whose leading principal minors are
     * nonzero factors, and chol_inertia reports the signs of D.  Not with
     * tile_min > 0. */
    int32_t ldlt;
} chol_options;

typedef struct chol_sym chol_sym;

void chol_default_options(chol_options* o);
/* colptr [n+1], rowind [nnz] (host): lower CSC pattern including the diagonal. */
int chol_analyze(int32_t n, const int32_t* colptr, const int32_t* rowind, const chol_options* opts,
                 chol_sym** out);
int chol_destroy(chol_sym* sym);
/* nsuper supernodes; nnz_l stored entries of L (supernodal, explicit zeros
 * included); flops of one factorization; bytes of device factor storage. */
int chol_info(const chol_sym* sym, int32_t* nsuper, int64_t* nnz_l, double* flops, int64_t* factor_bytes);
/* Host outputs: perm [n] (perm[k] = original index of pivot k), parent [n]
 * (elimination tree in pivot order, -1 for roots), colcount [n] (nonzeros
 * of each column of L incl. the diagonal), snode_ptr [nsuper+1] (first
 * pivot of each supernode), snode_rows_ptr [nsuper+1] / snode_rows (row
 * indices, pivot order, of each supernode incl. its own columns). */
int chol_perm(const chol_sym* sym, int32_t* perm);
int chol_etree(const chol_sym* sym, int32_t* parent, int32_t* colcount);
int chol_supernodes(const chol_sym* sym, int32_t* snode_ptr);
int chol_supernode_rows(const chol_sym* sym, int64_t* rows_ptr, int32_t* rows);
/* Numeric factorization of P K P^T = L L^T (or L D L^T, see ldlt) from
 * device values kval [nnz] in the analyzed pattern's order.  Synchronises
 * the stream; returns
 * OPF_E_NOT_PD and *bad_col = pivot index of the first rejected pivot
 * (see pivot_tol; the smallest such index within the first failing
 * elimination level), else OPF_OK and *bad_col = -1.  The factor stays in
 * HBM. */
int chol_factor(chol_sym* sym, const double* kval, void* stream, int32_t* bad_col);
/* Inertia of K from the last successful factorization (host outputs): npos
 * positive and nneg negative pivots, npos + nneg = n.  By Sylvester's law of
 * inertia these are K's numbers of positive and negative eigenvalues.  A
 * Cholesky factorization succeeds only for npos = n.  OPF_E_STATE without a
 * successful factorization. */
int chol_inertia(const chol_sym* sym, int64_t* npos, int64_t* nneg);
/* Diagnostics (process-wide, since load): how many factorization and solve
 * launch sequences were captured into HIP graphs (handles an IPM owns, on a
 * stream of its own), and how many of those captures failed and were
 * enqueued as plain launches instead (e.g. when another thread's work on the
 * legacy null stream invalidated them).  Host outputs. */
int chol_graph_stats(int64_t* captures, int64_t* fallbacks);
/* x = K^{-1} b using the last successful factor; b, x device [n*nrhs]
 * (column-major, leading dimension n; x may alias b).  Returns after the
 * solve has run on `stream`: fronts with many pivots are solved by
 * work-groups that wait on each other's ready flags with a bounded spin, and
 * a wait that ran out (never expected) is reported as OPF_E_DEVICE. */
int chol_solve(chol_sym* sym, const double* b, double* x, int32_t nrhs, void* stream);
/* chol_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result as chol_solve, but the solve's working
 * vectors, the wide-front exchange blocks and the fault word live in one
 * static device array of 64 MiB per GPU instead of the handle's buffers, and
 * the call makes no hipMalloc/hipFree or other allocating call.  The array is
 * resolved to its device address once per device, on the first call with
 * that device current, and is held until the process ends.  b, x: device
 * [n*nrhs] as for chol_solve (x may alias b).  Returns OPF_E_INVALID, with a
 * message giving the bytes needed, when the factor needs more than 64 MiB of
 * solve scratch (8 bytes per row, per row-structure entry, per update row
 * and per wide-front row, about 40 MB at 80k buses); OPF_E_STATE without a
 * successful factorization; OPF_E_DEVICE if a wide-front wait ran out.  All
 * calls on one GPU share the array: calls that overlap in time on one GPU
 * (different host threads or streams) race and must be serialized by the
 * caller.  Synchronizes the stream before returning, like chol_solve. */
int chol_solve_noalloc(chol_sym* sym, const double* b, double* x, int32_t nrhs, void* stream);
/* Kernel timing of the numeric factorizations (measurement aid).  `mask`
 * selects categories by bit: 1 assembly, 2 small fronts, 4 diagonal-block
 * Cholesky, 8 panel solve, 16 trailing MFMA update, 32 dense-front tile
 * launch (0 disables).  Every launch of a selected category is bracketed by
 * HIP events on the stream it runs on (the events themselves add a little
 * latency between launches); chol_timing_read returns, per category, the
 * summed kernel milliseconds ms[6], the launch counts launches[6], and the
 * algorithmic flops flops[6] and HBM bytes bytes[6] (flops filled for the
 * trailing update, the symmetric rank-64 update of each blocked step's lower
 * triangle, and for the dense-front launch, the factorization flops of its
 * fronts; bytes for the trailing update: every updated entry read and
 * written once plus the panel rows read once per launch).  Any output
 * pointer may be null.  Calling chol_timing resets them. */
int chol_timing(chol_sym* sym, int mask);
int chol_timing_read(const chol_sym* sym, double* ms, int64_t* launches, double* flops, double* bytes);
/* Copy L to the host as CSC in pivot order over the supernodal pattern
 * (lp [n+1], li [nnz_l], lx [nnz_l]); explicit zeros included.  For an
 * L D L^T factorization (ldlt) the diagonal entries are the pivots of D and
 * the entries below are L's (whose diagonal is 1). */
int chol_export_factor(chol_sym* sym, int64_t* lp, int32_t* li, double* lx);

/* ------------------------------------------------------------------------
 * Condensed-space IPM (Algorithm 1): inequality relaxation g(x) - s = 0 with
 * equality rows relaxed to [-tol, +tol] (Section IV-A), log barrier (IV-B),
 * Newton steps through the condensed system with primal regularization for
 * inertia correction and iterative refinement on the full system (IV-C),
 * filter line search and separate primal/dual step sizes (IV-D), scaled
 * convergence test.  Line-search, scaling and barrier-update constants are
 * those of Waechter & Biegler (2006), the reference the paper defers to.
 * The iterate, slacks, multipliers and the factor stay in HBM; each iteration
 * moves a handful of scalars to the host.
 * ---------------------------------------------------------------------- */
typedef struct {
    double tol;        /* eps_tol, default 1e-4 */
    int32_t max_iter;  /* default 500 */
    int32_t max_ir;    /* iterative-refinement steps, default 10 */
    double ir_tol;     /* default 1e-10 */
    double mu_init;    /* default 0.1 */
    double bound_relax;/* default 1e-8 */
    double pivot_tol;  /* pivot acceptance of the factorizations, default 1e-12 (see chol_options) */
    /* 1 (default): when the state's stream is not the null stream, the
     * factorization's and the triangular solves' launch sequences are
     * captured once into HIP graphs and replayed (one graph launch instead of
     * one launch per kernel; same kernels, same results); 0: plain launches */
    int32_t graphs;
    /* 1: second-order correction of a rejected first trial step in the
     * filter line search (up to 4 corrections, each cutting the
     * infeasibility by 0.99, Waechter & Biegler 2006); 0 (default): off */
    int32_t soc;
} ipm_options;

typedef struct {
    int32_t iter;
    double obj;     /* unscaled objective at the iterate entering the step */
    double e0;      /* scaled optimality error with mu = 0 */
    double inf_pr;  /* scaled primal infeasibility */
    double inf_du;  /* scaled dual infeasibility */
    double mu;      /* barrier parameter used by the step */
    double delta_w; /* primal regularization used */
    double alpha;   /* primal step size */
    double alpha_z; /* bound-multiplier step size */
    int32_t ls_trials, ir_steps, factorizations;
    /* stage times of this iteration in milliseconds (device events) */
    double t_ad, t_assembly, t_factor, t_solve, t_total;
    int32_t soc_steps;  /* second-order corrections tried in the line search */
} ipm_iter_info;

typedef struct ipm_state ipm_state;

void ipm_default_options(ipm_options* o);
/* Allocates the device state for one solve of ``model``; analyzes the
 * condensed pattern with ``copts`` (NULL = defaults) and initializes the
 * iterate (flat start pushed inside the bounds, z = 1, y = 0). */
int ipm_create(opf_model* model, const ipm_options* opts, const chol_options* copts, void* stream, ipm_state** out);
int ipm_destroy(ipm_state* state);
/* One iteration of Algorithm 1.  Returns OPF_OK while iterating, 1 when the
 * convergence test holds (no step taken), or a negative status. */
int ipm_step(ipm_state* state, ipm_iter_info* info);

typedef struct {
    int32_t status;      /* 1 converged, else the negative opf_status that ended the solve */
    int32_t iterations;  /* iterations taken (steps of Algorithm 1) */
    double objective;    /* unscaled objective at the final iterate */
    double e0;           /* scaled optimality error (mu = 0) at the final iterate */
    double inf_pr, inf_du;  /* its scaled primal and dual infeasibility */
    int32_t factorizations, ir_steps;  /* totals over the solve */
    /* stage times summed over the solve, milliseconds (device events; t_total host clock) */
    double t_ad, t_assembly, t_factor, t_solve, t_total;
    /* device pointers to the final primal iterate x [n], slacks s [m] and
     * multipliers y [m]; owned by the state, valid until it is destroyed or
     * stepped again */
    const double *x, *s, *y;
} ipm_result;

/* Iterate until converged or failed and fill *out (may be NULL).  Returns
 * OPF_OK when converged, else the status that ended the solve (also in
 * out->status). */
int ipm_solve(ipm_state* state, ipm_result* out);
/* Host copies of the current primal iterate x [n], slacks s [m] and multipliers y [m]. */
int ipm_get_iterate(const ipm_state* state, double* x, double* s, double* y);
/* The analysis used by the IPM (owned by the state). */
chol_sym* ipm_chol(ipm_state* state);
/* Host copies of the whole primal-dual state: x [n], s [m], y [m], bound
 * multipliers zl, zu [n] and vl, vu [m] (0 where a bound is absent), the
 * barrier parameter and the last primal regularization (NULL outputs skipped). */
int ipm_get_state(const ipm_state* state, double* x, double* s, double* y, double* zl, double* zu, double* vl,
                  double* vu, double* mu, double* dw_last);
/* Replace the state from host arrays of the same shapes (all required, mu > 0)
 * and re-evaluate the derivatives there; the filter is kept. */
int ipm_set_state(ipm_state* state, const double* x, const double* s, const double* y, const double* zl,
                  const double* zu, const double* vl, const double* vu, double mu, double dw_last);
/* The Newton direction of the current state for its barrier parameter (the
 * direction step of an iteration: regularized factorization, condensed solve,
 * recovery, iterative refinement), without moving the iterate.  Outputs are
 * host arrays (NULL skipped); *delta_w and *ir_steps report the
 * regularization and refinement steps used. */
int ipm_direction(ipm_state* state, double* dx, double* ds, double* dy, double* dzl, double* dzu, double* dvl,
                  double* dvu, double* delta_w, int32_t* ir_steps);

/* ----------------------------------------------------------------------
 * Continuous-batching solve server (serving many ACOPF instances at once).
 *
 * The paper solves one instance at a time; this server keeps several solves
 * on the device together.  Requests (grids) arrive at any time through
 * opf_serve_submit.  A request is admitted when one of the server's worker
 * slots is free and its device footprint fits in the server's HBM pool: the
 * slot creates the request's model and IPM state (analysis on the host, all
 * device buffers carved from one region of the pool, whose size is the
 * request's exact footprint) and then runs the whole IPM (Algorithm 1) on the
 * slot's own HIP stream, so the work of admitted requests overlaps on the
 * device.  When a solve ends its region returns to the pool and the next
 * waiting request is admitted.  A request never shares a buffer with another,
 * so its result does not depend on what else is in flight.
 *
 * Ownership: the grid is copied at submission (the caller may free it after
 * the call returns).  Results stay in the server until taken with
 * opf_serve_poll / opf_serve_get_x.  The pool is one device allocation made
 * by opf_serve_create and freed by opf_serve_destroy.  A server is safe to
 * use from one host thread at a time (its workers are internal threads).
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t slots;        /* worker slots = requests on the device at once (default 8, at most 64) */
    int64_t hbm_budget;   /* bytes of the device pool (default 8 GiB) */
    ipm_options ipm;      /* options of every solve (defaults of ipm_default_options) */
    chol_options chol;    /* analysis options of every solve (defaults of chol_default_options) */
} serve_options;

typedef struct {
    int64_t tag;          /* the caller's tag from opf_serve_submit */
    int32_t status;       /* final status of the solve: 1 converged, or a negative opf_status */
    int32_t iterations;
    double objective;     /* unscaled objective at the final iterate */
    int32_t n, m;         /* variables and rows of the request's model */
    int64_t footprint;    /* device bytes the request held while admitted */
    double t_submit, t_admit, t_done;  /* host steady-clock seconds (same clock as opf_serve_now) */
    char message[160];    /* status < 0: the library's message for the failure (NUL-terminated), else "" */
} serve_result;

typedef struct opf_server opf_server;

void serve_default_options(serve_options* o);
/* Allocates the pool and starts the workers on the current device. */
int opf_serve_create(const serve_options* o, opf_server** out);
/* Queue one request.  The grid is checked and copied here (OPF_E_INVALID for
 * a bad grid, or for a tag already queued, running or holding a result); the
 * model's host structure, the analysis, admission and the solve happen on a
 * worker, so submissions do not wait for one another's host work. */
int opf_serve_submit(opf_server* srv, const opf_grid* grid, int64_t tag);
/* Up to ``max`` finished results (oldest first) into ``out``; *count receives
 * how many.  With wait != 0 the call blocks until at least one is ready or
 * nothing is queued or running. */
int opf_serve_poll(opf_server* srv, serve_result* out, int32_t max, int32_t* count, int32_t wait);
/* Host copy of the final iterate x [n] of a finished request (any time before
 * opf_serve_destroy); OPF_E_INVALID for an unknown tag or a wrong n. */
int opf_serve_get_x(opf_server* srv, int64_t tag, double* x, int32_t n);
/* Pool statistics: bytes in use now and the largest in use at once. */
int opf_serve_stats(const opf_server* srv, int64_t* in_use, int64_t* peak_in_use, int32_t* running,
                    int32_t* queued);
/* Seconds on the server's steady clock. */
double opf_serve_now(void);
/* Waits for every queued and running request, stops the workers, frees the pool. */
int opf_serve_destroy(opf_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* OPF_H */
