/*
 * l1ls.h -- C ABI of the MI355X (gfx950) solver core for l1-regularised
 * least squares,
 *
 *     minimise  f_tau(x) = tau * ||x||_1 + 0.5 * ||A x - b||_2^2      (1)
 *
 * (Fountoulakis & Gondzio, arXiv:1503.03520, section 1, problem (1)), on
 * instances from the paper's scalable generator (section 3.1 Procedure
 * IGen with the SVD-known A = Q Sigma G^T of eq. (16), section 4).
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers (HBM of the current HIP
 *    device); all other pointers are host pointers.
 *  - Vectors are dense, contiguous, 0-based.  x-like vectors have n FP64
 *    entries, b-like vectors m FP64 entries, unless stated otherwise.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Every call returns an l1ls_status; nothing aborts, exits or throws
 *    across the ABI.  On an error return no output is written and the
 *    objects passed in stay valid.
 *  - Objects (l1ls_instance, l1ls_fista) are owned by the library; the
 *    caller releases them with the matching *_free / *_destroy call.
 *    Caller-owned buffers are never retained after a call returns.
 *  - Calls on different objects may run concurrently on different streams.
 *    Calls on the same object must not overlap.
 */
#ifndef L1LS_H
#define L1LS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    L1LS_OK = 0,
    L1LS_NOT_CONVERGED = 1,  /* max_iter reached; outputs are valid */
    L1LS_E_ARG = -1,         /* invalid argument (sizes, NULL, ranges) */
    L1LS_E_NOMEM = -2,       /* device allocation failed */
    L1LS_E_HIP = -3,         /* a HIP runtime call failed */
    L1LS_E_NONFINITE = -4,   /* NaN/Inf met in the data or the iterates */
    L1LS_E_STATE = -5,       /* object not in a state that allows the call */
    L1LS_E_UNSUPPORTED = -6  /* option combination not built */
} l1ls_status;

/* Arithmetic of the bulk iteration. */
typedef enum { L1LS_F32 = 0, L1LS_F64 = 1 } l1ls_precision;

/* Operator used for products with A and A^T. */
typedef enum {
    L1LS_OP_STORED = 0,      /* stored CSR (A x) and CSC (A^T y) */
    L1LS_OP_MATRIX_FREE = 1, /* Givens stages applied on the fly (MvPA/MvPAt) */
    L1LS_OP_BLOCKED = 2      /* stored runs of four (L1LS_STORE_BLK32), FP32 only */
} l1ls_operator;

/* Row/column order of the stored CSR/CSC.  NATURAL: A as defined.  STAGE:
 * rows ordered by the m-side bijection pi_m and columns by pi_n (position p
 * holds original index pi(p)), so that every Givens stage pairs neighbours
 * and the gathers of a row (column) fall into runs of consecutive entries.
 * The order is internal: every entry point takes and returns vectors in
 * the original order of A. */
typedef enum { L1LS_LAYOUT_NATURAL = 0, L1LS_LAYOUT_STAGE = 1 } l1ls_layout;

/* Storage kept by l1ls_generate_ex (bit mask). */
#define L1LS_STORE_F32 1u    /* CSR + CSC values in FP32 (int32 indices)   */
#define L1LS_STORE_F64 2u    /* CSR + CSC values in FP64 (same indices)     */
/* Blocked A for two stages in the STAGE layout.  With G = S_2 S_1 and
 * Q = S~_2 S~_1 (eq. (16)), A is the sum over the middle indices i < n of
 * sigma_i (Q e_i)(G e_i)^T, and Q e_i, G e_i each cover four consecutive
 * stage positions (section 4.2 pairs).  Every row of A is then stored as
 * 0..4 runs (one int32 start and four FP32 values each) and every column as
 * exactly four, 20 bytes per four entries against 32 for CSR/CSC; values
 * are rounded once from FP64 per term, so they differ from the CSR/CSC
 * values (sums of terms) by FP32 rounding.  Requires rounds = 2,
 * layout = STAGE and n >= 4 (else L1LS_E_UNSUPPORTED). */
#define L1LS_STORE_BLK32 4u
/* Windowed gathers for the fused matrix-free passes (FISTA and CG-Newton with
 * L1LS_OP_MATRIX_FREE).  Each random gather of the Sigma embedding becomes a
 * bucketing pass, which copies the gathered vector so that the elements read
 * by each window of consecutive target positions lie together, followed by
 * a gather within the window.  That costs about 16 bytes per element more,
 * and saves the whole cache line that a random load costs once the vector
 * outgrows the caches.  Built when this bit is set, and always for
 * n >= 2^22; results are bitwise those of the plain gathers.  Extra device
 * memory: 4 (m + 5n) bytes for the tables, and the solvers' matrix-free
 * buffers hold the bucketed copies (n entries each). */
#define L1LS_STORE_MF_WINDOWS 8u
/* Windowed gathers for the stored FP32 FISTA passes (with L1LS_STORE_F32):
 * the CSR pass gathers x, and the CSC pass r_y, at a few runs of four
 * consecutive positions per row (column) at random places, a cache line per
 * run once the vector outgrows the caches.  With this bit each pass's
 * targets are grouped in windows (about 2^20 stored entries each), and a
 * bucketing pass before it copies the gathered vector in units of 4
 * consecutive elements so that each window's units lie in whole cache lines
 * (one copy per window that reads a unit); the pass then gathers inside
 * those lines, which stay in the L2 of the XCD that runs the window.
 * Results are bitwise those of the plain passes.  Extra device memory:
 * 4 bytes per stored entry for each pass's positions in the copy, 2 bytes
 * per unit, and the bucketed copies in the solver (16 bytes per unit; about
 * n units per pass at two stages).  L1LS_E_UNSUPPORTED when a copy would
 * reach 4 GiB. */
#define L1LS_STORE_WINDOWS 32u

typedef struct {
    int32_t rounds;      /* Givens stages per side, 1 or 2 (nnz/col <= 4^rounds) */
    uint32_t storage;    /* L1LS_STORE_* mask; 0 = matrix-free only            */
    void* stream;        /* stream the build runs on                            */
    int32_t layout;      /* l1ls_layout of the stored CSR/CSC                   */
} l1ls_gen_opts;

/* Read-only description of an instance.  Device pointers stay valid until
 * l1ls_free.  CSR/CSC pointers are NULL when that storage was not built. */
typedef struct {
    int64_t m, n, s, nnz;
    int32_t rounds;
    uint32_t storage;
    int32_t layout;      /* l1ls_layout of the CSR/CSC below                    */
    double kappa, tau;
    double L;            /* lambda_max(A^T A) = sigma_1^2 (= 1)                 */
    double f_star;       /* f_tau(x*) = tau ||x*||_1 + 0.5 ||e||^2              */
    uint64_t seed;
    const double* b_dev;       /* m  */
    const double* x_star_dev;  /* n, planted minimiser                         */
    const double* g_dev;       /* n, subgradient chosen in IGen step 2         */
    const double* e_dev;       /* m, e = b - A x*                               */
    const double* sigma_dev;   /* n, singular values                            */
    const int32_t* support_dev;/* s, supp(x*) in draw order                     */
    const int32_t* perm_n_dev; /* n, bijection pi of the n side                 */
    const int32_t* perm_m_dev; /* m, bijection pi of the m side                 */
    const double* cs_n_dev[2]; /* per stage: n/2 pairs of (c, s), interleaved   */
    const double* cs_m_dev[2]; /* per stage: m/2 pairs of (c, s), interleaved   */
    /* Stored A in `layout` order: row r of the CSR is original row pi_m(r),
     * column c original column pi_n(c) (identity for NATURAL). */
    const int32_t* csr_ptr_dev;  /* m+1 */
    const int32_t* csr_col_dev;  /* nnz, sorted within each row    */
    const float* csr_val32_dev;  /* nnz */
    const double* csr_val64_dev; /* nnz */
    const int32_t* csc_ptr_dev;  /* n+1 */
    const int32_t* csc_row_dev;  /* nnz, sorted within each column */
    const float* csc_val32_dev;  /* nnz */
    const double* csc_val64_dev; /* nnz */
} l1ls_info;

typedef struct l1ls_instance l1ls_instance;

/*
 * Source of the library's device memory (a contract of this boundary; the
 * paper has nothing to say on memory management).  Every block the library
 * allocates (instances, solver workspaces and iterates,
 * temporaries, batch slots, the serving pool's blocks) comes from
 * alloc(ctx, bytes) once an allocator is installed, and goes back through
 * free(ctx, ptr, bytes) to the allocator that made it, even after another
 * one has been installed.  alloc returns NULL when it cannot serve the
 * request (the call then fails with L1LS_E_NOMEM).  Before it calls free the
 * library waits for the device (as hipFree does), so the allocator may hand
 * the block to any stream at once.  The callbacks may run on the library's
 * worker threads (the serving loop).  NULL restores hipMalloc / hipFree for
 * new blocks.  L1LS_E_ARG when alloc or free is NULL.  The Python binding
 * installs PyTorch's caching allocator.  l1ls_objective_gap_noalloc never
 * calls the allocator.
 */
typedef struct {
    void* (*alloc)(void* ctx, size_t bytes);
    void (*free)(void* ctx, void* ptr, size_t bytes);
    void* ctx;
} l1ls_allocator;
l1ls_status l1ls_set_allocator(const l1ls_allocator* allocator);

/*
 * Build an instance on the current device (section 3.1 Procedure IGen with
 * A = Q Sigma G^T, eq. (16), section 4):
 *   sigma_j = kappa^(-(j-1)/(n-1)); G, Q = `rounds` Givens stages of random
 *   disjoint pairs with angles uniform on [0, 2 pi); x* has s nonzeros at
 *   random positions with N(0,1) values; g = sign(x*) on the support and
 *   U[-0.9, 0.9] elsewhere; e = tau Q Sigma^{+T} G^T g; b = A x* + e.
 * All random draws come from Philox-4x32-10 keyed by `seed`, so an instance
 * is a function of (m, n, kappa, s, tau, seed, rounds).
 * Requires m >= n >= 2, m and n even, m < 2^31, 0 <= s <= n, kappa >= 1,
 * tau > 0, 1 <= rounds <= 2; with the CSR/CSC stored also 16 n < 2^31 and
 * m < 2^29 (else L1LS_E_UNSUPPORTED).  l1ls_generate uses rounds = 1, both
 * storages and the STAGE layout on the null stream.  The call returns after
 * the build finished.
 *
 * m < n builds Procedure IGen2 (section 3.2) instead: B (m x m) is the
 * instance above with n = m, x* (s <= m nonzeros) and g lie in its columns
 * and e = tau B^{-T} g; column k of N (m x (n-m)) is a copy of column p(k) of
 * B, p injective over the columns j with |g_j| >= 1/2 (a random bijection of
 * that list), rescaled by step 4 to N~_k = xi_k tau / |N_k^T e| N_k, xi_k
 * uniform on [-1, 1]; A = [B, N~] and b = A x* + e (x* is zero on N~).
 * Then A^T e = tau g with g_{m+k} = xi_k sign(N_k^T e), and the instance's
 * L = 1 + max_k (xi_k tau / |N_k^T e|)^2 bounds lambda_max(A^T A).  Only the
 * stored operator exists (A has no rotation form): rounds must be 1 and the
 * storage must include a CSR/CSC (F32 and/or F64; the FP64 copy is always
 * kept), without BLK32 or MF_WINDOWS (else L1LS_E_UNSUPPORTED); m >= 2
 * even, 0 <= s <= m, and n - m at most the number of B's columns with
 * |g_j| >= 1/2 (about 0.44 m + s; else L1LS_E_ARG).  The rotation tables and
 * sigma in l1ls_info describe B.
 */
l1ls_status l1ls_generate(int64_t m, int64_t n, double kappa, int64_t s,
                          double tau, uint64_t seed, l1ls_instance** out);
l1ls_status l1ls_generate_ex(int64_t m, int64_t n, double kappa, int64_t s,
                             double tau, uint64_t seed, const l1ls_gen_opts* opts,
                             l1ls_instance** out);
l1ls_status l1ls_instance_info(const l1ls_instance* inst, l1ls_info* out);
/* Device bytes the instance holds (the sum of its blocks as requested from
 * the allocator); 0 for NULL. */
size_t l1ls_instance_bytes(const l1ls_instance* inst);
void l1ls_free(l1ls_instance* inst);

/*
 * Products with the instance's operator (section 4, Algorithms MvPA and
 * MvPAt, or the stored CSR/CSC of the same A):
 *   trans = 0: out_dev (m) = A in_dev (n);  trans = 1: out_dev (n) = A^T in_dev (m).
 * prec selects the value type of in_dev/out_dev and of the arithmetic
 * (float for L1LS_F32, double for L1LS_F64).  Asynchronous on `stream`.
 */
l1ls_status l1ls_apply(const l1ls_instance* inst, int32_t trans, int32_t op,
                       int32_t prec, const void* in_dev, void* out_dev, void* stream);

/*
 * Duality gap of problem (1) at x (FP64 stored operator):
 *   P = f_tau(x), r = A x - b, theta = min(1, tau/||A^T r||_inf),
 *   D = -0.5 ||theta r||^2 - b^T (theta r)  (Lasso dual, a lower bound on
 *   the optimum of (1)),  rel_gap = (P - D)/|P|.
 * Outputs are host doubles; the call synchronises `stream`.
 */
l1ls_status l1ls_objective_gap(const l1ls_instance* inst, double tau, const double* x_dev,
                               double* primal, double* dual, double* rel_gap, void* stream);

/*
 * l1ls_objective_gap for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops that must not call hipMalloc,
 * harnesses that forbid it): the same kernels and the same result, bit for
 * bit, with every temporary (x in operator order, r, the partial sums) in a
 * fixed scratch array of the library (about 12 MB on each device it runs
 * on, held until the process ends) instead of fresh allocations.  The call
 * allocates nothing, neither device nor host memory.
 *   Limit: m <= 2^19 (524288); larger instances give L1LS_E_ARG before any
 *   HIP call.  Needs the FP64 stored operator (else L1LS_E_UNSUPPORTED).
 *   The scratch is shared by every call on one device: calls that overlap on
 *   the same device (from other threads or on other streams) race and must
 *   be serialised by the caller.  Synchronises `stream`.
 */
l1ls_status l1ls_objective_gap_noalloc(const l1ls_instance* inst, double tau, const double* x_dev,
                                       double* primal, double* dual, double* rel_gap, void* stream);

typedef struct {
    double tau;            /* <= 0: the instance's tau                          */
    double rel_gap_tol;    /* stop when (P - D)/|P| <= tol; 0: run max_iter     */
    int64_t max_iter;
    int32_t check_every;   /* gap evaluated every this many iterations (>= 1)   */
    int32_t precision;     /* l1ls_precision of the bulk iteration              */
    int32_t op;            /* l1ls_operator                                     */
    int32_t polish;        /* FP64 polish of the reduced problem (13) at the end:
                              0 never, 1 always, 2 only when the FP64 gap of
                              the FISTA result exceeds rel_gap_tol; a polish
                              whose result has a larger objective f_tau than
                              its starting point (by more than 1e-12 relative,
                              the FP64 rounding of f_tau) returns the
                              starting point */
    double L;              /* <= 0: the instance's L (sigma_1^2)                 */
    const double* x0_dev;  /* n, warm start; NULL: x0 = 0                       */
    void* stream;
    int32_t time_kernels;  /* 1: accumulate per-kernel HIP-event times          */
    /* CG-Newton only (section 8.1 item pdNCG, section 8.3): */
    double mu;             /* pseudo-Huber parameter; <= 0: 1e-5                */
    double pcg_rtol;       /* <= 0: 0.1                                         */
    int32_t max_backtrack; /* <= 0: 50                                          */
    int32_t pcg_maxit;     /* <= 0: 1000                                        */
    int32_t hessian;       /* 0: primal-dual diagonal, 1: exact primal Hessian  */
    /* Batch only: rounds of 4 tiles per workgroup task; 0: chosen per slot
     * size by the library's autotuner (timed on a slot's first pass). */
    int32_t tile_chunk;
    /* l1ls_sgt_solve_fista / _pcdm only: stop once f_tau(x_k) <= f_target (0: off). */
    double f_target;
    /* l1ls_sgt_solve_pcdm only: probability that a coordinate is updated in a step (<= 0: 1). */
    double pcdm_p;
    /* Batch only: 1 = enqueue whole check periods as one HIP graph (captured
     * once per set of resident slots, replayed; the kernels read the
     * iteration count from device memory), 0 = launch every kernel.  The
     * iterates are the same bit for bit. */
    int32_t graph;
    /* Batch only: slots with at most this many rows run all of an iterate
     * call's iterations in one launch, one workgroup per slot (workgroup
     * barriers only), beside the shared passes of the larger slots; 0: the
     * library's default (none), -1: never.  The iterates are the same bit for
     * bit. */
    int32_t persist_rows;
    /* l1ls_solve_pcdm only: coordinates updated together in a step (section
     * 8.3's varpi), 1 <= varpi <= min(n, 1024); 0: 40. */
    int32_t pcdm_tau_nice;
} l1ls_solve_opts;

typedef struct {
    int64_t iterations;    /* FISTA iterations, or Newton steps                 */
    int64_t inner;         /* total PCG iterations (CG-Newton, polish)          */
    double primal, dual, rel_gap;   /* FP64 gap at the returned x              */
    double rel_err;        /* ||x - x*|| / ||x*|| against the planted x*        */
    double seconds;        /* wall time of the solve                             */
    int32_t converged;
    int32_t polish_rounds;
} l1ls_report;

/* Fill opts with defaults: tau from the instance, tol 1e-8, 10000 iters,
 * check every 32, FP64, stored operator, no polish. */
void l1ls_solve_opts_default(l1ls_solve_opts* opts);

/*
 * FISTA (section 8.1; separable model (4) with H = L I, exact
 * soft-threshold step of section 2) from x0, then optionally the FP64
 * polish.  x_out_dev receives n FP64 values.  Returns L1LS_OK when the
 * relative gap reached rel_gap_tol, L1LS_NOT_CONVERGED at max_iter.
 * opts.op selects the operator: STORED (CSR/CSC in opts.precision),
 * MATRIX_FREE (requires m times the value size below 4 GiB) or BLOCKED
 * (L1LS_STORE_BLK32, FP32 only); L1LS_E_UNSUPPORTED when the instance lacks
 * what the choice needs.  FP64 solves on the stored operator whose CSR, CSC
 * and iterates fit in one compute unit's LDS run in a single workgroup; the
 * iterates are those of the multi-kernel passes bit for bit.
 */
l1ls_status l1ls_solve_fista(const l1ls_instance* inst, const l1ls_solve_opts* opts,
                             double* x_out_dev, l1ls_report* report);

/*
 * Second-order path (section 2, problem (8) with the pseudo-Huber function
 * (7) and Newton model (9); section 8.1 item pdNCG, section 8.3): Newton
 * directions from preconditioned CG with the inverse Hessian diagonal as
 * preconditioner, relative residual pcg_rtol, Armijo backtracking of at most
 * max_backtrack halvings; then the FP64 polish if opts.polish.  With
 * opts.precision = L1LS_F32 the Hessian-vector products of the Newton
 * directions read the FP32 values of A (vectors, gradients and all sums stay
 * FP64; both storages are needed).  The Newton
 * loop stops when ||grad f_mu(x)||_inf <= rel_gap_tol * tau, or after
 * max_iter Newton steps (report.iterations; report.inner = PCG iterations).
 * opts.op = L1LS_OP_STORED uses the stored FP64 operator (L1LS_STORE_F64).
 * opts.op = L1LS_OP_MATRIX_FREE applies A and A^T from the rotation tables
 * (Algorithms MvPA / MvPAt, section 4), so it needs no stored A: vectors and
 * sums are FP64, and with precision L1LS_F32 the Hessian products of the
 * Newton directions read the FP32 copies of the rotation coefficients and
 * sigma; it requires the STAGE layout and 8 m < 2^32, and the final
 * certificate (report.primal / dual / rel_gap) is evaluated with FP64
 * products; opts.polish still needs L1LS_STORE_F64.
 * L1LS_E_UNSUPPORTED for other combinations.
 */
l1ls_status l1ls_solve_cg_newton(const l1ls_instance* inst, const l1ls_solve_opts* opts,
                                 double* x_out_dev, l1ls_report* report);

/*
 * PCDM (section 8.1 item PCDM, section 8.3) on the stored FP64 operator:
 * step k updates varpi = opts.pcdm_tau_nice coordinates, each by the exact
 * minimiser of its separable model at the current x,
 *   x_i <- soft(x_i - A_i^T (A x - b) / (beta L_i), tau / (beta L_i)),
 *   L_i = (A^T A)_ii, beta = 1 + (omega - 1)(varpi - 1)/(n - 1), omega the
 *   largest number of nonzeros in a row of A,
 * all from the same x (a synchronous step; the paper's cores update
 * asynchronously), then keeps r = A x - b up to date on the rows those
 * columns touch.  The varpi coordinates form a tau-nice sample: original
 * indices pi_e((k mod q) varpi + j), j < varpi, e = k div q, q = n div varpi,
 * with pi_e the generator's Feistel bijection of [0, n) under the instance's
 * seed and counter tag 0x10000 + e.  From opts.x0_dev (NULL: 0).  Every
 * opts.check_every steps (and at the end) the FP64 gap is evaluated; the
 * solve stops when it is <= opts.rel_gap_tol (> 0) or after opts.max_iter
 * steps (report.iterations).  Needs L1LS_STORE_F64, precision L1LS_F64, op
 * L1LS_OP_STORED, polish 0 (else L1LS_E_UNSUPPORTED); L1LS_E_ARG for varpi
 * outside [1, min(n, 1024)] or more than 65534 epochs.
 */
l1ls_status l1ls_solve_pcdm(const l1ls_instance* inst, const l1ls_solve_opts* opts, double* x_out_dev,
                            l1ls_report* report);

/*
 * lambda_max(A^T A), the Lipschitz constant L of the gradient of
 * 0.5 ||A x - b||^2 (section 8.1 uses it as the FISTA step 1/L), by the
 * power method in FP64: v_0 = v0_dev / ||v0_dev|| (n values in the original
 * order, device; NULL: the all-ones vector), then `iters` steps
 * w = A^T (A v), lambda = v^T w, v = w / ||w||; *lambda_out receives the
 * last lambda.  The generator's sigma law gives L = sigma_1^2 = 1 in closed
 * form (l1ls_info.L); this is the estimate for operators without one.  op is
 * L1LS_OP_STORED (needs L1LS_STORE_F64) or L1LS_OP_MATRIX_FREE (STAGE
 * layout).  L1LS_E_ARG for iters < 1 or a zero start, L1LS_E_UNSUPPORTED
 * when the operator is not available.  Blocks until done.
 */
l1ls_status l1ls_power_iteration(const l1ls_instance* inst, int32_t op, int32_t iters,
                                 const double* v0_dev, double* lambda_out, void* stream);

/*
 * Stepping interface of FISTA (the iteration above, state kept on the
 * device).  create: x_0 = x0 (or 0), one residual pass.  iterate: enqueue
 * `iters` iterations on opts.stream without synchronising; once the gap test
 * has passed, further iterations are no-ops on the device.  report:
 * synchronises and returns the last evaluated gap.  get_x: copies the
 * current iterate (FP64) to x_out_dev.
 */
typedef struct l1ls_fista l1ls_fista;
l1ls_status l1ls_fista_create(const l1ls_instance* inst, const l1ls_solve_opts* opts,
                              l1ls_fista** out);
l1ls_status l1ls_fista_iterate(l1ls_fista* st, int64_t iters);
l1ls_status l1ls_fista_report(l1ls_fista* st, l1ls_report* report);
l1ls_status l1ls_fista_get_x(l1ls_fista* st, double* x_out_dev);
/* Per-kernel HIP-event times (ms, summed) and launch counts accumulated since
 * create when opts.time_kernels = 1: [0] residual pass (CSR A x),
 * [1] transpose pass (CSC A^T r + prox), [2] gap evaluation. */
l1ls_status l1ls_fista_kernel_times(l1ls_fista* st, double ms[3], int64_t launches[3]);
/* The same for `count` slots (1..5): [3] the bucketing pass of x and [4] of
 * r_y of the windowed stored passes (L1LS_STORE_WINDOWS; zero otherwise). */
l1ls_status l1ls_fista_kernel_times_ex(l1ls_fista* st, int32_t count, double* ms, int64_t* launches);
void l1ls_fista_destroy(l1ls_fista* st);

/*
 * Batched FISTA (the iteration of l1ls_solve_fista, FP32 bulk, stored
 * operator) over many instances in shared launches.  Each slot keeps its own
 * iteration count, momentum and gap state on the device, so instances may be
 * added and removed between calls (continuous batching); a slot's iterates and
 * its convergence test do not depend on which other slots are resident.
 *   create: capacity slots; hbm_budget_bytes > 0 makes batch_add refuse
 *           (L1LS_E_NOMEM) an instance whose l1ls_instance_footprint would
 *           exceed the budget; opts: rel_gap_tol, check_every, stream
 *           (precision must be L1LS_F32, op L1LS_OP_STORED).
 *   add:    admit an instance (not owned; it must outlive its slot) with its
 *           tau (<= 0: the instance's); x_0 = 0; returns the slot.
 *           L1LS_E_STATE when no slot is free.
 *   iterate: enqueue `iters` iterations of every running slot (async).
 *   poll:   synchronise; reports[capacity] (iterations = -1 for free slots;
 *           converged = 1 once the gap test passed); *active_out = slots
 *           still iterating.
 *   get_x:  the slot's current iterate (FP64, original order) to x_out_dev.
 *   remove: free the slot and its buffers.
 */
typedef struct l1ls_batch l1ls_batch;
l1ls_status l1ls_batch_create(int32_t capacity, size_t hbm_budget_bytes, const l1ls_solve_opts* opts,
                              l1ls_batch** out);
l1ls_status l1ls_batch_add(l1ls_batch* batch, const l1ls_instance* inst, double tau, int32_t* slot_out);
/* As l1ls_batch_add, with this slot's own relative-gap tolerance
 * (rel_gap_tol < 0: the batch's; 0: never converge) and iteration cap
 * (max_iter <= 0: none; at the cap the slot stops with converged = 0 and
 * iterations = max_iter).  L1LS_E_ARG for a NaN tolerance. */
l1ls_status l1ls_batch_add_ex(l1ls_batch* batch, const l1ls_instance* inst, double tau, double rel_gap_tol,
                              int64_t max_iter, int32_t* slot_out);
l1ls_status l1ls_batch_iterate(l1ls_batch* batch, int64_t iters);
l1ls_status l1ls_batch_poll(l1ls_batch* batch, l1ls_report* reports, int32_t* active_out);
l1ls_status l1ls_batch_get_x(l1ls_batch* batch, int32_t slot, double* x_out_dev);
l1ls_status l1ls_batch_remove(l1ls_batch* batch, int32_t slot);
void l1ls_batch_destroy(l1ls_batch* batch);
/* Device bytes an instance occupies while resident in a batch (its stored
 * operator, vectors and the slot's iterates): the admission footprint. */
size_t l1ls_instance_footprint(const l1ls_instance* inst);
/*
 * Serving: a FIFO queue of solve requests in front of batches (continuous
 * batching).  A request names an instance of Procedure IGen (section 3.1;
 * the arguments of l1ls_generate, with the stage-order layout and FP32
 * storage) and its own tolerance and iteration cap.  Requests are grouped
 * by size (n < 2^14, n < 2^18, larger), with a FIFO queue per group; each
 * group's residents are a batch on a stream of its own, so small requests
 * iterate at their own rate while large ones run.  The largest group holds
 * one resident at a time (its iterations alone saturate HBM).  Each tick
 *   1. enqueues iterations of every group: the slowest at least
 *      iters_per_tick, the others as many as fit the same time (multiples of
 *      check_every);
 *   2. admits, oldest first, group-queue heads while fewer than max_slots
 *      are resident, the group is below its limit and the head's estimated
 *      footprint (l1ls_request_footprint) fits hbm_budget_bytes (0: no
 *      budget); admission generates the instance on the device;
 *   3. retires requests whose gap test passed, whose iterate went
 *      non-finite, or which reached max_iter: the iterate (FP64, original
 *      order) moves to a result buffer held until l1ls_server_take, and the
 *      slot and instance are freed.
 * A request with flags & L1LS_REQ_FP64_FINISH is generated with the FP64
 * operator as well; on retirement a worker thread of the server (its own
 * stream) evaluates the FP64 gap of the iterate and, when it exceeds
 * rel_gap_tol, runs the FP64 polish of the reduced problem (13) (section
 * 3.2), exactly as l1ls_solve_fista with polish = 2; the result is then the
 * one that function returns for the same instance, tolerance, check period
 * and max_iter, and its report carries the FP64 gap (converged = 1 when it
 * is within rel_gap_tol).  Such requests count against the budget until
 * finished.
 * A result is bit-identical to the one the request gets alone in the server,
 * and to l1ls_solve_fista (FP32, the same tolerance and check period) on the
 * same instance.  report.seconds of a taken result is the time from
 * submission to retirement (host steady clock).
 *   create: 1 <= max_slots <= 65535, iters_per_tick >= 1, check_every >= 1
 *           (gap test period of every request); stream (NULL: default)
 *           orders the copies of take.
 *   submit: L1LS_E_ARG for an invalid request (the checks of l1ls_generate,
 *           rounds 1 or 2, rel_gap_tol > 0, max_iter > 0), L1LS_E_NOMEM if its
 *           estimate alone exceeds the budget; *id_out is its id (0, 1, ...).
 *   tick:   *admitted / *completed (either may be NULL) count this tick's
 *           admissions and retirements.  Returns after the tick's work.
 *   completed: copies up to cap ids retired since the last call into ids,
 *           oldest first; returns how many.
 *   take:   copies the result of a retired id to x_out_dev (n FP64; NULL to
 *           drop it) and its report, then frees it; L1LS_E_STATE if the id is
 *           not retired or already taken.
 *   stats:  queued requests, resident requests (in a batch or being
 *           finished), estimated bytes resident.
 */
typedef struct l1ls_server l1ls_server;
typedef struct {
    int64_t m, n;
    double kappa;
    int64_t s;
    double tau;
    uint64_t seed;
    int32_t rounds;
    int32_t flags;         /* L1LS_REQ_FP64_FINISH: see below                   */
    double rel_gap_tol;
    int64_t max_iter;
} l1ls_request;
#define L1LS_REQ_FP64_FINISH 1
l1ls_status l1ls_server_create(int32_t max_slots, size_t hbm_budget_bytes, int32_t iters_per_tick,
                               int32_t check_every, void* stream, l1ls_server** out);
l1ls_status l1ls_server_submit(l1ls_server* server, const l1ls_request* req, int64_t* id_out);
l1ls_status l1ls_server_tick(l1ls_server* server, int32_t* admitted, int32_t* completed);
int32_t l1ls_server_completed(l1ls_server* server, int64_t* ids, int32_t cap);
l1ls_status l1ls_server_take(l1ls_server* server, int64_t id, double* x_out_dev, l1ls_report* rep);
l1ls_status l1ls_server_stats(l1ls_server* server, int32_t* queued, int32_t* resident, size_t* used_bytes);
void l1ls_server_destroy(l1ls_server* server);
/* The admission estimate of a request (bytes): l1ls_instance_footprint of its
 * FP32 instance with nnz at its bound; 0 for an invalid request or NULL. */
size_t l1ls_request_footprint(const l1ls_request* req);

/* Solve `count` instances together (taus may be NULL); x_outs[i] receives
 * n_i FP64 values; reports[i] per instance.  L1LS_OK when all converged. */
l1ls_status l1ls_solve_fista_batched(const l1ls_instance* const* insts, const double* taus, int32_t count,
                                     const l1ls_solve_opts* opts, double* const* x_outs, l1ls_report* reports);

/*
 * Regularisation path (section 8.6 varies tau): FISTA for k <= 64 values of
 * tau on one instance at once, FP32 bulk over the stored operator, all
 * columns from x_0 = 0.  X_out_dev receives n x k FP64 values, column-major
 * (column c is the solution for taus[c], original order); reports[c] per
 * column.  opts: rel_gap_tol, max_iter, check_every, L, stream, and polish:
 * 0 returns the FP32 iterates with the device's gap; 2 finishes each column
 * in FP64 at its tau (the FP64 gap of the FP32 result, the FP64 polish of the
 * reduced problem (13) where it misses rel_gap_tol, then the FP64 gap of the
 * result in reports[c]); 1 polishes every column.  A polish that raises the
 * objective f_tau (beyond 1e-12 relative) leaves the column as it was.  polish needs
 * L1LS_STORE_F64 (else L1LS_E_UNSUPPORTED).
 */
l1ls_status l1ls_solve_fista_path(const l1ls_instance* inst, const double* taus, int32_t k,
                                  const l1ls_solve_opts* opts, double* X_out_dev, l1ls_report* reports);

/* ---------------------------------------------------------------------------
 * The A = Sigma G^T instance class of sections 8.4 to 8.9 (Table 1).
 *
 * A = Sigma G^T with m >= n rows (m = 2n in all of these experiments) and
 * rank n: Sigma has sigma_1..sigma_n on its top n x n diagonal and zeros
 * below (section 4); G is the product of the n/2 Givens rotations
 * G(2k-1, 2k, theta), k = 1..n/2, on adjacent pairs with one shared angle
 * (section 4.1 without Q-side rotations or permutation), G(i, j, theta)
 * mapping (z_i, z_j) to (c z_i - s z_j, s z_i + c z_j).
 *   sigma_law ALTERNATING (section 8.9): sigma_i = sigma_odd for odd i and
 *     sigma_even for even i (1-based).
 *   sigma_law UNIFORM (sections 8.4 to 8.6): sigma_i = u_i sigma_scale +
 *     sigma_shift, u_i uniform on [0, 1) (the sections' [0, 10^q] shifted by
 *     0.1: sigma_scale = 10^q, sigma_shift = 0.1); pair k draws Philox
 *     counter (k, 0, 0x500, 0), words (0, 1) for element 2k, (2, 3) for 2k+1.
 *   xstar_law TABLE1 (section 8.9): s nonzeros at the first s outputs of the
 *     support bijection (the Philox-keyed Feistel bijection of
 *     l1ls_generate); the first floor(s/2) are x_neg, the rest x_pos.
 *   xstar_law OSGEN (section 6, Procedure OsGen): the same positions, values
 *     gamma (2u - 1), u from the x* counter of l1ls_generate.
 *   xstar_law OSGEN3 (section 6, Procedure OsGen3): x = G gamma (Sigma^T
 *     Sigma)^{-1} 1_n (the exact minimiser of eq. (19)); its s1 smallest and
 *     s2 largest components in the order (|x_i|, i) are kept, s1 + s2 = s.
 * The subgradient g is sign(x*) on the support and U[-0.9, 0.9] elsewhere;
 * e = tau Sigma^{+T} G^T g and b = A x* + e (Procedure IGen, section 3.1).
 * A is block diagonal with one 2 x 2 block per pair and rows n..m-1 of A
 * and b are zero: the library stores the top n entries of b only (8 n
 * bytes) and recomputes sigma, x* and g from (seed, index) where it needs
 * them.
 *
 * m < n selects Procedure IGen2 (section 3.2): A = [B, N~] with B (m x m) =
 * Sigma_B G_B^T as above over the first m columns and N (m x (n - m)),
 * n - m <= m, = [Sigma_N G_N^T; 0] on the same adjacent pairs (uniform law:
 * Philox counter (k, 1, 0x500, 0) for N's pair k); x* has its s <= m
 * nonzeros among the first m components (TABLE1 or OSGEN law over [0, m));
 * g (eq. (14)) is defined on the first m; e = tau B^{-T} g; N~_j = xi_j tau /
 * |N_j^T e| N_j with xi_j = 2u - 1 from Philox counter (j, 0, 0x700, 0);
 * b = A x* + e (m entries).  The n - m column scales are stored (8 bytes
 * each).  kappa_rho is not defined for m < n (L1LS_E_UNSUPPORTED).
 *
 * Device vectors passed to these calls must be 16-byte aligned
 * (L1LS_E_ARG otherwise).  Calls on the same instance must not overlap.
 * ------------------------------------------------------------------------- */
enum { L1LS_SIGMA_ALTERNATING = 0, L1LS_SIGMA_UNIFORM = 1 };
enum { L1LS_XSTAR_TABLE1 = 0, L1LS_XSTAR_OSGEN = 1, L1LS_XSTAR_OSGEN3 = 2 };

typedef struct l1ls_sgt l1ls_sgt;

typedef struct {
    int64_t n;          /* variables: even, 2 <= n <= 2^32                      */
    int64_t m;          /* rows: even; m >= n (section 8.9: 2n), or IGen2 with  */
                        /* n/2 <= m < n                                         */
    int64_t s;          /* nonzeros of x*, 0 <= s <= min(m, n) (8.9: n / 2^10)  */
    double theta;       /* angle of every rotation of G (section 8.9: 2 pi / 3) */
    double sigma_odd;   /* sigma_i, odd i (section 8.9: 0.1); > 0               */
    double sigma_even;  /* sigma_i, even i (section 8.9: 100); > 0              */
    double x_neg;       /* first floor(s/2) support values (section 8.9: -1e4)  */
    double x_pos;       /* other support values (section 8.9: 0.1)              */
    double tau;         /* > 0 (section 8.3: 1)                                 */
    uint64_t seed;
    int32_t sigma_law;  /* L1LS_SIGMA_*                                         */
    int32_t xstar_law;  /* L1LS_XSTAR_*                                         */
    double sigma_scale; /* UNIFORM: >= 0 (sections 8.4-8.6: 10^q)               */
    double sigma_shift; /* UNIFORM: > 0 (sections 8.4-8.6: 0.1)                 */
    double gamma;       /* OSGEN, OSGEN3: > 0 (8.4: 10, 1e3; 8.5, 8.6: 100)     */
    int64_t s1, s2;     /* OSGEN3: smallest / largest kept, s1 + s2 = s         */
} l1ls_sgt_params;

typedef struct {
    l1ls_sgt_params params;
    double L;            /* lambda_max(A^T A) = max(sigma_odd, sigma_even)^2      */
    double f_star;       /* f_tau(x*) = tau ||x*||_1 + 0.5 ||e||^2               */
    double c, s_rot;     /* cos theta, sin theta as used by the kernels          */
    const double* b_dev; /* n: the top n entries of b (the others are zero)       */
    double sigma_min, sigma_max; /* of B's (m >= n: A's) singular values; kappa(A^T A) =
                                    (sigma_max / sigma_min)^2 when m >= n (section 5) */
    const double* colscale_dev;  /* IGen2: the n - m column scales xi_j tau / |N_j^T e| of N~; else NULL */
} l1ls_sgt_desc;

/* params = the section 8.9 values for n: m = 2n, s = floor(n / 1024),
 * theta = 2 pi / 3, ALTERNATING sigma 0.1 / 100, TABLE1 x* values -1e4 /
 * 0.1, tau = 1 (and sigma_scale 1, sigma_shift 0.1, gamma 1, s1 = floor(s/2),
 * s2 = s - s1 for the other laws). */
void l1ls_sgt_params_default(int64_t n, uint64_t seed, l1ls_sgt_params* params);
/* Device bytes of an instance, and the extra device bytes of a CG-Newton
 * solve on it (besides the caller's x): 8 n + O(1) and 40 n + O(1). */
size_t l1ls_sgt_bytes(int64_t n);
size_t l1ls_sgt_solve_bytes(int64_t n);

/* Build an instance on the current device (b and f_star); returns after
 * the build finished.  L1LS_E_ARG for parameters outside the ranges above. */
l1ls_status l1ls_sgt_generate(const l1ls_sgt_params* params, void* stream, l1ls_sgt** out);
l1ls_status l1ls_sgt_describe(const l1ls_sgt* inst, l1ls_sgt_desc* out);
void l1ls_sgt_free(l1ls_sgt* inst);

/* x_star_dev, g_dev (n each, either may be NULL, not both): the planted x*
 * and the subgradient g of IGen step 2.  Asynchronous on `stream`. */
l1ls_status l1ls_sgt_planted(const l1ls_sgt* inst, double* x_star_dev, double* g_dev, void* stream);

/* trans = 0: out_dev (m) = A in_dev (n); trans = 1: out_dev (n) =
 * A^T in_dev (m; entries n..m-1 are not read).  FP64, asynchronous. */
l1ls_status l1ls_sgt_apply(const l1ls_sgt* inst, int32_t trans, const double* in_dev,
                            double* out_dev, void* stream);

/* kappa_rho(x*) of eq. (17) (section 5): ||x*|| / ||P_rho x*|| with P_rho the
 * projection on the eigenvectors of A^T A = G Sigma^2 G^T whose eigenvalues
 * sigma_i^2 are >= rho (+inf when that projection is 0).  rho >= 0.
 * Blocks until done. */
l1ls_status l1ls_sgt_kappa_rho(const l1ls_sgt* inst, double rho, double* kappa, void* stream);

/* FP64 P = f_tau(x), the dual value at the scaled residual and the relative
 * gap, as l1ls_objective_gap.  Blocks until done. */
l1ls_status l1ls_sgt_objective_gap(const l1ls_sgt* inst, double tau, const double* x_dev,
                                    double* primal, double* dual, double* rel_gap, void* stream);

/*
 * CG-Newton on problem (8) (section 2, section 8.1 item pdNCG, section 8.3),
 * as l1ls_solve_cg_newton: pseudo-Huber mu, PCG with the inverse Hessian
 * diagonal as preconditioner to relative residual pcg_rtol, Armijo
 * backtracking (constant 1e-4) by halving at most max_backtrack times,
 * stop when ||grad f_mu||_inf <= rel_gap_tol * tau or after max_iter Newton
 * steps.  All arithmetic FP64 (opts.precision must be L1LS_F64 and
 * opts.polish 0, else L1LS_E_UNSUPPORTED).  x_dev (n) holds the iterate
 * throughout and the result at the end; opts.x0_dev (may equal x_dev) is the
 * start, NULL for 0.  report: Newton steps, PCG iterations, FP64 gap,
 * ||x - x*|| / ||x*||.  Allocates l1ls_sgt_solve_bytes(n) for the call.
 */
l1ls_status l1ls_sgt_solve_cg_newton(const l1ls_sgt* inst, const l1ls_solve_opts* opts,
                                      double* x_dev, l1ls_report* report);

/*
 * FISTA (section 8.1) on the instance, FP64, from opts.x0_dev (NULL: 0) with
 * L = opts.L (<= 0: sigma_max^2): x_k = soft(y_k - A^T (A y_k - b) / L,
 * tau / L), y_{k+1} = x_k + ((t_k - 1) / t_{k+1}) (x_k - x_{k-1}), t_1 = 1.
 * Every opts.check_every iterations the FP64 gap at x_k is evaluated; the
 * solve stops when the relative gap is <= opts.rel_gap_tol (> 0), when
 * f_tau(x_k) <= opts.f_target (> 0; the comparison protocol of section 8.3),
 * or after opts.max_iter iterations.  x_dev (n) receives the result;
 * opts.precision must be L1LS_F64 and opts.polish 0.  Allocates 8 n bytes
 * for the call.  Returns L1LS_OK when a stop test passed, else
 * L1LS_NOT_CONVERGED.
 */
l1ls_status l1ls_sgt_solve_fista(const l1ls_sgt* inst, const l1ls_solve_opts* opts, double* x_dev,
                                 l1ls_report* report);

/*
 * PCDM (section 8.1 item PCDM, section 8.3) on the instance, FP64, from
 * opts.x0_dev (NULL: 0): step k updates, in parallel and from the same x,
 * every coordinate i of the sampled set S_k to soft(x_i - A_i^T (A x - b) /
 * (beta L_i), tau / (beta L_i)), L_i = (A^T A)_ii.  S_k holds each coordinate
 * independently with probability p = opts.pcdm_p (<= 0 or >= 1: every
 * coordinate), drawn from Philox counter (pair, step, 0x600, 0); for this
 * doubly uniform sampling beta = 1 + (omega - 1) p with omega = 2 nonzeros per
 * row.  Stops as l1ls_sgt_solve_fista (gap tolerance, f_target, max_iter
 * steps < 2^32).  No extra device memory beyond O(1).
 */
l1ls_status l1ls_sgt_solve_pcdm(const l1ls_sgt* inst, const l1ls_solve_opts* opts, double* x_dev,
                                l1ls_report* report);

/* The same CG-Newton one call at a time, for callers that report between
 * Newton steps.  create: validates opts as l1ls_sgt_solve_cg_newton (max_iter
 * is not used), allocates l1ls_sgt_solve_bytes(n), sets x_dev to the start;
 * x_dev must stay valid until destroy.  step: up to `steps` more Newton steps
 * (none once converged); report: totals since create, FP64 gap and
 * ||x - x*|| / ||x*|| at the current x_dev; returns L1LS_OK once converged,
 * else L1LS_NOT_CONVERGED.  destroy waits for the object's stream. */
typedef struct l1ls_sgt_newton l1ls_sgt_newton;
l1ls_status l1ls_sgt_newton_create(const l1ls_sgt* inst, const l1ls_solve_opts* opts, double* x_dev,
                                    l1ls_sgt_newton** out);
l1ls_status l1ls_sgt_newton_step(l1ls_sgt_newton* newton, int64_t steps, l1ls_report* report);
void l1ls_sgt_newton_destroy(l1ls_sgt_newton* newton);

/* HIP-event times of the passes of the last CG-Newton (solve or stepping
 * object) or FISTA on inst run with opts.time_kernels = 1: ms[q] total milliseconds and
 * calls[q] launches of q = 0 the PCG iteration pass (p, dx, r; the first
 * iteration of each PCG, which reads neither p nor dx, is left out), 1 the
 * line-search pass, 2 the Newton setup pass (gradient, d, PCG start); after
 * l1ls_sgt_solve_fista: 0 the iteration pass, 1 the gap pass; after
 * l1ls_sgt_solve_pcdm: 0 the step pass. */
l1ls_status l1ls_sgt_kernel_times(const l1ls_sgt* inst, double* ms, int64_t* calls);

/*
 * The autotuner's cache.  The library times its launch choices the first
 * time it meets a size class (ceil(log2) of the rows) and keeps the fastest:
 *   "fista_f32_residual/<class>", "fista_f32_transpose/<class>": the tile
 *     schedule of the stored FP32 passes (0-3: entries per lane issued
 *     together, 10/8/16/10 and 16/12/16/8, nontemporal index and value loads
 *     in all but the residual's 3 and the transpose's 2);
 *   "batch_rounds/<class>": rounds of four tiles per workgroup task (1, 2, 4, 8).
 * Every choice computes the same values in the same order.  With the
 * environment variable L1LS_TUNE_CACHE naming a file, the cache is read from
 * it (JSON) on first use and written back after every new choice.
 * get: the cached choice, -1 if none.  set: fix a choice (choice < 0
 * forgets it; L1LS_E_ARG for a key with quotes, backslashes or newlines).
 */
int32_t l1ls_tune_get(const char* key);
l1ls_status l1ls_tune_set(const char* key, int32_t choice);

const char* l1ls_status_string(int32_t status);
/* ABI version of this header (incremented on incompatible changes). */
int32_t l1ls_version(void);

#ifdef __cplusplus
}
#endif
#endif /* L1LS_H */
