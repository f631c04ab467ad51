/*
 * afsai.h -- C ABI of the MI355X (gfx950) adaptive FSAI library: setup of the factored sparse
 * approximate inverse G (M^-1 = G^T G ~ A^-1) with adaptive pattern growth, its application,
 * and the preconditioned conjugate gradient method, for sparse SPD matrices in CSR.
 *
 * Method: Isotton, Janna, Bernaschi, "A GPU-accelerated adaptive FSAI preconditioner for
 * massively parallel simulations" (arXiv 2010.14175), Sec. 2 (FSAI with dynamic pattern
 * selection) and Sec. 3 (GPU kernels: Kaporin gradient and selection, systems gather, batched
 * Cholesky, group-per-row SpMV).  One GPU; no communication.
 *
 * Conventions for every entry point
 *   - Pointers marked (device) are HIP device pointers on the current device; pointers marked
 *     (host) are host memory.  Sizes are element counts.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All device work of
 *     a call is enqueued on that stream.
 *   - Return value: AFSAI_OK (0) or one of the AFSAI_ERR_* codes below; no C++ exception ever
 *     crosses this interface.  afsai_last_error() returns a message for the calling thread's
 *     most recent failure.
 *   - Caller-owned buffers (A, b, x, r, z, export targets) must stay valid until the enqueued
 *     work has finished; the library never frees or retains them after returning.
 */
#ifndef AFSAI_H
#define AFSAI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define AFSAI_OK 0
#define AFSAI_ERR_INVALID_ARG 1   /* null pointer, n <= 0, kmax < 0, s < 1, eps < 0, rtol <= 0 ... */
#define AFSAI_ERR_BAD_MATRIX 2    /* CSR structure: unsorted/duplicate/out-of-range columns, missing
                                     diagonal, row pointers not monotone, or (with AFSAI_VALIDATE)
                                     an asymmetric matrix */
#define AFSAI_ERR_NOT_SPD 3       /* a_ii <= 0, a Cholesky pivot <= 0 or not finite, or p.Ap <= 0 */
#define AFSAI_ERR_NO_MEMORY 4     /* device allocation failed */
#define AFSAI_ERR_NOT_CONVERGED 5 /* PCG reached maxit; x and info are still filled */
#define AFSAI_ERR_TOO_LARGE 6     /* 1 + kmax*s > 64, or a pattern's candidate set cannot be held
                                     on chip, or nnz(G) would exceed 2^31 - 1 */
#define AFSAI_ERR_HIP 7           /* a HIP runtime call failed (message in afsai_last_error) */

/* value type of G and G^T storage */
#define AFSAI_F64 0
#define AFSAI_F32 1

/* afsai_params.flags */
#define AFSAI_VALIDATE 1u /* check the CSR structure and exact symmetry on the device first */
/* per-row setup arithmetic (gradient, selection, dense factorisation, g) in FP32, A's values
 * rounded to FP32 where they are read: the fully single-precision setup the paper discusses
 * (Sec. 3).  Patterns may then differ from an FP64 setup where gradients are within FP32
 * rounding of each other.  Needs every row of A to have at most 128 entries and n <= 2^24
 * (AFSAI_ERR_INVALID_ARG otherwise). */
#define AFSAI_SETUP_F32 2u
/* the precision form's gradient: the Kaporin gradient (the product over the pattern rows that
 * ranks the candidates, eq. grapsi) reads an FP32 copy of A's values (the paper's A_s =
 * single(A) of Sec. 4.3), while the gathered systems, the dense factorisation, g and psi stay
 * FP64.  Halves the value bytes of the gradient pass; candidates whose gradients are within
 * FP32 rounding of each other may rank differently from an FP64 gradient, and then the
 * pattern (and G) of that row differs.  Inverse-factor form only: needs FP64 setup arithmetic,
 * rows of at most 128 entries and n <= 2^24 (AFSAI_ERR_INVALID_ARG otherwise).  The setup
 * allocates the copy (4 bytes per entry) for the call. */
#define AFSAI_GRAD_F32 4u

/*
 * Square sparse matrix in CSR, 0-based, int32 indices (the paper's 4-byte local indices,
 * Sec. 4.1).  Both triangles stored; columns strictly ascending within each row; the diagonal
 * present in every row.  For the setup, A must be symmetric bit for bit (a_ij == a_ji): the
 * gather of A[P,P] reads each pair from whichever of the two rows it has loaded.
 */
typedef struct afsai_csr {
    int32_t n;              /* rows = columns, > 0 */
    int32_t nnz;            /* stored entries = row_ptr[n] */
    const int32_t *row_ptr; /* (device) n+1 */
    const int32_t *col_idx; /* (device) nnz */
    const double *val;      /* (device) nnz */
} afsai_csr;

/*
 * Controls of the adaptive procedure (Sec. 2, the three user parameters).
 *   kmax      maximum number of pattern-growth steps per row, >= 0 (kmax = 0 gives
 *             G = diag(a_ii^-1/2), i.e. Jacobi, the paper's baseline of Sec. 5.2)
 *   s         positions added to a row per step, >= 1 (1 + kmax*s <= 64)
 *   eps       a row stops growing once psi_k / psi_0 <= eps (eq. exit_crit), >= 0
 *   tie_rtol  relative tie band of the selection: every candidate whose |gradient| is within
 *             tie_rtol of the largest counts as tied and the smallest column wins; in [0, 1);
 *             2^-26 recommended (exact ties of stencil matrices then resolve identically on
 *             any hardware)
 *   g_prec    AFSAI_F64 or AFSAI_F32 storage for G and G^T (values widened to FP64 in every
 *             product; the per-row Cholesky is FP64 in both cases)
 *   flags     AFSAI_VALIDATE, AFSAI_SETUP_F32, AFSAI_GRAD_F32 (or-ed; not the last two together)
 */
typedef struct afsai_params {
    int32_t kmax;
    int32_t s;
    double eps;
    double tie_rtol;
    int32_t g_prec;
    uint32_t flags;
} afsai_params;

/* opaque preconditioner: owns G and G^T (CSR, device), per-row diagnostics and a PCG workspace */
typedef struct afsai_precond_s *afsai_precond;

/* setup diagnostics (host) */
typedef struct afsai_setup_info {
    int32_t n;
    int32_t mmax;              /* 1 + kmax*s */
    int64_t nnz_g;             /* entries of G (= entries of G^T) */
    int32_t g_prec;
    int32_t rows_stop_kmax;    /* rows that took all kmax steps */
    int32_t rows_stop_eps;     /* rows stopped by eq. exit_crit */
    int32_t rows_stop_nocand;  /* rows that ran out of eligible candidates */
    int32_t rows_retried;      /* rows redone with a larger on-chip candidate table */
    double sum_log_psi;        /* sum_i log psi_i (final); kappa = exp((this - log det A)/n), eq. kap2 */
    double ms;                 /* wall time of the setup call */
} afsai_setup_info;

/* PCG diagnostics (host) */
typedef struct afsai_pcg_info {
    int32_t iters;       /* iterations performed */
    int32_t converged;   /* 1 if ||r_k|| <= rtol ||b|| */
    double relres;       /* ||r_k|| / ||b||, recursively updated residual */
    double true_relres;  /* ||b - A x|| / ||b|| recomputed at the end */
    double ms;           /* wall time of the solve call */
} afsai_pcg_info;

/*
 * afsai_setup -- adaptive FSAI setup (Sec. 2; kernels of Sec. 3).
 *   Every row i starts from P_i = {i}, g = a_ii^-1/2 (G_0 = I scaled) and, up to kmax times,
 *   (1) forms the Kaporin gradient v_j = (A g)_j over the lower candidates j < i, j not in P_i
 *       (eq. grapsi), (2) appends the s candidates of largest |v_j| (ties: tie_rtol band,
 *       smallest column; candidates with |v_j| <= 2^-40 max|v| are not eligible; no eligible
 *       candidate stops the row), (3) gathers A[P_i,P_i], (4) factors it A[P,P] = L L^T in FP64
 *       and sets row i of G to L^-T e_m (eq. DensSys scaled by eq. diagScal, so that
 *       (G A G^T)_ii = 1), with psi_i = L_mm^2, and (5) stops the row when psi_i/a_ii <= eps.
 *   A    (host struct, device arrays) the SPD matrix, see afsai_csr.
 *   p    (host) parameters.
 *   out  (host) receives a new handle on success (NULL on failure).
 *   Synchronous: returns after the device work is done.  The handle does not reference A.
 */
int afsai_setup(const afsai_csr *A, const afsai_params *p, void *stream, afsai_precond *out);

/*
 * afsai_apply -- z = G^T (G r), the preconditioner application M^-1 r (eq. prec).
 *   r, z (device) length n; must not alias.  Asynchronous on `stream`.
 *   Uses the handle's workspace: one apply or solve per handle at a time.
 */
int afsai_apply(afsai_precond P, const double *r, double *z, void *stream);

/*
 * afsai_apply_noalloc -- afsai_apply for callers that cannot allocate device memory (code
 *   under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 *   products and the same result as afsai_apply, bit for bit, with the intermediate t = G r in
 *   a fixed device array of the library instead of the handle's workspace.  The call itself
 *   allocates nothing (no hipMalloc, hipFree or pinned host memory; with the kernel timer off,
 *   its default).
 *   r, z (device) length n, caller-owned, must not alias.  n <= 16,777,216 (the array holds
 *   2^24 doubles, 128 MiB per GPU the library runs on, kept until the process ends).
 *   Asynchronous on `stream`.  Every call on one GPU shares that GPU's array: calls that
 *   overlap in time on one GPU (different streams or host threads) race on it.
 *   Errors: AFSAI_ERR_INVALID_ARG (null or aliased pointers), AFSAI_ERR_TOO_LARGE (n above
 *   the limit), AFSAI_ERR_HIP.
 */
int afsai_apply_noalloc(afsai_precond P, const double *r, double *z, void *stream);

/*
 * pcg_solve -- preconditioned conjugate gradient for A x = b with M^-1 = G^T G (P != NULL) or
 *   M = I (P == NULL, plain CG).  Textbook PCG (Sec. 5.2 stops at a residual reduction of eight
 *   orders of magnitude): x holds x0 on entry and the last iterate on return; the iteration
 *   stops when ||r_k||_2 <= rtol ||b||_2 (recursive residual) or after maxit iterations.
 *   b, x (device) length n.  rtol > 0, maxit >= 0.  info (host, may be NULL).
 *   ||b|| = 0 gives x = 0 and 0 iterations.
 *   Returns AFSAI_OK, AFSAI_ERR_NOT_CONVERGED (x, info filled) or AFSAI_ERR_NOT_SPD (p.Ap <= 0).
 *   Synchronous.
 */
int pcg_solve(const afsai_csr *A, afsai_precond P, const double *b, double *x, double rtol,
              int32_t maxit, void *stream, afsai_pcg_info *info);

/*
 * Batches of independent systems (many small SPD systems solved together).
 *   The systems are given as one block-diagonal CSR matrix: system k owns rows (and columns)
 *   offsets[k] .. offsets[k+1]-1, and no row has an entry outside its system.  Because rows are
 *   set up independently (Sec. 2) and gradients never leave a block, the setup of the batch is
 *   one launch of the setup over the whole matrix; the candidate tie rule (smallest column) does
 *   not depend on where a system sits, so each system's G is the one a separate afsai_setup of
 *   that system gives, bit for bit.  The solver then runs all systems together, each with its
 *   own scalars and stopping test; a system's iterates and x are those of a separate pcg_solve
 *   of it, bit for bit (its dot products are summed over the same partition).
 *   offsets (host) nsys + 1 entries, offsets[0] = 0, strictly increasing, offsets[nsys] = n.
 */

/*
 * afsai_setup_batched -- afsai_setup of a batch.  Returns AFSAI_ERR_BAD_MATRIX when a row has
 *   an entry outside its system.  The handle's products follow the systems (every system
 *   starts a new 64-row slice); it can only be used with pcg_solve_batched and the same
 *   offsets, or with afsai_apply.
 */
int afsai_setup_batched(const afsai_csr *A, int32_t nsys, const int32_t *offsets, const afsai_params *p,
                        void *stream, afsai_precond *out);

/*
 * pcg_solve_batched -- pcg_solve of every system of a batch at once.  P is NULL (plain CG) or
 *   a handle from afsai_setup_batched with the same offsets.  b, x (device) length n.
 *   info (host, may be NULL): nsys entries, one per system.  Iteration ends when every system
 *   has stopped.  Returns AFSAI_OK when all converged, else the status of the first system
 *   that did not (AFSAI_ERR_NOT_SPD, AFSAI_ERR_NOT_CONVERGED; x and info filled).  Synchronous.
 */
int pcg_solve_batched(const afsai_csr *A, afsai_precond P, int32_t nsys, const int32_t *offsets, const double *b,
                      double *x, double rtol, int32_t maxit, void *stream, afsai_pcg_info *info);

/*
 * Serving: a request loop that admits SPD systems of mixed sizes, sets each up (afsai_setup)
 *   and solves it (pcg_solve, x0 = 0) while others are in progress.
 *   Requests wait in arrival order and are admitted while fewer than max_slots are admitted and
 *   the admitted requests' device footprints (setup results, G and G^T, the SELL copy of A,
 *   the solver vectors; an estimate from n, nnz and params, reported per request) fit in
 *   hbm_budget; a finished request frees its slot and memory at once and admits the next
 *   (continuous batching).  Each admitted request has its own stream: setup threads set up new
 *   requests while one scheduler thread keeps the PCG iterations of all solving requests in
 *   flight together.  A request's x is the one a separate afsai_setup + pcg_solve with the same
 *   parameters gives, bit for bit, whatever else is served.  Kernel timing (afsai_profile_*)
 *   must be off while a server runs.
 */
typedef struct afsai_server_s *afsai_server;

typedef struct afsai_server_config {
    size_t hbm_budget;      /* bytes of device memory admitted requests may hold (> 0) */
    int32_t max_slots;      /* requests admitted at once (>= 1; 1 serves one request at a time) */
    int32_t setup_threads;  /* host threads running setups (1..64) */
    afsai_params params;    /* setup parameters of every request */
    double rtol;            /* PCG stopping tolerance of every request */
    int32_t maxit;          /* PCG iteration limit of every request */
    int32_t max_heavy;      /* heavy requests admitted at once (0: 1; < 0: no limit) */
    int64_t heavy_nnz;      /* matrix entries from which a request is heavy (0: 2^22) */
} afsai_server_config;

typedef struct afsai_request_result {
    int64_t ticket;         /* from afsai_server_submit */
    int32_t status;         /* AFSAI_OK, or the error of its setup or solve */
    int32_t iters;
    int32_t converged;
    double true_relres;     /* ||b - A x|| / ||b|| */
    int64_t footprint;      /* device bytes the request held while admitted (estimate) */
    double submit_ms, admit_ms, setup_done_ms, done_ms;  /* times since the server was created */
} afsai_request_result;

/* afsai_server_create -- starts the setup threads and the scheduler on the current device. */
int afsai_server_create(const afsai_server_config *cfg, afsai_server *out);

/*
 * afsai_server_submit -- queues the solve of A x = b (A, b, x device arrays; A's arrays, b and
 *   x must stay valid and untouched until the request's result has been polled).  p (host) are
 *   this request's setup parameters (NULL: the server's).  x is set to 0 before the solve.
 *   Returns AFSAI_ERR_TOO_LARGE when the request alone exceeds the budget.
 */
int afsai_server_submit(afsai_server S, const afsai_csr *A, const afsai_params *p, const double *b, double *x,
                        int64_t *ticket);

/*
 * afsai_server_poll -- moves up to max_results finished requests (in completion order) into out
 *   (host) and sets *count; waits up to wait_ms for one when none has finished.
 */
int afsai_server_poll(afsai_server S, afsai_request_result *out, int32_t max_results, int32_t *count,
                      int32_t wait_ms);

/* afsai_server_pending -- requests not yet finished, device bytes and slots currently admitted. */
int afsai_server_pending(afsai_server S, int64_t *outstanding, int64_t *bytes_in_use, int32_t *slots_in_use);

/* afsai_server_destroy -- waits for every submitted request, then stops the server. */
int afsai_server_destroy(afsai_server S);

/* afsai_spmv -- y = A x (group-per-row CSR product used by the solver).  Asynchronous. */
int afsai_spmv(const afsai_csr *A, const double *x, double *y, void *stream);

/*
 * afsai_spmm -- Y = A X for k right-hand sides at once (the product of a PCG over several
 *   right-hand sides, where every iteration multiplies one block of k vectors; Sec. 4.1 keeps
 *   such dense blocks with each row's entries contiguous, for systems with several
 *   right-hand sides).
 *   X, Y (device): n x k, row-major (entry (i, j) at i * k + j, so the k values of a row are
 *   contiguous); caller-owned, must not alias.  k: 1, 2, 4 or 8.
 *   A is converted to its SELL-64 layout for the call (rows ordered by length when uneven) and
 *   every matrix entry is read once for the k vectors; column j of Y equals the single-vector
 *   SELL product of column j bit for bit.  Synchronous on stream.
 *   Errors: AFSAI_ERR_INVALID_ARG (k, null or aliased blocks, a split layout forced with
 *   AFSAI_OPT_SELL_UNEVEN = 1), AFSAI_ERR_NO_MEMORY, AFSAI_ERR_HIP.
 */
int afsai_spmm(const afsai_csr *A, int32_t k, const double *X, double *Y, void *stream);

/*
 * Prepared matrices: A's SELL-64 layout (the layout pcg_solve and afsai_spmm convert A to on
 * every call) made once and kept, for callers that multiply by, or solve with, one matrix many
 * times.  The products and iterates are those of the unprepared calls bit for bit.
 */
typedef struct afsai_matrix_s *afsai_matrix;

/*
 * afsai_matrix_prepare -- converts A to its SELL-64 layout on the current device.
 *   A's arrays are read during the call only; the handle owns a device copy (about
 *   12 bytes per entry plus padding, 13.3 when A's rows are made of runs of three
 *   consecutive columns and run indices are kept beside the columns) and A's values may change afterwards without affecting it
 *   (prepare again to take them).  *out = NULL on failure.  Synchronous on stream.
 *   Errors: AFSAI_ERR_INVALID_ARG, AFSAI_ERR_NO_MEMORY, AFSAI_ERR_TOO_LARGE, AFSAI_ERR_HIP.
 */
int afsai_matrix_prepare(const afsai_csr *A, void *stream, afsai_matrix *out);

/* afsai_matrix_destroy -- waits for the device, then frees the handle (NULL is ignored). */
void afsai_matrix_destroy(afsai_matrix M);

/*
 * afsai_spmm_prepared -- afsai_spmm with a prepared A (same arguments and results; no
 *   conversion, no allocation).  Errors: as afsai_spmm, and AFSAI_ERR_INVALID_ARG when the
 *   current device is not the one M was prepared on, or M holds a split layout (prepared with
 *   AFSAI_OPT_SELL_UNEVEN = 1).  Synchronous on stream.
 */
int afsai_spmm_prepared(afsai_matrix M, int32_t k, const double *X, double *Y, void *stream);

/*
 * pcg_solve_prepared -- pcg_solve (Sec. 5.2) with a prepared A: the same iterates, x and info
 *   bit for bit as pcg_solve with the A that M was prepared from (with the default SELL
 *   product for A), without converting A.  P: a single-system preconditioner or NULL.
 *   Errors: as pcg_solve, and AFSAI_ERR_INVALID_ARG for a device mismatch or a split layout.
 *   Synchronous.
 */
int pcg_solve_prepared(afsai_matrix M, afsai_precond P, const double *b, double *x, double rtol, int32_t maxit,
                       void *stream, afsai_pcg_info *info);

/*
 * pcg_solve_multi -- PCG (M^-1 = G^T G, or plain CG with P == NULL) for k right-hand sides at
 *   once, A X = B: k independent textbook recurrences (each with its own alpha, beta, rho and
 *   stopping test ||r_j|| <= rtol ||b_j||, as pcg_solve) whose products with A, G and G^T are
 *   block products reading each matrix once per iteration for all k columns (Sec. 4.1 keeps
 *   such blocks with each row's entries contiguous).  A column that has stopped keeps its x.
 *   B, X (device): n x k row-major, caller-owned, must not alias; X0 = 0 (X is overwritten).
 *   k: 1, 2, 4 or 8.  P: a single-system preconditioner of A (not a batch, no split layouts).
 *   info (host, may be NULL): k entries.  Synchronous (the host reads the stop flags after
 *   every iteration).
 *   Returns AFSAI_OK, AFSAI_ERR_NOT_CONVERGED (some column reached maxit), AFSAI_ERR_NOT_SPD
 *   (p.Ap <= 0 in some column), AFSAI_ERR_INVALID_ARG, AFSAI_ERR_NO_MEMORY, AFSAI_ERR_HIP.
 */
int pcg_solve_multi(const afsai_csr *A, afsai_precond P, int32_t k, const double *B, double *X, double rtol,
                    int32_t maxit, void *stream, afsai_pcg_info *info);

/* afsai_get_setup_info -- diagnostics of a handle (host struct). */
int afsai_get_setup_info(afsai_precond P, afsai_setup_info *info);

/*
 * afsai_export -- copies G as CSR (FP64 values, widened if stored in FP32) into caller
 *   buffers (device): row_ptr n+1, col and val nnz_g entries.  Synchronous.
 */
int afsai_export(afsai_precond P, int32_t *row_ptr, int32_t *col, double *val, void *stream);

/*
 * afsai_export_rows -- per-row diagnostics (device buffers, n entries each, any may be NULL):
 *   psi (final psi_i), steps (growth steps taken), reason (0 kmax reached, 1 eps test,
 *   2 no eligible candidate).  Synchronous.
 */
int afsai_export_rows(afsai_precond P, double *psi, int32_t *steps, int32_t *reason, void *stream);

/*
 * afsai_import -- builds a handle from a given lower-triangular G (device CSR, copied; the
 *   caller keeps ownership of its arrays), storing values as g_prec.  Lets a caller persist a
 *   preconditioner and skip the setup.  Synchronous.
 */
int afsai_import(const afsai_csr *G, int32_t g_prec, void *stream, afsai_precond *out);

/* afsai_destroy -- frees a handle and everything it owns (NULL is a no-op). */
void afsai_destroy(afsai_precond P);

/*
 * afsai_release_cache -- the library keeps device blocks it has freed (temporaries of setup
 *   and solve, destroyed handles) and the pinned host blocks of finished solves for reuse;
 *   this returns them all to the HIP runtime.
 *   Call only while no other library call is running.
 */
int afsai_release_cache(void);

/* afsai_last_error -- message of the calling thread's most recent failure ("" if none). */
const char *afsai_last_error(void);

/*
 * afsai_set_option -- process-wide tuning knobs (0 restores the automatic choice):
 *   AFSAI_OPT_SETUP_GROUP     rows appended to a row's Cholesky factor together in one
 *                             update of the per-row setup kernel (1..4; any choice gives
 *                             identical G)
 *   AFSAI_OPT_SETUP_TABLE     slots of the first on-chip candidate table (power of two,
 *                             64..1024; the inverse-factor form takes 64..1024, the
 *                             Cholesky form 128..1024)
 *   AFSAI_OPT_SPMV_GROUP      lanes per row of the CSR products (4, 8, 16, 32 or 64)
 *   AFSAI_OPT_SPMV_UNROLL     independent loads per lane per round in the sparse products
 *                             (1, 2, 4, 8)
 *   AFSAI_OPT_PCG_CSR_A       1: pcg_solve multiplies by A in CSR (group per row) instead of
 *                             converting it to the SELL-64 layout first
 *   AFSAI_OPT_PCG_FORM        0: automatic (products that also form the updated vectors
 *                             below 200,000 rows, separate update kernels above); 1: separate
 *                             update kernels; 2: fused products (used only when no SELL
 *                             matrix of the solve is split, see AFSAI_OPT_SELL_WIDTH); all
 *                             forms give identical results
 *   AFSAI_OPT_SELL_WIDTH      entries per row held by the 64-row slices of every SELL layout
 *                             built afterwards; longer rows keep their leading entries in a
 *                             second, length-sorted layout multiplied first (0: split only
 *                             when padding would exceed a tenth of the entries, at the width
 *                             that minimises the work; products are identical either way)
 *   AFSAI_OPT_PCG_GRAPH       0 (automatic) and 1: the kernels of each PCG iteration are
 *                             enqueued one by one; 2: the iteration is captured once per solve
 *                             into a HIP graph (once per buffer parity in the fused form) and
 *                             replayed (never while the kernel timer is on). Results are
 *                             identical.
 *   AFSAI_OPT_SETUP_SLOTS     where the setup kernel keeps the table slots of the pattern rows'
 *                             entries: 0 automatic (registers when every row of A has at most
 *                             128 entries and n <= 2^24, else LDS), 1 LDS, 2 registers
 *                             (AFSAI_ERR_INVALID_ARG from afsai_setup when not possible)
 *   AFSAI_OPT_SELL_TAIL       products with a split SELL-64 layout: 0 (automatic) the leading
 *                             entries of the long rows run in a launch of their own first,
 *                             1 inside the slices' kernel (identical results)
 *   AFSAI_OPT_SELL_UNEVEN     SELL-64 layouts of matrices with uneven rows (G^T): 0 (automatic)
 *                             the rows of each window of 4 slices (256 rows, within one system
 *                             of a batch) ordered by length and dealt to the window's slices,
 *                             every lane reading its own row's entries only; 1 split layouts
 *                             (the slices keep each row's last w entries, a second layout the
 *                             leading ones).  Products are identical row by row; fused dot
 *                             products are summed in another order
 *   AFSAI_OPT_SETUP_FORM      per-row factorisation of the setup: 0 (automatic) the
 *                             inverse-factor form where it applies (FP64 setup arithmetic,
 *                             every row of A at most 128 entries, n <= 2^24), else the
 *                             Cholesky form; 1 the Cholesky form (a factor appended row by
 *                             row, then a back substitution per step); 2 the inverse-factor
 *                             form (AFSAI_ERR_INVALID_ARG from afsai_setup when it does not
 *                             apply).  Both forms compute the same G in exact arithmetic and
 *                             differ by rounding only
 *   AFSAI_OPT_SETUP_LANES     inverse-factor form: lanes that own one row (8, 16, 32 or 64;
 *                             64 / lanes rows per wavefront; 0 automatic: 8 or 16 when they hold
 *                             the pattern, else 64; 32 only when asked for).  A request smaller
 *                             than the pattern takes the next size that holds it.  Any choice
 *                             gives identical G
 *   AFSAI_OPT_SETUP_CLAIM     wavefronts' worth of rows one atomic claim of the setup kernel takes
 *                             from its XCD's counter (1..64; 0 automatic: enough rows for about
 *                             4,000 table entries of work, at most 16).  Any choice gives
 *                             identical G
 *   AFSAI_OPT_SELL_RUNS       pcg_solve's SELL-64 layout of A (separate-update form): 0
 *                             (automatic) one column index per run of three consecutive
 *                             columns when every row of A is made of such runs (3 x 3 blocks
 *                             of a 3-dof discretisation), 1 one index per entry.  Identical
 *                             results.  A prepared matrix takes the setting in force at
 *                             afsai_matrix_prepare
 * Returns AFSAI_ERR_INVALID_ARG for an unknown option or value.  Not thread safe against
 * concurrent calls of the library.
 */
#define AFSAI_OPT_SETUP_GROUP 1
#define AFSAI_OPT_SETUP_TABLE 2
#define AFSAI_OPT_SPMV_GROUP 3
#define AFSAI_OPT_SPMV_UNROLL 4
#define AFSAI_OPT_PCG_CSR_A 5
#define AFSAI_OPT_PCG_FORM 6
#define AFSAI_OPT_SELL_WIDTH 7
#define AFSAI_OPT_PCG_GRAPH 8
#define AFSAI_OPT_SETUP_SLOTS 9
#define AFSAI_OPT_SELL_TAIL 10
#define AFSAI_OPT_SELL_UNEVEN 11
#define AFSAI_OPT_SETUP_FORM 12
#define AFSAI_OPT_SETUP_LANES 13
#define AFSAI_OPT_SETUP_CLAIM 14
#define AFSAI_OPT_SELL_RUNS 15
int afsai_set_option(int32_t option, int64_t value);

/*
 * Kernel timing: with profiling on, the library brackets every kernel launch with HIP events
 * on the launch stream and accumulates, per kernel name, the number of launches and the total
 * event-measured duration.  Off by default; enabling it adds event overhead.
 */
typedef struct afsai_kernel_time {
    char name[48];
    int64_t launches;
    double total_ms;
} afsai_kernel_time;

int afsai_profile_enable(int32_t on);
/* restricts the timing to the kernels named in `names` (comma-separated timer names such as
 * "afsai_rows,spmv_A_dot", host string); NULL or "" times every kernel again.  The other
 * kernels then run without events, so the timed ones are measured inside an undisturbed run. */
int afsai_profile_only(const char *names);
/* copies up to cap entries into out (host), sets *count; reset != 0 clears the counters */
int afsai_profile_read(afsai_kernel_time *out, int32_t cap, int32_t *count, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* AFSAI_H */
