/*
 * mdp.h - C ABI of the MI355X solver for mixed-dimensional scalar elliptic
 * systems (Hu, Keilegavlen, Nordbotten 2022, "Effective Preconditioners for
 * Mixed-Dimensional Scalar Elliptic Problems").
 *
 * The library solves A p = f for the 2x2 host/fracture block system of
 * eq. (4) with flexible GMRES, right-preconditioned (Section 3.2) by the
 * inexact block lower-triangular preconditioner M_L of eq. (8), applied as
 * Algorithm 1: Q_OO = smoothed-aggregation AMG V-cycles on the approximate
 * Schur complement S~ of eq. (7), the fracture residual update with A_GO,
 * and Q_GG = V-cycles on A_GG (Section 3.3).  The other two block forms of
 * Section 3.2 (block diagonal, block upper) are available with the same
 * Q's (mdp_options.block_form).
 *
 * Conventions for every call:
 *  - Sparse inputs are 0-based CSR in HOST memory, int32 indices, FP64 values.
 *    The library copies what it needs; it never keeps caller pointers.
 *  - Vectors passed to solve calls are FP64 in DEVICE memory, in the
 *    caller's unknown order (the library permutes to [Omega; Gamma]
 *    internally).
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Blocking calls
 *    synchronise that stream before returning.
 *  - Return value: MDP_OK (0) or a positive status, or a negative error code.
 *    mdp_last_error() gives a message for the last failure on this thread.
 *  - A handle may be used by one thread at a time.
 */
#ifndef MDP_H
#define MDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status and error codes ---------------------------------------------- */
#define MDP_OK 0
#define MDP_NOT_CONVERGED 1 /* iteration budget spent; x holds the last iterate */
#define MDP_PENDING 2       /* mdp_poll: request not finished yet              */
#define MDP_STAGNATED 3     /* no progress: a full restart cycle, or two shorter
                               ones in a row, lowered the true residual by less
                               than 0.1%; x holds the last iterate              */
#define MDP_EINVAL (-1)     /* bad argument, malformed CSR, part not in {0,1}   */
#define MDP_ENONPOS_DIAG (-2) /* a diagonal entry of A_GG or S~ <= 0 (eq. (7) and
                                 the smoothers divide by them)                  */
#define MDP_ESINGULAR (-3)  /* coarsest dense factorisation failed             */
#define MDP_ENAN (-4)       /* NaN/Inf in the input or during the iteration    */
#define MDP_ENOMEM (-5)     /* device allocation failed / budget exceeded       */
#define MDP_EHIP (-6)       /* HIP runtime error                                */
#define MDP_EBUSY (-7)      /* server full: request refused                      */

/* ---- precision modes (options.precision) --------------------------------- */
#define MDP_FP64 0  /* everything in FP64                                         */
#define MDP_MIXED 1 /* preconditioner (S~, A_GG, A_GO, P, R, smoother) in FP32;
                       outer FGMRES residual, orthogonalisation and the coarsest
                       dense solve in FP64                                        */

/* ---- option flags (options.flags) ---------------------------------------- */
#define MDP_USE_X0 1u      /* mdp_solve: start from the x passed in, not zero  */
#define MDP_HOST_ONLY 2u   /* mdp_setup: build the hierarchy on the host only
                              (no device upload); for inspection on machines
                              without a GPU.  Solve calls then return EINVAL. */
#define MDP_GRAPHS 8u      /* mdp_solve, mdp_solve_batch: replay each Arnoldi
                              step from a HIP graph captured on first use
                              instead of launching its kernels one by one
                              (never while kernel timers run; a solve handed
                              the legacy stream runs on a stream of its own).
                              Same kernels and results.  Measured on small,
                              launch-bound systems (4k-70k unknowns): 5-20%
                              less time per iteration; on 100^3 systems: about
                              2% more. */
#define MDP_FALLBACK_FP64 16u /* mdp_solve in MDP_MIXED: a column whose
                              iteration produced a NaN/Inf from finite input
                              (e.g. matrix values beyond FP32's range) or that
                              ended MDP_STAGNATED is solved again from zero with
                              the FP64 preconditioner, built on first need and
                              kept with the handle (its Krylov directions
                              widen to FP64 too); stats report fallback = 1,
                              the iterations and cycles of both attempts and
                              the status of the second.  mdp_solve's four-
                              column groups and mdp_solve_batch re-solve their
                              failed columns one by one, each with its own
                              handle's flag. */
#define MDP_HOST_PRODUCTS 32u /* mdp_setup: form every sparse product of the
                              set-up (A P_t, R A, (R A) P of Section 3.3 and
                              A_OG diag(A_GG)^-1 A_GO of eq. (7)) on the host
                              threads.  By default, unless MDP_HOST_ONLY is
                              set, products of at least 2^22 terms (or the
                              count in the environment variable
                              MDP_DEVICE_PRODUCT_TERMS) are formed on the
                              device (expansion, stable radix sort by
                              row and column, in-order sums): the same
                              matrices bit for bit, so the same hierarchy; a
                              product of more than 2^29 terms, or one that does
                              not fit in free device memory, is formed on the
                              host. */
#define MDP_NO_AUTOTUNE 4u /* mdp_setup: keep the fixed rule for each matrix's
                              device format instead of timing the candidates
                              (diagonal storage for stencil matrices,
                              diagonals plus a CSR remainder for stencils
                              with irregular couplings, sliced ELL, CSR with
                              one thread per row, CSR with 2..64 lanes per
                              row and 4 or 8 entries in flight per lane) on
                              the device and keeping the fastest.  The format
                              changes only the order of the additions in each
                              row; equal matrices get equal formats within a
                              process. */

/* ---- block preconditioner (Section 3.2: the factorisation eq. (5) gives
 *      B_L = (D L)^-1, B_D = D^-1 and B_U = (U D)^-1; each is made inexact
 *      with the same Q_OO, V-cycles on S~ of eq. (7), and Q_GG, V-cycles on
 *      A_GG) ------------------------------------------------------------------ */
#define MDP_BLOCK_LOWER 0 /* M_L of eq. (8), Algorithm 1: Q_OO, A_GO update, Q_GG */
#define MDP_BLOCK_DIAG 1  /* M_D: Q_OO and Q_GG on their blocks, independently     */
#define MDP_BLOCK_UPPER 2 /* M_U: Q_GG, then r_O - A_OG z_G, then Q_OO             */

/* ---- smoother of the V-cycles (options.smoother) --------------------------- */
#define MDP_SMOOTH_L1JACOBI 0 /* l1-Jacobi, d_i = sum_j |a_ij| (default)             */
#define MDP_SMOOTH_GS 1       /* multicolour Gauss-Seidel, the smoothing of Section 4:
                                 greedy natural-order colouring of every level;
                                 forward sweeps (colours ascending) before the
                                 coarse correction, backward sweeps after; one
                                 launch per colour.  The swept coarsest level
                                 keeps l1-Jacobi. */

/* ---- operators for mdp_apply ---------------------------------------------- */
#define MDP_OP_A 0    /* y = A x, the full system matrix (FP64)                     */
#define MDP_OP_ML 1   /* y = M x, one application of the handle's block preconditioner
                         (M_L of Algorithm 1 unless block_form says otherwise)     */
#define MDP_OP_QOO 2  /* y = Q_OO x on the Omega block (x, y of length n_Omega)     */
#define MDP_OP_QGG 3  /* y = Q_GG x on the Gamma block (x, y of length n_Gamma)     */

/* ---- blocks / matrices for inspection ------------------------------------- */
#define MDP_BLOCK_OMEGA 0 /* hierarchy built on S~ (eq. 7)   */
#define MDP_BLOCK_GAMMA 1 /* hierarchy built on A_GG (eq. 4) */
#define MDP_MAT_A 0
#define MDP_MAT_P 1
#define MDP_MAT_R 2

typedef struct mdp_handle mdp_handle;
typedef struct mdp_server mdp_server;

/* The system matrix A of eq. (4), any unknown order. */
typedef struct {
  int32_t n;              /* rows = columns                                */
  int64_t nnz;            /* row_ptr[n]                                    */
  const int32_t *row_ptr; /* n + 1 entries, non-decreasing, row_ptr[0] = 0 */
  const int32_t *col;     /* nnz entries in [0, n)                          */
  const double *val;      /* nnz entries                                    */
} mdp_csr;

typedef struct {
  int32_t precision;      /* MDP_FP64 (default) or MDP_MIXED                          */
  int32_t vcycles;        /* V-cycles per Q application (default 1, Section 3.3)      */
  int32_t pre_sweeps;     /* l1-Jacobi sweeps before the coarse correction (1; 1..8)  */
  int32_t post_sweeps;    /* l1-Jacobi sweeps after it (1; 1..8)                       */
  double strength_theta;  /* SA strength threshold (0.02)                              */
  int32_t max_coarse;     /* stop coarsening at or below this size (400)               */
  int32_t max_dense;      /* coarsest solved densely up to this size (2000); with
                             l1-Jacobi smoothing, a one-system solve also runs the
                             V-cycle from its first level l >= 1 of at most this size
                             down as one dense product (the same operator, formed at
                             upload in FP64)                                         */
  int32_t max_levels;     /* at most this many levels per hierarchy (10)               */
  int32_t restart;        /* FGMRES restart length m (64, at most 64)                  */
  int32_t max_iter;       /* total preconditioner applications per solve (1000)       */
  double rtol;            /* stop when ||b - A x|| <= rtol ||b|| (1e-8)                */
  uint32_t flags;         /* MDP_USE_X0 | MDP_HOST_ONLY | MDP_NO_AUTOTUNE | MDP_GRAPHS |
                             MDP_FALLBACK_FP64                                       */
  int32_t block_form;     /* MDP_BLOCK_LOWER (default), MDP_BLOCK_DIAG, MDP_BLOCK_UPPER */
  int32_t smoother;       /* MDP_SMOOTH_L1JACOBI (default) or MDP_SMOOTH_GS             */
} mdp_options;

typedef struct {
  int32_t iters;          /* preconditioner applications                       */
  int32_t restarts;       /* FGMRES cycles after the first                     */
  int32_t converged;      /* 1 if ||b - A x|| <= rtol ||b||                    */
  int32_t status;         /* MDP_OK, MDP_NOT_CONVERGED, MDP_STAGNATED or < 0  */
  double rel_res_true;    /* ||b - A x|| / ||b|| recomputed in FP64 at the end */
  double rel_res_est;     /* the Arnoldi estimate |g_{k+1}| / ||b||            */
  double setup_ms;        /* host + upload time of mdp_setup for this handle  */
  double solve_ms;        /* wall time of this solve                            */
  int32_t fallback;       /* 1 if MDP_FALLBACK_FP64 re-solved the column in FP64 */
} mdp_stats;

/* Fill *opt with the defaults listed above.  Returns MDP_OK or MDP_EINVAL
 * (NULL). */
int mdp_options_default(mdp_options *opt);

/* Build the solver for A (eq. 4).  part[i] = 0 marks an Omega unknown, 1 a
 * Gamma unknown.  Two readings of Section 3.1 are served the same way:
 * Omega = host-cell pressures and Gamma = fracture-cell pressures (the
 * primal pressure system), or Omega = the pressures of every subdomain
 * (host, fractures, intersection lines and points) and Gamma = the interface
 * fluxes of eq. (2) (the paper's own reading; A_GG is then diagonal and
 * A_GO = -A_OG^T).  Setup (host C++):
 * stable [Omega; Gamma] permutation, the four blocks, S~ of eq. (7) with
 * diag(A_GG), SA-AMG hierarchies on S~ and A_GG (Section 3.3), dense inverse
 * of each coarsest level, then one upload to the device on hip_stream, where
 * each matrix of at least 32k entries gets the fastest of its candidate
 * device formats, timed there (see MDP_NO_AUTOTUNE).
 * n_Gamma = 0 is allowed (M_L is then the AMG on A_OO).  A nonsymmetric A is
 * accepted (the paper does not rely on A_OG = A_GO^T).
 * Errors: EINVAL (NULL, n <= 0, malformed CSR, part not 0/1, bad options),
 * ENONPOS_DIAG, ENAN (non-finite value), ESINGULAR, ENOMEM, EHIP.
 * On success *out owns all device memory until mdp_destroy. */
int mdp_setup(const mdp_csr *A, const int32_t *part, const mdp_options *opt,
              void *hip_stream, mdp_handle **out);

/* mdp_setup with dimension-aware aggregation (Section 3.3, last paragraph:
 * aggregates built inside the subdomains of one dimension before crossing
 * dimensions): label[i] (n entries, host memory) is the dimension of the
 * subdomain of unknown i (any integers; equal labels share a subdomain
 * dimension).  On the finest level of each hierarchy a strong neighbour must
 * carry the same label; coarser levels are not restricted.  label = NULL is
 * mdp_setup.  Meant for the interface-flux reading, whose Omega block mixes
 * host, fracture, line and point unknowns.  Same errors as mdp_setup. */
int mdp_setup_labeled(const mdp_csr *A, const int32_t *part, const int32_t *label, const mdp_options *opt,
                      void *hip_stream, mdp_handle **out);

/* A second handle for the same system as src with other solve options
 * (typically the other precision), reusing src's host-built blocks and AMG
 * hierarchies instead of repeating the setup of eq. (7) and Section 3.3.
 * The AMG options (strength_theta, max_coarse, max_dense, max_levels) must
 * equal src's (EINVAL otherwise).  src is not modified and stays valid. */
int mdp_setup_like(const mdp_handle *src, const mdp_options *opt, void *hip_stream,
                   mdp_handle **out);

/* Write the complete host setup of h (the [Omega; Gamma] permutation, the
 * blocks of eq. (4), S~ of eq. (7) and both SA-AMG hierarchies of Section
 * 3.3, with the AMG options they were built with) to the file `path`, so
 * that mdp_load can re-create the handle without repeating the setup.
 * Binary, little-endian, with a tag, a format version and a 64-bit FNV-1a
 * checksum.  Version 2 also stores each level's fused restriction
 * R (I - A D^-1); version 1 files (without it) are still read, and their
 * V-cycles compute the residual and restrict it in two products.  EINVAL if
 * the file cannot be written. */
int mdp_save(const mdp_handle *h, const char *path);

/* Re-create a handle from a file written by mdp_save and upload it as
 * mdp_setup would (MDP_HOST_ONLY in opt skips the upload).  opt may be NULL
 * (defaults, with the file's AMG options); otherwise its AMG options
 * (strength_theta, max_coarse, max_dense, max_levels) must equal the file's.
 * The solve options (precision, vcycles, restart, ...) are free.  A file that
 * is missing, truncated, altered or inconsistent returns EINVAL with *out =
 * NULL. */
int mdp_load(const char *path, const mdp_options *opt, void *hip_stream, mdp_handle **out);

/* Release the handle and its device memory (NULL is a no-op). */
int mdp_destroy(mdp_handle *h);

/* Solve A x_k = b_k for nrhs right-hand sides stored column-major with
 * leading dimension ld (>= n) in device memory.  Zero initial guess unless
 * the handle's options carry MDP_USE_X0.  stats (nrhs entries, may be NULL)
 * receives the per-column result.  Returns MDP_OK when every column
 * converged, otherwise the most severe column status: a negative error (ENAN
 * for NaN/Inf in b or a breakdown producing one) before MDP_STAGNATED before
 * MDP_NOT_CONVERGED (x holds the last iterate of those columns).
 * With nrhs >= 4, columns are solved four at a time as one batch of this
 * system whose sparse products read each matrix once for all four (each
 * column keeps its own Krylov process; results equal one-column solves up to
 * rounding).  That batch (a four-fold copy of the system matrix and one copy
 * of the preconditioner) is built on first use and kept with the handle
 * until mdp_destroy; its four-column Krylov workspace is one per device,
 * shared by every handle's batch there (sized to the largest, released with
 * the last batch), so four-column solves on one device take turns.  The
 * batches and the shared workspaces together hold at most
 * MDP_MULTI_RHS_BYTES bytes of device memory (an environment variable, read
 * at each build; default a quarter of the device's memory): a handle whose
 * batch does not fit solves its columns one by one, and tries again once
 * others have been destroyed; one whose build ran out of device memory stays
 * with one column at a time.  Remaining columns are solved one by one.
 * Synchronises hip_stream before returning. */
int mdp_solve(mdp_handle *h, const double *b_dev, double *x_dev, int32_t nrhs,
              int64_t ld, void *hip_stream, mdp_stats *stats);

/* Solve several independent systems together: system s has nrhs[s]
 * right-hand sides in b_dev[s] / x_dev[s] (column-major, leading dimension
 * its own n).  All handles must share precision, block form, V-cycles,
 * smoother and sweep counts, restart, max_iter, rtol, MDP_USE_X0 and
 * MDP_GRAPHS (EINVAL otherwise).  The pairs
 * (system, rhs) are concatenated block-diagonally and every sparse product
 * runs once for all of them; each pair has its own Krylov process (per-pair
 * reductions never mix pairs), so its iterates are those of a solve of its
 * own up to the rounding of the sparse products, and a pair that has stopped
 * is skipped row by row.  When every system of a batch (or chunk) has
 * exactly four right-hand sides, the preconditioner's matrices are stored
 * once and each sparse product applies them to all four.  Batches above
 * MDP_BATCH_MAX_UNKNOWNS unknowns (an environment variable, default 48 Mi)
 * run as consecutive chunks on one workspace, cut between systems where a
 * system's right-hand sides fit together; the plan is kept while the same
 * handles, counts and bound come back.  stats has sum(nrhs) entries in
 * system-major order.  Synchronises hip_stream. */
int mdp_solve_batch(mdp_handle *const *hs, int32_t nsys, const double *const *b_dev,
                    double *const *x_dev, const int32_t *nrhs, void *hip_stream,
                    mdp_stats *stats);

/* One operator application y = op(x) with device vectors (see MDP_OP_*):
 * the building blocks of the solve, exposed for verification.
 * Synchronises hip_stream. */
int mdp_apply(mdp_handle *h, int32_t op, const double *x_dev, double *y_dev, void *hip_stream);

/* mdp_apply for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same operators and kernels as mdp_apply (the results are identical), but
 * the call allocates nothing and does not synchronise: it only enqueues the
 * launches on hip_stream, and y is complete when the stream reaches that
 * point.  In mixed precision the FP32 copies of x and y live in a fixed
 * device array of 64 MiB that the library holds on each GPU it runs on until
 * the process ends, so the operator's length (n, n_Omega or n_Gamma) is at
 * most 8,388,608 there (EINVAL beyond); FP64 operators use no extra memory.
 * All calls on one GPU share that array: calls that overlap in time on one
 * GPU (different streams, or threads) race on it and must be serialised by
 * the caller; calls on one stream are ordered and safe.  Refused (EINVAL)
 * for host-only handles, unknown operators and while kernel timers run. */
int mdp_apply_noalloc(mdp_handle *h, int32_t op, const double *x_dev, double *y_dev, void *hip_stream);

/* ---- introspection (host memory; works for MDP_HOST_ONLY handles) ---------- */

/* Sizes: n, n_Omega, n_Gamma and the number of levels of each hierarchy. */
int mdp_info(const mdp_handle *h, int32_t *n, int32_t *n_omega, int32_t *n_gamma,
             int32_t *levels_omega, int32_t *levels_gamma);

/* Residual history of the handle's last one-column solve (an mdp_solve
 * column solved alone or a served request; not four-column groups or
 * batches): the Arnoldi estimate |g_{k+1}| / ||b|| after each iteration, in
 * order across restarts (after a MDP_FALLBACK_FP64 re-solve, of the FP64
 * attempt).  *count (may be NULL) receives the number of iterations; the
 * first min(cap, count) values are copied to out (host memory).  EINVAL for
 * NULL h, cap < 0, or cap > 0 with NULL out. */
int mdp_residual_history(const mdp_handle *h, double *out, int32_t cap, int32_t *count);

/* Device memory of mdp_solve's four-column batches (any pointer may be
 * NULL): the bytes h's batch holds (0 before its first four-column solve or
 * when it did not fit), the bytes of the shared four-column Krylov workspace
 * of the device h's batch runs on (0 without a batch), and the bytes all
 * batches and shared workspaces hold together against the budget
 * MDP_MULTI_RHS_BYTES (its current value in *budget). */
int mdp_multi_rhs_memory(const mdp_handle *h, int64_t *plan_bytes, int64_t *shared_bytes, int64_t *held,
                         int64_t *budget);

/* Shape of one hierarchy matrix (block = MDP_BLOCK_*, mat = MDP_MAT_*, level
 * 0 = finest; P and R do not exist on the coarsest level). */
int mdp_level_shape(const mdp_handle *h, int32_t block, int32_t level, int32_t mat,
                    int32_t *rows, int32_t *cols, int64_t *nnz);

/* Copy one hierarchy matrix (FP64, as built on the host) into caller
 * buffers sized from mdp_level_shape.  Columns are sorted within rows. */
int mdp_level_export(const mdp_handle *h, int32_t block, int32_t level, int32_t mat,
                     int32_t *row_ptr, int32_t *col, double *val);

/* Aggregate label per node of a level (-1 = left unaggregated), n entries. */
int mdp_level_aggregates(const mdp_handle *h, int32_t block, int32_t level, int32_t *agg);

/* ---- serving: continuous batching over resident hierarchies -------------- */

/* A server owns max_slots worker threads (1..64), each with its own
 * non-blocking device stream at the default priority; up to max_slots
 * requests run on the device at once, on different handles (requests on a
 * handle that is already being solved wait).  Requests start in arrival order
 * as soon as they can be admitted: a free slot, an idle handle, and its Krylov
 * workspace (a handle's V and Z bases and step arrays, allocated on first use)
 * within mem_budget_bytes together with the workspaces of all registered
 * handles (0 = no bound).  To admit a request the server frees workspaces of
 * idle handles, least recently used first; a request whose workspace alone
 * exceeds the budget runs when no other request is running.  Grouping (off
 * by default, see mdp_server_set_grouping): the slot that admits a request
 * also takes every other queued request of the same handle, and solves all
 * their columns as mdp_solve solves the columns of one call (four at a time
 * through the handle's four-column batch within its memory budget, the rest
 * one by one).  Every kernel's reductions have a fixed order, so a column's
 * result depends only on the columns grouped with it (equal to its solve
 * alone up to rounding, as for mdp_solve), and without grouping it is bit
 * for bit the one-column mdp_solve result, whatever else runs.  Returns
 * EINVAL for bad arguments. */
int mdp_server_create(size_t mem_budget_bytes, int32_t max_slots, mdp_server **out);

/* Grouping of queued requests of one handle: 1, or 0 (the default: each
 * request alone, column by column).  Grouping pays once the handles' four-
 * column batches exist (hot systems of a long-running server): the first
 * grouped solve of a handle builds its batch inside the serving loop, and
 * grouped solves on one device take turns on the shared four-column
 * workspace.  Applies to requests admitted from now on.  EINVAL for NULL or
 * another value. */
int mdp_server_set_grouping(mdp_server *srv, int32_t on);

/* Columns solved so far, and how many of them four at a time (either may
 * be NULL).  EINVAL for NULL. */
int mdp_server_counts(mdp_server *srv, int64_t *columns, int64_t *grouped);

/* Make a handle servable.  Its hierarchy stays resident in device memory.
 * The handle must outlive the server (destroy the server first). */
int mdp_server_register(mdp_server *srv, mdp_handle *h);

/* Enqueue one solve (nrhs columns, leading dimension n, caller order, as in
 * mdp_solve).  Returns at once with a ticket.  b must already hold its values
 * when the call is made (synchronise the stream that wrote it first); b/x must
 * stay valid and untouched until mdp_poll reports a final code, after which x
 * is complete on the device.  EINVAL for an unregistered handle or after
 * destroy has begun, EBUSY if 2^20 requests are queued. */
int mdp_submit(mdp_server *srv, mdp_handle *h, const double *b_dev, double *x_dev,
               int32_t nrhs, uint64_t *ticket);

/* MDP_PENDING while the request runs; afterwards its final code, with
 * *stats (one entry per rhs, may be NULL) filled.  A ticket can be polled to
 * completion once. */
int mdp_poll(mdp_server *srv, uint64_t ticket, mdp_stats *stats);

/* Runs every queued request to completion, joins the workers and frees the
 * server; uncollected tickets are dropped.  Handles stay owned by the caller
 * (their workspaces may have been freed; they are re-created on demand). */
int mdp_server_destroy(mdp_server *srv);

/* ---- measurement ------------------------------------------------------ */

/* Kernel classes for mdp_ktimer_*. */
#define MDP_KC_OUTER_SPMV 0    /* w = A z_j with the FP64 system matrix                  */
#define MDP_KC_FINE_SMOOTH 1   /* finest S~ level: the l1-Jacobi sweeps after the first
                                  (post-smoothing, and pre-smoothing beyond one sweep)    */
#define MDP_KC_VCYCLE_OTHER 2  /* the rest of both V-cycles and the A_GO update          */
#define MDP_KC_ARNOLDI_DOT 3   /* fused reduction pass of each Arnoldi step              */
#define MDP_KC_ARNOLDI_AXPY 4  /* update pass of each Arnoldi step                       */
#define MDP_KC_OTHER 5         /* casts, reductions, Givens, update of x, residual       */
#define MDP_KC_FINE_RESID 6    /* finest S~ level: residual after the first sweep, whose
                                  iterate D^-1 b the producer of b has written already;
                                  where the level restricts with R (I - A D^-1), that
                                  one product instead                                    */

/* Start timing every launch of one kernel class (process-wide; not for use
 * while server slots are solving): HIP events
 * are recorded around each launch on the stream it is launched on, and the
 * launch's algorithmic bytes (each matrix value/index and each vector read
 * or written once) are accumulated.  Resets the class's counters. */
int mdp_ktimer_begin(int32_t kind);

/* Stop timing a class and report the summed kernel time (ms), the number of
 * launches and the algorithmic bytes.  Waits for the recorded events. */
int mdp_ktimer_end(int32_t kind, double *total_ms, int64_t *launches, double *bytes);

/* Keep the device-format autotuner's choices (see MDP_NO_AUTOTUNE) in the
 * text file `path`, one line per matrix signature (value size, rows,
 * columns, longest row, entries, sliced-ELL size) and format.  Choices
 * already recorded there are loaded now and used instead of timing, when the
 * matrix has that layout; every new choice is appended.  Setups in later
 * processes then pick the same formats, so their results are bit-identical
 * and their set-up skips the timing.  NULL stops recording (loaded choices
 * stay in use).  EINVAL if the file can neither be read nor created. */
int mdp_tune_file(const char *path);

/* ---- memory ----------------------------------------------------------- */

/* Route device allocations through the caller's allocator (e.g. a framework
 * caching allocator).  alloc(size, ctx) returns device memory or NULL;
 * free_(ptr, ctx) releases it.  Pass NULLs to restore hipMalloc/hipFree.
 * Affects allocations made after the call. */
int mdp_set_allocator(void *(*alloc)(size_t, void *), void (*free_)(void *, void *), void *ctx);

/* Message for the last failing call on this thread ("" if none). */
const char *mdp_last_error(void);

/* Library version string. */
const char *mdp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MDP_H */
