/*
 * mgr355.h - multigrid-reduction (MGR) preconditioned flexible GMRES on one AMD Instinct
 * MI355X (gfx950), as a C ABI.
 *
 * The method (Bui, Osei-Kuffuor, Castelletto, White, "A Scalable Multigrid Reduction
 * Framework for Multiphase Poromechanics of Heterogeneous Media"):
 *   - the Jacobian A of fully implicit multiphase poromechanics (Sec. 4, eq.
 *     block_linear_system) is solved with right-preconditioned GMRES (Sec. 4);
 *   - the preconditioner M is built level by level from a user-given C/F splitting of the
 *     rows by unknown type (Sec. 5.1, Sec. 5.3): Jacobi interpolation W_p = -D_FF^{-1} A_FC
 *     and injection restriction W_r = 0 (eq. injective_rp), coarse grid
 *     A_{l+1} = A_CC - G(A_CF D_FF^{-1} A_FC) with the optional dropping operator G
 *     (eq. drop_operator; without dropping this is the Galerkin product R~ A P~);
 *   - M^{-1} is applied by the V-cycle of Algorithm 2: global relaxation, F-relaxation,
 *     restriction of the residual, recursion, interpolation and correction; the coarsest
 *     grid and the F-relaxation of the displacement block use an algebraic multigrid
 *     V-cycle (smoothed aggregation, l1-Jacobi) or a dense solve.
 *
 * Conventions for every entry point
 *   - Pointers are DEVICE pointers unless marked [host].
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Work is
 *     ordered on that stream; entry points that must know sizes synchronise it (stated).
 *   - Matrices are CSR with int64 row pointers and int32 column indices, sorted and unique
 *     within each row; explicit zeros are part of the pattern.  Values are FP64.
 *   - Functions return mgr_status and never throw; on failure mgr_last_error() returns a
 *     message for the calling thread and outputs are left unwritten (unless stated).
 *   - The caller owns every array it passes; the library keeps no pointer to caller
 *     arrays after a call returns.  A handle owns its hierarchy until mgr_destroy().
 */
#ifndef MGR355_H
#define MGR355_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MGR_OK = 0,
  MGR_ERR_ARG = 1,            /* invalid argument, label, option or size               */
  MGR_ERR_ALLOC = 2,          /* device allocation failed                               */
  MGR_ERR_HIP = 3,            /* a HIP runtime call failed                              */
  MGR_ERR_ZERO_PIVOT = 4,     /* zero/missing diagonal in D_FF, an AMG level, or a
                                 singular dense or block-diagonal inverse               */
  MGR_ERR_NOT_CONVERGED = 5,  /* FGMRES reached maxit; x holds the last iterate         */
  MGR_ERR_PATTERN = 6,        /* mgr_setup_numeric: sparsity pattern differs            */
  MGR_ERR_UNSUPPORTED = 7     /* a size or structure outside the documented limits     */
} mgr_status;

/* ---------------------------------------------------------------------------------- */
typedef struct {
  int64_t nrows, ncols;        /* [host] rows / columns; of blocks when block > 1     */
  const int64_t *row_ptr;      /* nrows + 1 entries, row_ptr[0] = 0, nondecreasing     */
  const int32_t *col;          /* row_ptr[nrows] entries (block columns when block > 1) */
  const double *val;           /* row_ptr[nrows] entries; when block > 1,
                                  row_ptr[nrows] * block^2 values, each block's
                                  entries row-major                                    */
  int32_t block;               /* [host] 0 or 1: CSR; 2 or 3: BSR with block x block
                                  blocks (scalar row br*block + r, column bc*block + c);
                                  a zero-initialised descriptor is CSR                 */
  int32_t reserved;            /* must be 0                                            */
} mgr_csr;

/* Algebraic multigrid used for F-relaxation and for the coarsest grid.  Smoothed
 * aggregation: strength |a_ij| >= theta_l sqrt(|a_ii a_jj|) (squared Frobenius norms of
 * bxb blocks when block = 3), theta_l = theta0 * 0.5^l; MIS(2) aggregation with SplitMix64
 * priorities; P = (I - omega D^{-1} A) T, omega = (4/3)/max_i(sum_j|a_ij|/|a_ii|);
 * A_c = P^T A P; one l1-Jacobi pre- and post-sweep; dense inverse at the coarsest level. */
typedef struct {
  double theta0;               /* default 0.08                                           */
  int32_t max_levels;          /* default 10                                             */
  int32_t coarse_size;         /* dense solve when n <= coarse_size; default 256, max 4096 */
} mgr_amg_opts;

enum { MGR_INTERP_JACOBI = 0, MGR_INTERP_ZERO = 1 };
enum { MGR_FRELAX_JACOBI = 0, MGR_FRELAX_AMG = 1, MGR_FRELAX_DENSE = 2 };
enum { MGR_GSMOOTH_NONE = 0, MGR_GSMOOTH_BLOCK_JACOBI = 1, MGR_GSMOOTH_BLOCK_GS = 2,
       MGR_GSMOOTH_ILU = 3 };
enum { MGR_COARSE_AMG = 0, MGR_COARSE_DENSE = 1 };
enum { MGR_COUPLING_FULL = 0, MGR_COUPLING_QUASI_IMPES = 1 };
enum { MGR_RESTRICT_INJECTION = 0, MGR_RESTRICT_JACOBI = 1 };
enum { MGR_PREC_FP64 = 0, MGR_PREC_FP32 = 1 };

/* One reduction level (Sec. 5.2, Algorithm 2). */
typedef struct {
  uint32_t f_label_mask;       /* bit t set: rows with label t are F-points               */
  int32_t interp;              /* MGR_INTERP_JACOBI (eq. injective_rp) or _ZERO (W_p = 0) */
  int32_t nmax_drop;           /* < 0: no dropping (Galerkin); >= 0: N_max of G, kept in
                                  addition to the sub-block diagonals (eq. drop_operator) */
  int32_t frelax;              /* MGR_FRELAX_*: Jacobi sweeps, one AMG V-cycle on A_FF, or
                                  a dense solve with A_FF (n_F <= 4096)                  */
  int32_t frelax_sweeps;       /* Jacobi sweeps (default 1)                              */
  double frelax_omega;         /* Jacobi weight (default 1.0)                            */
  int32_t frelax_block;        /* 1 scalar AMG, 3 nodal AMG with 3x3 block storage; the F
                                  rows must then come in consecutive triples with full
                                  3x3 block patterns                                     */
  int32_t global_smoother;     /* MGR_GSMOOTH_*: block Jacobi over same-cell blocks, or
                                  multicolour block Gauss-Seidel over them (the hybrid
                                  block Gauss-Seidel of the Sec. 5.3 remarks, cells
                                  coloured by Jones-Plassmann rounds, sweeps in colour
                                  order from z = 0; global_omega unused), i.e.
                                  rows of equal rank within their label; the level's rows
                                  must be interleaved cell by cell                       */
  int32_t global_sweeps;       /* default 1                                              */
  int32_t coupling;            /* A_CF in the coarse product A_CF D_FF^{-1} A_FC:
                                  MGR_COUPLING_FULL (eq. coarse_grid_pressure, default) or
                                  MGR_COUPLING_QUASI_IMPES: only its entries between points
                                  of the same entity (equal rank within their labels), the
                                  diagonal that the quasi-IMPES reduction described with
                                  that equation uses; W_p and residuals keep all of A_CF  */
  double global_omega;         /* weight of sweeps after the first (default 1.0)         */
  double drop_tol;             /* >= 0: the tolerance form of G named beside eq.
                                  drop_operator instead of N_max (nmax_drop must be < 0):
                                  an entry off the sub-block diagonals is kept when it is
                                  nonzero and its |value| >= drop_tol times the largest
                                  |value| of its row; < 0: off (default)                */
  /* MGR_GSMOOTH_ILU: the pointwise ILU(k) global smoother of the Sec. 5.3 remarks and
     Sec. 6 by the fine-grained fixed-point method (Chow and Patel), factorising the level
     matrix left-scaled by its same-cell block inverses, D_B^{-1} A_l; one step is
     z (+)= (LU)^{-1} D_B^{-1} (v - A_l z), the first from z = 0, later ones weighted by
     global_omega; the rows must be interleaved cell by cell as for block Jacobi         */
  int32_t ilu_level;           /* k of ILU(k): 0 or 1 (default 1)                        */
  int32_t ilu_sweeps;          /* fixed-point sweeps of the factorisation, 0..100 (3)    */
  int32_t ilu_tri_sweeps;      /* Jacobi sweeps per triangular solve, 0..100 (3)         */
  int32_t restrict_;           /* MGR_RESTRICT_INJECTION (W_r = 0, eq. injective_rp,
                                  default) or MGR_RESTRICT_JACOBI: R~ = [W_r I] with
                                  W_r = -A_CF D_FF^{-1} (Sec. 5.1); the coarse grid is then
                                  A_CC - G(A_CF M + N A_FC - N A_FF M), M = D_FF^{-1} A_FC,
                                  N = A_CF D_FF^{-1} (each product in the pinned order), and
                                  the restricted residual r_C + W_r r_F.  Needs
                                  MGR_COUPLING_FULL and MGR_INTERP_JACOBI               */
  int32_t dff_block;           /* D_FF: 1 pointwise diagonal (eq. injective_rp, default);
                                  2 or 3: the diagonal blocks of that many consecutive F
                                  rows (a node's displacement components; the dense
                                  blocks of the Sec. 5.3 remark), inverted by their
                                  closed form, for W_p, W_r and Jacobi F-relaxation     */
  int32_t reserved1;           /* must be 0                                              */
} mgr_level_opts;

#define MGR_MAX_LEVELS 8

typedef struct {
  int32_t nlevels;                       /* number of reductions, 1..MGR_MAX_LEVELS     */
  mgr_level_opts level[MGR_MAX_LEVELS];
  int32_t coarse;                        /* MGR_COARSE_AMG or MGR_COARSE_DENSE (n<=4096) */
  mgr_amg_opts amg_frelax;               /* AMG used by MGR_FRELAX_AMG levels            */
  mgr_amg_opts amg_coarse;               /* AMG used on the coarsest grid                */
  int32_t precision;                     /* MGR_PREC_FP64 or MGR_PREC_FP32: storage and
                                            arithmetic of the whole hierarchy in apply;
                                            setup always runs in FP64                    */
  int32_t use_graph;                     /* 1: capture the apply V-cycle in a HIP graph  */
  int32_t keep_setup;                    /* 1: keep the FP64 setup matrices for export   */
} mgr_opts;

typedef struct mgr_handle mgr_handle;

/* Fill `o` with defaults: zero levels, coarse AMG, FP64, graphs on, level defaults as
 * documented above.  [host] */
void mgr_default_opts(mgr_opts *o);

/* Build the MGR hierarchy for A (Sec. 5.2: per level the C/F split by label, D_FF,
 * W_p = -D_FF^{-1} A_FC, A_cor = A_CF D_FF^{-1} A_FC by sparse product with a fixed
 * summation order, G, A_{l+1} = A_CC - G(A_cor); then the AMG and dense solvers).
 *   A        square CSR, n = A->nrows; nnz < 2^31.
 *   labels   n int8 labels in [0, 7] (unknown type of every row).
 *   opts     [host] options.
 *   out      [host] receives the new handle on success.
 * Synchronises `stream` (sizes of the coarse operators are data dependent), also when it
 * fails.  A's arrays are read during the call only (the handle copies what it keeps), so
 * the caller may free or overwrite them once mgr_setup returns.
 * Errors: ARG (labels outside [0,7], empty F or C set, bad options, A not square),
 * ZERO_PIVOT, UNSUPPORTED (a row of an intermediate product beyond 1 << 20 entries, a
 * dense solve beyond 4096 unknowns, a nodal level without full 3x3 blocks), ALLOC, HIP. */
mgr_status mgr_setup(const mgr_csr *A, const int8_t *labels, const mgr_opts *opts,
                     void *stream, mgr_handle **out);

/* Rebuild the hierarchy of `h` for a new matrix with exactly the same pattern as the one
 * given to mgr_setup (e.g. the next Newton step), keeping the handle, its options, labels
 * and captured-graph stream: the pattern is checked against the original by a hash, then
 * every level is rebuilt from the new values (the symbolic work is redone too, since G and
 * the AMG aggregates depend on values), so the result equals a fresh mgr_setup.  Waits for
 * the setup stream and for the last apply of the handle before releasing the old
 * hierarchy.  Synchronises `stream`.  Errors: PATTERN (size or row pointer / column arrays
 * differ; the old hierarchy is kept and stays usable), ARG, ZERO_PIVOT, ALLOC, HIP; after
 * any error other than PATTERN and ARG the handle holds no hierarchy: mgr_apply and
 * fgmres_solve reject it with ARG until a later mgr_setup_numeric succeeds, and it must
 * still be destroyed. */
mgr_status mgr_setup_numeric(mgr_handle *h, const mgr_csr *A, void *stream);

/* z = M^{-1} v (Algorithm 2).  v and z are FP64 vectors of length n; they may not alias.
 * With MGR_PREC_FP32 the vector is rounded to FP32 at entry and z widened at exit.
 * Asynchronous on `stream`; calls that overlap on one handle race (one work area per
 * handle).  Errors: ARG (null pointers), HIP. */
mgr_status mgr_apply(mgr_handle *h, const double *v, double *z, void *stream);

typedef struct {
  int32_t restart;            /* m, Krylov vectors per cycle (1..64), default 30       */
  int32_t maxit;              /* total preconditioner applications, default 1000       */
  double rtol;                /* stop when ||b - A x|| <= rtol ||b|| (FP64)             */
} fgmres_opts;

typedef struct {
  int32_t iters;              /* preconditioner applications                           */
  int32_t restarts;           /* cycles started after the first                        */
  int32_t converged;          /* 1 if the true residual met rtol                       */
  double true_relres;         /* ||b - A x|| / ||b|| recomputed in FP64 at the end      */
  double est_relres;          /* last Givens estimate |g_{j+1}| / ||b||                */
  double *history;            /* [host] optional, history_cap entries: relative residual
                                 estimate after every iteration (plus one entry per
                                 restart: the true relative residual)                  */
  int32_t history_cap;
  int32_t history_len;        /* entries written                                       */
} fgmres_result;

/* Bytes of device workspace fgmres_solve needs for n unknowns and restart m. [host] */
size_t fgmres_workspace_bytes(int64_t n, int32_t restart);

/* Solve A x = b by flexible GMRES(m) (Saad 1993; equal to right-preconditioned GMRES,
 * Sec. 4, for a fixed M), FP64 throughout: SpMV, classical Gram-Schmidt with one
 * re-orthogonalisation, norms, Givens rotations, x = x0 + Z y.  After every cycle the
 * true residual is recomputed; the solve ends when it is <= rtol ||b||.
 *   A      the FP64 matrix (may be the one given to mgr_setup).
 *   M      preconditioner handle, or NULL for M = I.
 *   b      n entries.  x  n entries: initial guess in, solution out.
 *   work   device workspace of at least fgmres_workspace_bytes(n, m) bytes, or NULL to let
 *          the library allocate and free it inside the call.
 *   res    [host] result record (may be NULL).
 * Synchronises `stream` once per iteration (the convergence test).
 * Errors: ARG, NOT_CONVERGED (x holds the last iterate, res filled), ALLOC, HIP. */
mgr_status fgmres_solve(const mgr_csr *A, mgr_handle *M, const double *b, double *x,
                        const fgmres_opts *o, void *work, size_t work_bytes,
                        fgmres_result *res, void *stream);

/* fgmres_solve for callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same solve, the same launches in
 * the same order and bitwise the same x and res, with the Krylov workspace in a static
 * device array of fgmres_noalloc_max_bytes() = 64 MiB per device (held from the
 * library's first use on that device until the process ends) instead of a caller or
 * library allocation.  Nothing is allocated or created inside the call: read-backs go to
 * host stack memory and the host waits on `stream` itself.
 *   A, M, b, x, o, res   as for fgmres_solve.  M, when not NULL, must have been applied at
 *          least once (mgr_apply or fgmres_solve), which captures its graph.
 * The static workspace keeps the last call's contents; the solve writes every part of it
 * before reading it, so nothing needs clearing.  Every call on one device shares that
 * device's array: calls that overlap on one device (other streams or host threads) race
 * and must be serialised by the caller.
 * Errors: ARG (fgmres_workspace_bytes(n, restart) above the static size, an M that has
 * not been applied yet, and those of fgmres_solve), NOT_CONVERGED, HIP. */
size_t fgmres_noalloc_max_bytes(void);
mgr_status fgmres_solve_noalloc(const mgr_csr *A, mgr_handle *M, const double *b, double *x,
                                const fgmres_opts *o, fgmres_result *res, void *stream);

/* Batched solve of k independent systems A_i x_i = b_i (i < k) of any sizes under one set
 * of options, for small systems whose solves are bound by launch latency.  The systems are
 * placed on the diagonal of one block-diagonal matrix, which gets one MGR setup (Sec. 5:
 * every step of it is row-local and no AMG aggregate crosses two systems, so the
 * hierarchy is that of each system, up to the AMG's random priorities and its coarsest
 * dense level) and one FGMRES(m) in which every system keeps its own Arnoldi process
 * (basis coefficients, Hessenberg matrix, Givens rotations, restarts and the test
 * ||b_i - A_i x_i|| <= rtol ||b_i||); the SpMV, the preconditioner and the Gram-Schmidt
 * passes are shared launches over the union.  A converged system stops contributing.
 *   A       [host] array of k matrices (device arrays), square, row_ptr[0] = 0.
 *   labels, b, x   [host] arrays of k device pointers; x: initial guesses in, solutions
 *           out (x_i = 0 where b_i = 0).
 *   relres  [host] k entries out: ||b_i - A_i x_i|| / ||b_i|| (0 where b_i = 0).
 *   iters   [host] optional, k entries out: iterations of each system.
 *   res     [host] optional: iters = steps of the shared loop (the largest iters[i]),
 *           true_relres = the largest relres[i], converged; no history is recorded.
 * Allocates the union (matrix, vectors, hierarchy and Krylov workspace) for the call and
 * frees it before returning; synchronises `stream` once per step.
 * Errors: ARG (k outside 1..65535, null pointers, a non-square or empty system, a
 * non-finite b, restart outside 1..64), UNSUPPORTED (the union has 2^31 rows or entries
 * or more), NOT_CONVERGED (some relres[i] > rtol after maxit steps; x and relres filled),
 * and those of mgr_setup. */
mgr_status mgr_batch_solve(int32_t k, const mgr_csr *A, const int8_t *const *labels,
                           const double *const *b, double *const *x, const mgr_opts *opts,
                           const fgmres_opts *o, double *relres, int32_t *iters,
                           fgmres_result *res, void *stream);

/* Free every device allocation of the handle, after waiting for the setup stream and for
 * the stream of the handle's last mgr_apply / fgmres_solve (applies of one handle on
 * different streams must be ordered by the caller: they share the handle's work vectors).
 * NULL is ignored. */
void mgr_destroy(mgr_handle *h);

/* Bytes of device memory the handle holds. [host out] */
mgr_status mgr_footprint(const mgr_handle *h, size_t *bytes);

/* Upper bound of the device bytes mgr_setup will hold for a matrix with n rows and nnz
 * entries under `opts` (peak including setup temporaries), computed on the host from the
 * sizes only. [host in/out] */
mgr_status mgr_estimate_footprint(int64_t n, int64_t nnz, const mgr_opts *opts,
                                  size_t *bytes);

/* Route every device allocation of the library through caller functions (e.g. a caching
 * allocator).  Pass NULLs to restore the default: the library's own caching allocator over
 * hipMalloc (described with mgr_release_cache below).  Not thread-safe with respect to
 * concurrent calls. [host] */
void mgr_set_allocator(void *(*alloc_fn)(size_t bytes, void *stream, void *ctx),
                       void (*free_fn)(void *ptr, void *stream, void *ctx), void *ctx);

/* Message of the last failing call on this thread ("" if none). [host] */
const char *mgr_last_error(void);

/* The default allocator keeps freed device blocks for reuse on the stream they were freed
 * on (size-binned free lists); a failing allocation releases the cache and retries.
 * mgr_release_cache synchronises the device and returns every cached block to HIP;
 * mgr_cached_bytes reports the bytes held in the cache. [host] */
mgr_status mgr_release_cache(void);
size_t mgr_cached_bytes(void);
/* Bytes currently handed out by the default allocator and the peak since the last reset
 * (reset_peak != 0 sets the peak to the current value). [host] */
void mgr_alloc_stats(size_t *live, size_t *peak, int32_t reset_peak);

/* ---------------------------------------------------------------------------------- */
/* Serving: a request loop over mgr_setup / mgr_setup_numeric / fgmres_solve with HBM
 * admission, a setup cache across requests of one key, and concurrent HIP streams.
 * `slots` worker threads each own a stream; an admitted request runs on a free slot while
 * others run on theirs, so solves of different requests overlap on the device.  Admission
 * is first-in first-out by the request's peak footprint (mgr_estimate_footprint for a
 * fresh setup, plus the FGMRES workspace) against budget_bytes; idle cached setups are
 * evicted least recently used first.  A request larger than the whole budget completes
 * with MGR_ERR_ALLOC.  Requests that share `key` run one at a time in submission order and
 * share the cached setup when the matrix has the same size (e.g. the Newton steps of one
 * realization): reused as is (refresh_setup = 0, a lagged preconditioner) or recomputed
 * with mgr_setup_numeric (refresh_setup = 1).
 * Small requests can be batched (batch_rows > 0): a request of at most batch_rows rows
 * whose key has no cached setup is solved together with the other such requests admissible
 * at that moment (up to batch_max of them, keys not in flight) by mgr_batch_solve, on one
 * slot; batched requests leave no cached setup. */
typedef struct mgr_server mgr_server;
typedef struct {
  size_t budget_bytes;        /* HBM admission budget (default 64 GiB)                 */
  int32_t slots;              /* concurrent requests on the device, 1..64 (default 4) */
  mgr_opts opts;              /* MGR options of every request                           */
  fgmres_opts fopts;          /* FGMRES options (default restart 30, rtol 1e-6)         */
  int32_t cache_setups;       /* keep setups between requests of a key (default 1)     */
  int32_t batch_rows;         /* batch requests of at most this many rows (default 0:
                                 no batching)                                          */
  int32_t batch_max;          /* requests per batch, 1..65535 (default 16)             */
} mgr_server_config;
typedef struct {
  const mgr_csr *A;           /* [host struct, device arrays] valid until completion   */
  int64_t nnz;                /* [host] A->row_ptr[A->nrows]                            */
  const int8_t *labels;       /* n labels                                              */
  const double *b;            /* right-hand side                                       */
  double *x;                  /* initial guess in, solution out                        */
  uint64_t key;               /* setup-cache key                                       */
  int32_t refresh_setup;      /* 1: mgr_setup_numeric on a cached setup; 0: reuse it  */
  int32_t last_use;           /* 1: drop the key's cached setup after this request     */
} mgr_request;
typedef struct {
  int32_t status;             /* mgr_status of the request                             */
  int32_t iters;              /* FGMRES iterations                                     */
  int32_t setup_reused;       /* 1 if a cached setup served it                         */
  int32_t slot;               /* worker slot that ran it                               */
  double true_relres;         /* FP64 relative residual recomputed at the end          */
  double t_submit_ms, t_admit_ms, t_start_ms, t_end_ms;  /* since server creation      */
  double setup_ms, solve_ms;
  size_t footprint;           /* bytes of the setup that served it                     */
  int32_t batch;              /* requests solved together with it (1: alone); for a
                                 batch, setup_ms is 0 and solve_ms covers the batched
                                 setup and solve                                        */
} mgr_result;
typedef struct {
  int64_t completed, queued, cache_hits, cache_misses, evictions, cached_setups;
  size_t reserved_bytes, peak_reserved_bytes;
} mgr_server_stats_t;

void mgr_server_default_config(mgr_server_config *c);                       /* [host] */
/* Start the worker threads.  Errors: ARG. */
mgr_status mgr_server_create(const mgr_server_config *cfg, mgr_server **out);
/* Queue a request (non-blocking); *ticket identifies it.  Errors: ARG. */
mgr_status mgr_server_submit(mgr_server *s, const mgr_request *r, uint64_t *ticket);
/* Block until the request completes; returns its status and fills *res (may be NULL).
 * A ticket can be waited on once. */
mgr_status mgr_server_wait(mgr_server *s, uint64_t ticket, mgr_result *res);
/* 1 if done, 0 if pending, -1 if unknown. */
int32_t mgr_server_poll(mgr_server *s, uint64_t ticket);
mgr_status mgr_server_stats(mgr_server *s, mgr_server_stats_t *out);
/* Finish every queued request, stop the workers and free the cached setups; the memory
 * they held, and every other block the library's allocator keeps cached, goes back to HIP
 * (as mgr_release_cache). */
void mgr_server_destroy(mgr_server *s);

/* ---------------------------------------------------------------------------------- */
/* Inspection of a hierarchy (tests, diagnostics).  `what` selects an object:           */
enum {
  MGR_X_LEVEL_A = 0,   /* A_l (level 0: copy of the input)                         CSR */
  MGR_X_F = 1,         /* F index list of level l (ascending)               int in col */
  MGR_X_C = 2,         /* C index list of level l                           int in col */
  MGR_X_WP = 3,        /* W_p = -D_FF^{-1} A_FC                                    CSR */
  MGR_X_ACOR = 4,      /* A_cor = A_CF D_FF^{-1} A_FC before dropping              CSR */
  MGR_X_G = 5,         /* G(A_cor)                                                 CSR */
  MGR_X_COARSE = 6,    /* A_{l+1} = A_CC - G(A_cor)                                CSR */
  MGR_X_AMG_A = 7,     /* AMG level `sub` matrix of level l's F-relaxation AMG
                          (l = nlevels: the coarsest-grid AMG)                     CSR */
  MGR_X_AMG_P = 8,     /* AMG prolongator of level `sub`                           CSR */
  MGR_X_AMG_AGG = 9,   /* AMG aggregate id per node (-1: none)              int in col */
  MGR_X_AMG_NLEV = 10, /* number of AMG levels in out[0]                               */
  MGR_X_GS_COLOR = 11, /* colour of every same-cell block of level l (block
                          Gauss-Seidel smoother)                            int in col */
  MGR_X_ILU = 12,      /* ILU global smoother of level l: the factors on the ILU(k)
                          pattern of D_B^{-1} A_l (l_ij below the diagonal, u_ij on
                          and above)                                               CSR */
  MGR_X_WR = 13        /* W_r = -A_CF D_FF^{-1} (Jacobi restriction)               CSR */
};
/* Sizes of an object: out[0] = rows, out[1] = cols, out[2] = entries. [host out]
 * Requires opts.keep_setup = 1 for the CSR objects.  Errors: ARG. */
mgr_status mgr_query(const mgr_handle *h, int32_t what, int32_t level, int32_t sub,
                     int64_t out[3]);
/* Copy an object into caller arrays sized by mgr_query (row_ptr may be NULL for index
 * lists, val NULL to skip values).  Synchronises `stream`.  Errors: ARG, HIP. */
mgr_status mgr_export(const mgr_handle *h, int32_t what, int32_t level, int32_t sub,
                      int64_t *row_ptr, int32_t *col, double *val, void *stream);

/* ---------------------------------------------------------------------------------- */
/* Building blocks and measurement hooks.                                               */

/* y = A x with the FP64 CSR kernel used by fgmres_solve.  Asynchronous. */
mgr_status mgr_spmv(const mgr_csr *A, const double *x, double *y, void *stream);

/* Setup building blocks on caller matrices, each the same kernel the setup uses.  Results
 * are owned by an mgr_owned_csr (sizes[3] = rows, cols, entries), copied out with
 * mgr_owned_export into caller arrays of those sizes, and freed with mgr_owned_free.
 * All synchronise `stream`. */
typedef struct mgr_owned_csr mgr_owned_csr;
/* C = A B with the pinned summation order of the coarse-grid correction (Sec. 5.2):
 * c_ij = sum over ascending k of a_ik * b_kj, separate roundings, from +0.0; the pattern
 * keeps entries that cancel.  Errors: ARG, UNSUPPORTED (a row beyond 2^21 entries). */
mgr_status mgr_spgemm(const mgr_csr *A, const mgr_csr *B, mgr_owned_csr **C, int64_t sizes[3],
                      void *stream);
/* The same product C = A B (pattern and values equal to mgr_spgemm's to the bit), computed
 * `group` (2 or 3) consecutive rows of A at a time when every group's rows share one column
 * pattern, as the C rows of a cell do in A_CF for the coarse-grid correction (Sec. 5.2):
 * the group shares its symbolic count, the loads of B and the table of output columns.
 * Groups whose patterns differ, or output rows beyond 256 entries, take the row-by-row
 * path.  Errors: ARG (group not 1..3), as mgr_spgemm otherwise. */
mgr_status mgr_spgemm_grouped(const mgr_csr *A, const mgr_csr *B, int32_t group,
                              mgr_owned_csr **C, int64_t sizes[3], void *stream);
/* C = A B for matrices made of full 3x3 blocks (nodal elasticity levels of the AMG that
 * relaxes the displacement block, Sec. 5.3), computed on the block patterns with the same
 * per-entry products, roundings and order as mgr_spgemm on the scalar matrices, so the
 * result equals mgr_spgemm's bit for bit.  A and B are scalar CSR whose dimensions are
 * multiples of 3 and whose every 3x3 block is either absent or has all nine entries stored
 * (zeros included).  With diag_b != 0 only the diagonal of each block of B is used (the
 * tentative prolongator's form): the result is mgr_spgemm(A, B') where B' keeps the
 * diagonal entries of B's blocks.  C is returned with full 3x3 blocks.  Errors: ARG,
 * UNSUPPORTED (sizes not multiples of 3, a block not fully stored). */
mgr_status mgr_spgemm_b3(const mgr_csr *A, const mgr_csr *B, int32_t diag_b, mgr_owned_csr **C,
                         int64_t sizes[3], void *stream);
/* T = A^T (rows sorted by column). */
mgr_status mgr_transpose(const mgr_csr *A, mgr_owned_csr **T, int64_t sizes[3], void *stream);
/* S = A - diag(w) G(B) on the union pattern (eq. drop_operator with w = NULL; the AMG
 * prolongator P = T - diag(omega / a_ii) (A T) with w given).  nmax < 0 keeps all of B;
 * otherwise per row of B the entries whose coarse points have equal rank within their
 * label (labels_c, one per row/column of B) plus the nmax largest |b| (ties: smaller
 * column).  Errors: ARG. */
mgr_status mgr_merge_drop(const mgr_csr *A, const mgr_csr *B, const double *w, int32_t nmax,
                          const int8_t *labels_c, mgr_owned_csr **S, int64_t sizes[3],
                          void *stream);
/* Incomplete factors of A on its ILU(level) pattern (level 0 or 1: A's pattern, or A's
 * united with the level-1 fill of strict_lower(A) * strict_upper(A)), after `sweeps`
 * synchronous fixed-point sweeps from l_ij = a_ij / a_jj, u_ij = a_ij (the fine-grained
 * ILU named for the global smoother in the Sec. 5.3 remarks): one CSR holding l_ij below
 * the diagonal and u_ij on and above it, +0.0 on fill before the sweeps.  Each component
 * s_ij = a_ij - sum_{m < min(i,j)} l_im u_mj is accumulated in ascending m with separate
 * roundings.  Errors: ARG, ZERO_PIVOT (missing or zero diagonal), UNSUPPORTED (a row of
 * the pattern longer than 256, or level > 1). */
mgr_status mgr_ilu(const mgr_csr *A, int32_t level, int32_t sweeps, mgr_owned_csr **F,
                   int64_t sizes[3], void *stream);
/* Inverse of the dense n x n row-major matrix D into Inv (n x n row-major; both device,
 * not aliased): the coarsest-grid inverse of the setup, by Gauss-Jordan elimination with
 * partial pivoting (first row of largest |a| in the column), FP64: the matrix in LDS for
 * n <= 128, blocked in panels of 16 columns for n <= 512, streamed through global memory
 * above.  Synchronises `stream`.  Errors: ARG (n outside [1, 4096]), ZERO_PIVOT (a column
 * with no nonzero candidate: singular, or NaN). */
mgr_status mgr_dense_inverse(const double *D, double *Inv, int32_t n, void *stream);
/* The br x bc block CSR ((br, bc) = (2, 2), (3, 3) or (2, 3)) of a CSR matrix whose rows
 * come in groups of br (the unknowns of a cell) and whose columns come in groups of bc: the
 * storage of the level matrices for the block-Jacobi sweeps (Sec. 5.3 remarks on the
 * global smoother) and of A_CF for the restriction of the residual (eq. MGR-pre).  Block
 * row I holds the distinct column groups c / bc of scalar rows br I .. br I + br - 1 in
 * ascending order, each stored whole (row-major br x bc values, entries absent from A zero;
 * an explicit zero of A keeps its block).  Called twice: with bcol == NULL only *nblk is
 * set; then brow_ptr (nrows/br + 1 int32), bcol (capacity int32) and bval (capacity br bc
 * doubles), all device, receive the matrix when capacity >= *nblk.  Columns of every row
 * must ascend without repeats.  Synchronises `stream`.  Errors: ARG (another shape, nrows
 * not a multiple of br or ncols of bc, capacity below the block count). */
mgr_status mgr_csr_to_bsr(const mgr_csr *A, int32_t br, int32_t bc, int32_t *brow_ptr,
                          int32_t *bcol, double *bval, int64_t capacity, int64_t *nblk,
                          void *stream);
/* Strength graph (bs = 1 scalar, 3 nodal), SplitMix64 priorities of AMG level `level`,
 * MIS(2) and aggregation; agg receives nrows/bs aggregate ids (-1 = none). */
mgr_status mgr_aggregate(const mgr_csr *A, int32_t bs, double theta, int32_t level,
                         int32_t *agg, int64_t *nagg, void *stream);
mgr_status mgr_owned_export(const mgr_owned_csr *C, int64_t *row_ptr, int32_t *col,
                            double *val, void *stream);
void mgr_owned_free(mgr_owned_csr *C);

/* dst = src for n doubles with a plain streaming kernel (HBM counter calibration). */
mgr_status mgr_stream_copy(const double *src, double *dst, int64_t n, void *stream);

/* Per-kernel timing with HIP events recorded on the launching stream around every launch
 * of the named kernel family, inside mgr_apply / fgmres_solve of `h`:
 *   family 0 = nodal (3x3 block) AMG smoothing sweeps, 1 = outer FP64 CSR SpMV.
 * enable != 0 starts a new accumulation; mgr_profile_read synchronises and returns the
 * number of launches timed, their total milliseconds, and the algorithmic bytes they move
 * (matrix values and indices, row pointers, and each vector read or written once). */
mgr_status mgr_profile_enable(int32_t family, int32_t enable);
mgr_status mgr_profile_read(int32_t family, int64_t *launches, double *total_ms,
                            double *bytes);

/* ---------------------------------------------------------------------------------- */
/* Residual and Jacobian of two-phase poromechanics, and Newton time steps (Sec. 2-4).
 *
 * The fully discrete system of Sec. 3 (eq. IBVP_G; F(x) = 0 of eq. IBVP_G_res) for the
 * displacement / wetting saturation / pressure model of Sec. 2 on nx x ny x nz unit cubes:
 * trilinear displacement, cell-wise constant (s, p), two-point fluxes with harmonic
 * transmissibility and first-order upwinding on the phase potential (ties: the lower cell
 * index is upwind), backward Euler.  Model choices: porosity phi0 + b eps_v(u) with eps_v
 * the cell integral of div u; mixture weight (1 - phi0) rho_s + phi0 (rho_w s +
 * rho_nw (1 - s)); rho_l = rho0_l exp(c_l (p - p_ref)); k_rw = max(s, 0)^2,
 * k_rnw = max(1 - s, 0)^2; wells as fixed mass injection per phase and producers
 * q_l = -WI rho_l lambda_l (p - p_bhp); a mass row is accumulation + outflow - source;
 * Dirichlet displacement dofs are fixed at zero (their rows are K_dd u_d, their columns
 * eliminated).  Unknowns: displacement dofs node-major (x/y/z interleaved, nodes x fastest),
 * then (s, p) per cell (cells x fastest); rows in the same order, a cell's wetting-phase
 * mass balance on its s row and non-wetting on its p row.  Labels: 0 displacement,
 * 1 saturation, 2 pressure. */
typedef struct {
  int32_t nx, ny, nz;          /* cells per axis, >= 1                                  */
  int32_t reserved;            /* 0                                                      */
  double nu;                   /* Poisson ratio (Young's modulus is per cell)           */
  double phi0;                 /* reference porosity                                     */
  double biot;                 /* Biot coefficient b                                     */
  double grav;                 /* gravity (m/s^2), pointing along -z                     */
  double p_ref;                /* reference pressure of the densities (Pa)              */
  double rho_solid;            /* grain density (kg/m^3)                                 */
  double rho0[2];              /* wetting, non-wetting reference densities               */
  double comp[2];              /* their compressibilities c_l (1/Pa)                     */
  double visc[2];              /* their viscosities (Pa s)                               */
  double dt;                   /* time step (s)                                          */
} mgr_poro_params;

typedef struct mgr_poro mgr_poro;

/* Defaults: nu 0.25, phi0 0.2, b 1, g 9.81, p_ref 1e7, rho_s 2650, water 1000 kg/m^3,
 * 4.5e-10 1/Pa, 1e-3 Pa s; oil 800, 1e-9, 5e-3; dt one day.  [host] */
void mgr_poro_default_params(mgr_poro_params *p, int32_t nx, int32_t ny, int32_t nz);

/* Build the model: copies the cell arrays (device or host pointers, ncell entries each;
 * fixed: 3 * nnode bytes, nonzero = fixed displacement dof), builds the Jacobian pattern
 * (owned; sorted columns) and the constant displacement-displacement block.  well_index and
 * well_pbhp are given together or both NULL (no producers); inj_w / inj_nw (kg/s per
 * cell) may be NULL.  Synchronises `stream`.  Errors: ARG (null arrays, parameters out of
 * range, a non-positive Young's modulus), UNSUPPORTED (a grid whose Jacobian needs int64
 * column indices), ALLOC, HIP. */
mgr_status mgr_poro_create(const mgr_poro_params *prm, const double *perm, const double *young,
                           const uint8_t *fixed, const double *well_index,
                           const double *well_pbhp, const double *inj_w, const double *inj_nw,
                           void *stream, mgr_poro **out);

/* Change the time step of later assemblies.  Errors: ARG. [host] */
mgr_status mgr_poro_set_dt(mgr_poro *P, double dt);

/* Describe the owned Jacobian (values as of the last assembly) and its labels; the
 * pointers stay valid until mgr_poro_destroy.  [host] */
mgr_status mgr_poro_matrix(const mgr_poro *P, mgr_csr *A, const int8_t **labels);

/* sizes[0] = n (unknowns), sizes[1] = Jacobian entries, sizes[2] = displacement dofs,
 * sizes[3] = cells.  [host] */
mgr_status mgr_poro_sizes(const mgr_poro *P, int64_t sizes[4]);

/* Copy the Jacobian (n + 1 row pointers, entries' columns and values as of the last
 * assembly) and the n labels into caller arrays (device or host; any may be NULL).
 * Synchronises `stream`.  Errors: ARG, HIP. */
mgr_status mgr_poro_export(const mgr_poro *P, int64_t *row_ptr, int32_t *col, double *val,
                           int8_t *labels, void *stream);

/* F = F(x) for the step from x_old to x (n entries each, n = 3 nnode + 2 ncell), and with
 * with_jacobian != 0 the Jacobian values at x into the owned matrix.  norms [host, 6] may
 * be NULL; otherwise it receives, per row type (momentum, wetting, non-wetting), the sum of
 * squares and the largest magnitude of the residual in state units (momentum rows / the
 * largest Young's modulus; mass rows of phase l * dt / (phi0 rho0_l)), and the call
 * synchronises `stream`.  Errors: ARG, HIP. */
mgr_status mgr_poro_assemble(mgr_poro *P, const double *x, const double *x_old, double *F,
                             int32_t with_jacobian, double *norms, void *stream);

#define MGR_NEWTON_MAX_RECORD 32

typedef struct {
  int32_t max_newton;          /* Newton iterations per time step, 0..32 (default 12)   */
  int32_t max_backtracks;      /* halvings of the step per iteration (default 6)        */
  double tol_flow;             /* converged when every mass residual in state units is  */
  double tol_mech;             /*   <= tol_flow and every momentum one <= tol_mech      */
                               /*   (defaults 1e-6 and 1e-10)                           */
  double max_ds;               /* cap on |lambda ds| of any saturation (default 0.2)   */
  double armijo;               /* sufficient decrease factor (default 1e-4)            */
} mgr_newton_opts;

typedef struct {
  int32_t newton_iters;        /* linear solves done                                    */
  int32_t linear_iters;        /* FGMRES iterations over all of them                    */
  int32_t backtracks;          /* step halvings                                         */
  int32_t converged;           /* 1 if the test above held at the end                   */
  int32_t setups;              /* full MGR setups (1 when *h was NULL on entry)         */
  int32_t linear_failures;     /* solves that reached maxit (their iterate is used)     */
  int32_t lin_iters[MGR_NEWTON_MAX_RECORD];
  double merit[MGR_NEWTON_MAX_RECORD + 1];   /* ||residual in state units||_2 before
                                                every solve and at the end              */
  double lambda[MGR_NEWTON_MAX_RECORD];
  double assemble_ms, setup_ms, solve_ms;    /* host wall time of the phases           */
} mgr_newton_stats;

/* [host] */
void mgr_newton_default_opts(mgr_newton_opts *o);

/* One time step by Newton's method with backtracking (Sec. 4, eq. newton): at x^(k)
 * assemble F and A, scale both to state units row by row (D: momentum rows / the largest
 * Young's modulus, mass rows of phase l * dt / (phi0 rho0_l); MGR is invariant to it, the
 * FGMRES residual norm is not: unscaled, the momentum rows in newtons swamp the mass rows
 * in kg/s), solve (D A) d = D F by fgmres_solve preconditioned with MGR, take
 * x^(k+1) = x^(k) - lambda d where lambda starts at 1, is cut so no saturation moves by
 * more than max_ds, and is halved while the merit (the 2-norm of the residual in state
 * units) fails to fall by the factor (1 - armijo lambda); the last halving is accepted.
 * The MGR hierarchy is *h: built with mgr_setup(opts = mo) when *h is NULL, else rebuilt
 * with mgr_setup_numeric (the pattern never changes); the caller owns and destroys it.
 *   x      n entries: the initial guess in (usually x_old), the new time level out.
 *   x_old  the previous time level.
 * Synchronises `stream`.  A linear solve that reaches maxit is counted and its iterate
 * used.  Errors: ARG, ZERO_PIVOT and the other errors of mgr_setup / fgmres_solve, ALLOC,
 * HIP; Newton's own non-convergence is reported in st->converged, not as an error.
 * The row-scaled copy D A lives in a second value array of P; the owned matrix of
 * mgr_poro_matrix keeps the unscaled Jacobian of the last assembly. */
mgr_status mgr_poro_newton(mgr_poro *P, mgr_handle **h, const mgr_opts *mo,
                           const fgmres_opts *fo, double *x, const double *x_old,
                           const mgr_newton_opts *no, mgr_newton_stats *st, void *stream);

void mgr_poro_destroy(mgr_poro *P);

#ifdef __cplusplus
}
#endif
#endif /* MGR355_H */
