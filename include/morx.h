/*
 * morx.h -- C ABI of libmorx: shifted sparse solves with a reused SPAI
 * preconditioner on one AMD Instinct MI355X (gfx950).
 *
 * Problem (Singh & Ahuja, "Reusing Preconditioners in Projection based Model
 * Order Reduction Algorithms"; Section III-B lists the sequence
 * A_1 X_1 = F_1, ..., A_l X_l = F_l, appendix B gives the first-order form
 * A_i = sigma_i D - K used here with D -> E, K -> A, F -> B):
 *
 *     (sigma_i E - A) x_ij = b_j,   (sigma_i E - A)^T y_ij = c_j
 *
 * for every shift sigma_i of a shift set and every column j of B and C,
 * solved by right-preconditioned two-sided BiCG (Section III-A).  The
 * preconditioner of the first shift is a sparse approximate inverse (SPAI,
 * eqs. gen-precond / gen-precond-par); every later shift reuses it through a
 * column-wise least-squares update Q_i with min ||A_{i-1} - A_i Q_i||_F and
 * P_i = Q_i P_{i-1} (Table 2, second approach; Section III-C horizontal and
 * vertical directions; Algorithm 4 for the order), applied as a chain of
 * sparse products and never formed.
 *
 * Conventions for every call:
 *  - Matrices are FP64; indices are int32; dense blocks are column-major with
 *    a leading dimension (ld >= n).  Arguments marked (dev) are device
 *    pointers on the context's device, (host) are host pointers.
 *  - The caller owns every buffer it passes and keeps it alive until the call
 *    returns.  Calls that take a stream (a hipStream_t passed as void*, NULL
 *    for the null stream) order their device work after work already queued
 *    on it; every call in this header returns only after its device work is
 *    complete, so outputs are ready on return.
 *  - Every call returns a morx_status; on failure morx_last_error() describes
 *    the first failing check of the calling thread.  Inputs are not modified.
 *  - Calls on one context are not thread-safe unless stated otherwise.
 *  - The factor pattern S is pattern(A) plus the diagonal, shared by every
 *    SPAI and update factor; limits: |column of S| <= 31 entries, the union
 *    of rows touched by one column's pattern <= 512 rows, n < 2^31,
 *    nnz(S) < 2^31.  Larger patterns give MORX_E_UNSUPPORTED.
 */
#ifndef MORX_H
#define MORX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct morx_ctx_s* morx_ctx;        /* library-owned device context            */
typedef struct morx_system_s* morx_system;  /* library-owned resident copy of A, E, S  */
typedef struct morx_factor_s* morx_factor;  /* library-owned SPAI or update factor     */

typedef enum {
  MORX_OK = 0,
  MORX_E_INVALID = -1,       /* bad argument (size, pointer, unsorted CSR, ...)     */
  MORX_E_NOMEM = -2,         /* device or host allocation failed                    */
  MORX_E_HIP = -3,           /* a HIP runtime call failed                           */
  MORX_E_SINGULAR_LS = -4,   /* a local least-squares matrix is rank deficient      */
  MORX_E_NOT_CONVERGED = -5, /* a column missed the tolerance within the limits     */
  MORX_E_BREAKDOWN = -6,     /* BiCG breakdown persisted through every restart      */
  MORX_E_NONFINITE = -7,     /* NaN or Inf in an input                              */
  MORX_E_ADMISSION = -8,     /* serving: request does not fit the memory budget     */
  MORX_E_UNSUPPORTED = -9,   /* pattern beyond the documented limits                */
  MORX_E_PENDING = -10       /* serving: request not finished yet                   */
} morx_status;

typedef enum { MORX_F64 = 0, MORX_F32 = 1, MORX_BF16 = 2 } morx_prec;

typedef enum {
  MORX_CHAIN_RESET = 0,      /* SPAI at sigmas[0], then horizontal updates (round 1)  */
  MORX_CHAIN_NEXT_ROUND = 1, /* vertical update from the previous call's first shift
                                to sigmas[0], then horizontal updates (round z > 1)   */
  /* comparators (no vertical chain is kept; a later NEXT_ROUND call resets):     */
  MORX_CHAIN_DIRECT = 2,     /* a fresh SPAI at every shift, chains of one factor     */
  MORX_CHAIN_FIRST = 3       /* Table 2's first approach: P_i = Q_i P_1, Q_i from
                                min ||A_1 - A_i Q||_F (an update from sigmas[0])      */
} morx_chain_policy;

/* Solver options.  morx_opts_default() fills the defaults given here. */
typedef struct {
  double tol;            /* target true relative residual, primal and dual (1e-10) */
  int32_t maxit;         /* iterations per restart cycle; <= 0 means min(n, 20000)  */
  int32_t max_restarts;  /* true-residual restarts per column (3)                   */
  int32_t precond_prec;  /* morx_prec: storage of factor values (MORX_F64)          */
  int32_t chain;         /* morx_chain_policy (MORX_CHAIN_RESET)                    */
  int32_t want_dual;     /* 1: also solve the transposed systems with C (1)         */
  int32_t batched;       /* 1: all shifts x columns in one multi-column solve;
                            0: one shift and one column at a time (1)              */
  int32_t poll_iters;    /* iterations between host convergence checks (8)          */
  int32_t use_graph;     /* 1: replay the iteration segment as a HIP graph (1)      */
  int32_t apply_prec;    /* morx_prec of the preconditioner apply (MORX_F64):
                            MORX_F32 rounds the input of the chain and the result
                            of every factor pass to FP32 (each pass sums in FP64);
                            the operator, the BiCG recurrences, the residual
                            tests and the refinement stay FP64.  MORX_BF16 is
                            rejected with MORX_E_INVALID.                          */
} morx_opts;

/* Per-column result.  status is a morx_status. */
typedef struct {
  int32_t status;
  int32_t iters;         /* BiCG iterations over all restart cycles                */
  int32_t restarts;
  int32_t reserved;
  double relres_primal;  /* ||b - A_s x|| / ||b||, recomputed in FP64 at the end    */
  double relres_dual;    /* ||c - A_s^T y|| / ||c||                                 */
} morx_col_stats;

void morx_opts_default(morx_opts* opts);
const char* morx_status_str(int32_t status);
/* Message for the calling thread's last failure ("" if none). */
const char* morx_last_error(void);

/* Context on HIP device `device`.  Owns internal streams and graphs. */
morx_status morx_create(morx_ctx* out, int device);
morx_status morx_destroy(morx_ctx ctx);

/*
 * Copy A (CSR: rowptr[n+1], colind[nnz], val[nnz], all (dev); columns sorted
 * strictly increasing within each row) and E = diag(e_diag[n]) (dev) into
 * library-owned device memory, and prepare the pattern S, its transpose and
 * the sliced-ELL layouts used by every kernel (Section III-A: the n column
 * problems of the SPAI all come from S).  Unsorted or out-of-range indices
 * give MORX_E_INVALID; NaN/Inf values give MORX_E_NONFINITE.
 */
morx_status morx_system_create(morx_ctx ctx, int64_t n, int64_t nnz, const int32_t* rowptr,
                               const int32_t* colind, const double* val, const double* e_diag,
                               void* stream, morx_system* out);
morx_status morx_system_destroy(morx_system sys);
/* nnz(S) and the device bytes held by the system (excluding factors). */
morx_status morx_system_info(morx_system sys, int64_t* nnz_pattern, int64_t* resident_bytes);
/* Copy S in CSR form: rowptr[n+1], colind[nnz(S)] (dev, caller-allocated). */
morx_status morx_system_pattern(morx_system sys, int32_t* rowptr, int32_t* colind, void* stream);

/*
 * Y = (sigma E - A) X, or (sigma E - A)^T X when trans != 0, for ncol
 * columns (X, Y (dev), column-major, ldx, ldy >= n).  The shifted matrix is
 * never formed: E's diagonal is applied inside the product (appendix B form).
 * Runs the shifted-pair kernel of a solve (morx_shifted_apply_pair with one
 * side); ncol 1..1024.
 */
morx_status morx_shifted_apply(morx_system sys, double sigma, int32_t trans, int32_t ncol,
                               const double* X, int64_t ldx, double* Y, int64_t ldy,
                               void* stream);

/*
 * SPAI factor of A_s = sigma E - A on the pattern S: column k minimises
 * ||e_k - A_s p_k||_2 over vectors supported on column k of S (eq.
 * gen-precond-par).  Values are computed in FP64 and stored at `prec`.
 */
morx_status morx_factor_spai(morx_system sys, double sigma, int32_t prec, void* stream,
                             morx_factor* out);
/*
 * Reuse factor Q with min ||A_prev - A_new Q||_F on the pattern S, where
 * A_prev = sigma_prev E - A and A_new = sigma_new E - A (Table 2, second
 * approach; Section III-C).  The new preconditioner is Q P_prev.
 */
morx_status morx_factor_update(morx_system sys, double sigma_prev, double sigma_new,
                               int32_t prec, void* stream, morx_factor* out);
/* Stored values widened to FP64, in the CSR order of S (val[nnz(S)], dev). */
morx_status morx_factor_values(morx_factor f, double* val, void* stream);
morx_status morx_factor_destroy(morx_factor f);

/*
 * What a factor is: a SPAI of sigma_new E - A (is_spai = 1, sigma_prev
 * unused and 0), or the update with min ||A_prev - A_new Q||_F between
 * sigma_prev and sigma_new (is_spai = 0; Table 2, second approach).
 */
typedef struct {
  int32_t is_spai;
  int32_t reserved;
  double sigma_prev;
  double sigma_new;
} morx_factor_spec;

/*
 * Build njobs factors (jobs, host) in one launch of the least-squares
 * kernel, as a solve builds the factors of its shifts (Algorithm 4 builds
 * each shift's factor from the shifts alone, so every factor of a call is
 * independent).  out (host, njobs handles) receives the factors; on failure
 * none is returned.  Limits as morx_factor_spai; njobs 1..4096.
 */
morx_status morx_factor_build(morx_system sys, int32_t njobs, const morx_factor_spec* jobs,
                              int32_t prec, void* stream, morx_factor* out);

/*
 * A factor with given values: val (dev, nnz(S) entries in the CSR order of
 * S that morx_system_pattern returns) is rounded to prec (FP64 -> FP32 by
 * round-to-nearest-even, then -> BF16 by round-to-nearest-even on the FP32
 * bits) and stored in both orders, as the least-squares kernels store their
 * results.  The paper computes its preconditioners in a separate program
 * and loads them into the solver (Section IV); this is that hand-over.  The
 * factor's spec reads SPAI at sigma 0.
 */
morx_status morx_factor_import(morx_system sys, const double* val, int32_t prec, void* stream,
                               morx_factor* out);

/*
 * Apply the product F_{k-1} ... F_1 F_0 (chain[0] applied first) to ncol
 * columns, or its transpose F_0^T ... F_{k-1}^T when trans != 0, one sparse
 * product per factor (Section III-B: the product is never formed), in FP64,
 * by the chain kernels of a solve (morx_chain_apply_batch with one chain
 * for every column and one side).  X and Y (dev) may not overlap; ncol
 * 1..1024, nfactor 1..64.
 */
morx_status morx_chain_apply(morx_system sys, int32_t nfactor, const morx_factor* chain,
                             int32_t trans, int32_t ncol, const double* X, int64_t ldx,
                             double* Y, int64_t ldy, void* stream);

/*
 * The chain apply of a solve, outside a solve: column c of X is multiplied
 * by the chain chains[c * lcap + 0 .. lens[c] - 1] (factor 0 applied first),
 * column c of Xt by its transpose (factor lens[c] - 1 transposed first), by
 * the very kernels, work lists, tile widths and row blocks an iteration of
 * morx_solve_shifts launches for ncol column pairs with these chains
 * (Section III-B: one sparse product per factor, the product never formed).
 * apply_prec MORX_F32 rounds the input and every pass result to FP32, as
 * morx_opts.apply_prec does.  X/Y (dev, n x ncol, ldx/ldy >= n) and Xt/Yt
 * (likewise) may each be NULL as a pair: that direction's input is then
 * zero and its output dropped.  Every factor has one storage precision;
 * chains (host) holds ncol * lcap handles, lens (host) ncol lengths in
 * 1..lcap; ncol 1..1024, lcap 1..64.  Outputs do not overlap inputs.
 * Allocates a workspace for ncol columns for the duration of the call.
 */
morx_status morx_chain_apply_batch(morx_system sys, int32_t ncol, int32_t lcap,
                                   const morx_factor* chains, const int32_t* lens,
                                   const double* X, int64_t ldx, double* Y, int64_t ldy,
                                   const double* Xt, int64_t ldxt, double* Yt, int64_t ldyt,
                                   int32_t apply_prec, void* stream);

/*
 * The shifted pair of a solve, outside a solve: Y[:, c] = (sigmas[c] E - A)
 * X[:, c] and Yt[:, c] = (sigmas[c] E - A)^T Xt[:, c] by the kernel and
 * launch shape an iteration of morx_solve_shifts runs for ncol column pairs
 * (E's diagonal applied inside the product; appendix B form).  sigmas
 * (host, ncol finite values); either side may be NULL as a pair (its input
 * is then zero and its output dropped); ncol 1..1024.  Allocates a
 * workspace for ncol columns for the duration of the call.
 */
morx_status morx_shifted_apply_pair(morx_system sys, int32_t ncol, const double* sigmas,
                                    const double* X, int64_t ldx, double* Y, int64_t ldy,
                                    const double* Xt, int64_t ldxt, double* Yt, int64_t ldyt,
                                    void* stream);

/*
 * The hot path.  For the nshift shifts sigmas[] (host, chain order) and the
 * m columns of B (dev, n x m, ldb) and C (dev, n x m, ldc; NULL when
 * opts->want_dual == 0), build the preconditioner chain as Algorithm 4 does
 * (policy opts->chain; the system remembers the vertical chain and the first
 * shift between calls) and solve every pair to opts->tol.  Output X (dev,
 * n x (m*nshift), ldx) holds column j of shift i at column i*m + j; Y
 * likewise (NULL when want_dual == 0).  stats (host) has m*nshift entries in
 * the same order.  Returns the worst column status; other columns' results
 * stay valid.
 */
morx_status morx_solve_shifts(morx_system sys, int32_t nshift, const double* sigmas, int32_t m,
                              const double* B, int64_t ldb, const double* C, int64_t ldc,
                              double* X, int64_t ldx, double* Y, int64_t ldy,
                              const morx_opts* opts, morx_col_stats* stats, void* stream);

/*
 * The preconditioner chains of the last morx_solve_shifts,
 * morx_solve_moments or morx_gmres_shifts call on sys, one per shift in
 * the call's order (Algorithm 4 for MORX_CHAIN_RESET / NEXT_ROUND: the
 * vertical chain P_1^(1), Q_1^(2), ..., Q_1^(z), then Q_2^(z) ... Q_i^(z);
 * the comparator schedules otherwise), each factor described by its spec in
 * application order.  *nshift receives the call's shift count; for shifts
 * i < cap_shifts, lens[i] (host) receives the chain length and
 * specs[i * ldspec + k] (host) factor k, for k < min(lens[i], ldspec).
 * MORX_E_INVALID if no solve has run on the system.
 */
morx_status morx_last_chains(morx_system sys, int32_t cap_shifts, int32_t ldspec, int32_t* nshift,
                             int32_t* lens, morx_factor_spec* specs);

/*
 * Higher moments at the same shifts (the inner loop of AIRGA, Algorithm 1,
 * in first-order form): moment 0 is morx_solve_shifts' solve, and moment
 * j < nmom solves the same systems with E times moment j-1,
 *   X_j(i) = (sigma_i E - A)^{-1} E X_{j-1}(i),
 *   Y_j(i) = (sigma_i E - A)^{-T} E Y_{j-1}(i).
 * The factors and chains (policy opts->chain) are built once and serve every
 * moment; each moment is one batched solve (opts->batched).  X (dev) holds
 * column c of shift i of moment j at column (j * nshift + i) * m + c, Y
 * likewise; stats (host) has nmom * nshift * m entries in that order.  A
 * two-sided projection on all moments matches the transfer function and its
 * derivatives up to order 2 nmom - 1 at every shift.  Allocates two
 * n x (nshift m) blocks for the right-hand sides when nmom > 1.
 */
morx_status morx_solve_moments(morx_system sys, int32_t nshift, const double* sigmas, int32_t m,
                               const double* B, int64_t ldb, const double* C, int64_t ldc,
                               int32_t nmom, double* X, int64_t ldx, double* Y, int64_t ldy,
                               const morx_opts* opts, morx_col_stats* stats, void* stream);

/*
 * One right-hand side per shift (the tangential solves of Algorithm 2, lines 4
 * and 5, in the linear case): for the nshift shifts sigmas[] (host, chain
 * order), column i of B (dev, n x nshift, ldb) and of C (dev, likewise; NULL
 * when opts->want_dual == 0) belong to shift i only, and
 *   (sigma_i E - A) x_i = b_i,   (sigma_i E - A)^T y_i = c_i
 * are solved in one batch with the chains of morx_solve_shifts (policy
 * opts->chain; the factors are built in one launch).  X, Y (dev, n x nshift)
 * and stats (host, nshift entries) are in shift order.  Statuses as
 * morx_solve_shifts.
 */
morx_status morx_solve_pairs(morx_system sys, int32_t nshift, const double* sigmas,
                             const double* B, int64_t ldb, const double* C, int64_t ldc, double* X,
                             int64_t ldx, double* Y, int64_t ldy, const morx_opts* opts,
                             morx_col_stats* stats, void* stream);

/*
 * Second-order systems with proportional damping (Section II's AIRGA model
 * M x'' + D x' + K x = F u, y = C^T x, D = alpha M + beta K; Algorithm 1,
 * lines 4 and 10, with the preconditioner reuse of Section III-C): for the
 * system created from A = -K and E = M (a lumped, i.e. diagonal, mass given
 * as e_diag) and the npoint real expansion points points[] (host, chain
 * order), with A(s) = s^2 M + s D + K,
 *   X_0(i) = A(s_i)^{-1} F,       X_j(i) = -A(s_i)^{-1} M X_{j-1}(i),
 *   Y_0(i) = A(s_i)^{-T} C,       Y_j(i) = -A(s_i)^{-T} M Y_{j-1}(i),
 * for j < nmom (Algorithm 1 normalises each moment before the next solve;
 * these are the unnormalised moments, with the same span).  Each point is
 * solved as the first-order pair at sigma_i = (s_i^2 + alpha s_i) /
 * (1 + beta s_i), since A(s) = (1 + beta s)(sigma E - A), by the batched
 * path of morx_solve_moments, and moment j of point i is then scaled by
 * (-1)^j (1 + beta s_i)^{-(j+1)}.  The SPAI and update factors of A(s_i)
 * are those of sigma_i E - A times scalars, so the iterates, iteration
 * counts and relative residuals (stats) are those of the paper's method on
 * A(s_i).  Layout of F, C, X, Y, stats and the use of opts as in
 * morx_solve_moments (F in place of B; points in place of sigmas; the
 * system remembers sigma of the first point for opts->chain NEXT_ROUND).
 * The Galerkin projection of Section II is morx_project with W = V: it
 * returns Ar = -V^T K V and Er = V^T M V, so K^ = -Ar, M^ = Er and
 * D^ = alpha Er - beta Ar.  MORX_E_NONFINITE for a non-finite alpha, beta
 * or point; MORX_E_INVALID where 1 + beta s_i = 0 or sigma_i overflows;
 * otherwise the statuses of morx_solve_moments.
 */
morx_status morx_solve_second_order(morx_system sys, double alpha, double beta, int32_t npoint,
                                    const double* points, int32_t m, const double* F,
                                    int64_t ldf, const double* C, int64_t ldc, int32_t nmom,
                                    double* X, int64_t ldx, double* Y, int64_t ldy,
                                    const morx_opts* opts, morx_col_stats* stats, void* stream);

/*
 * Restarted GMRES(m), right-preconditioned (the solver of the paper's
 * experiments, Section IV; a comparator of morx_solve_shifts' BiCG on the
 * same factor chains, policy opts->chain).  Every system, the primal one with
 * P and the transposed one with P^T, is solved by its own GMRES, one system
 * at a time: Arnoldi on A_s P with classical Gram-Schmidt applied twice (on
 * the device), the (m+1) x m Hessenberg matrix, Givens rotations and the
 * triangular solve on the host (one synchronisation per Arnoldi step).  A
 * cycle ends when the residual estimate passes opts->tol or after `restart`
 * steps (1..64); the true residual is then recomputed, and the system
 * restarts (a refinement restart, when the estimate had passed, counts
 * against opts->max_restarts).  Layout of X, Y, stats as in
 * morx_solve_shifts; stats.iters and stats.restarts add up both systems.
 * opts->batched, use_graph, poll_iters and apply_prec are ignored.
 */
morx_status morx_gmres_shifts(morx_system sys, int32_t nshift, const double* sigmas, int32_t m,
                              const double* B, int64_t ldb, const double* C, int64_t ldc,
                              int32_t restart, double* X, int64_t ldx, double* Y, int64_t ldy,
                              const morx_opts* opts, morx_col_stats* stats, void* stream);

/*
 * Two-sided Petrov-Galerkin projection (Section II, reduced model after
 * Algorithm 2; descriptor form for E != I):
 *   Ar = W^T A V, Er = W^T E V (r x r), Br = W^T B (r x m), Cr = V^T C (r x q)
 * with V, W (dev, n x r, ldv/ldw) orthonormalised first when
 * orthonormalize != 0 (shifted Cholesky-QR, three passes).  Outputs are host
 * column-major arrays.  r <= 64, m, q <= 64.
 */
morx_status morx_project(morx_system sys, int32_t r, const double* V, int64_t ldv,
                         const double* W, int64_t ldw, int32_t m, const double* B, int64_t ldb,
                         int32_t q, const double* C, int64_t ldc, double* Ar, double* Er,
                         double* Br, double* Cr, int32_t orthonormalize, void* stream);

/*
 * morx_project with orthonormalize = 0 (V and W used as given), for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  It calls no hipMalloc
 * or hipFree; its partial sums and results live in a fixed device scratch of
 * 8.1 MiB that every GPU the library runs on holds from morx_create until the
 * process ends (up to 256 row slabs of 64 x 64 partials, then the four
 * results).  Work is queued on `stream` and the call returns once the host
 * outputs are written.  Limits as morx_project (r <= 64, m, q <= 64;
 * MORX_E_INVALID beyond them).  Calls that overlap on one GPU (other
 * threads, other contexts on the device) share the scratch and race: one
 * call at a time per GPU.  Results equal morx_project's with
 * orthonormalize = 0.
 */
morx_status morx_project_noalloc(morx_system sys, int32_t r, const double* V, int64_t ldv,
                                 const double* W, int64_t ldw, int32_t m, const double* B,
                                 int64_t ldb, int32_t q, const double* C, int64_t ldc,
                                 double* Ar, double* Er, double* Br, double* Cr, void* stream);

/*
 * Eigenvalues of the pencil (Ar, Er) (host, column-major r x r, r <= 64):
 * Er^{-1} Ar by LU with partial pivoting, Householder reduction to upper
 * Hessenberg form and double-shift QR steps.  wr, wi (host, r entries)
 * receive real and imaginary parts, ascending by real part.  MORX_E_INVALID
 * if Er is singular, MORX_E_NOT_CONVERGED if the QR steps do not deflate.
 */
morx_status morx_pencil_eigvals(int32_t r, const double* Ar, const double* Er, double* wr,
                                double* wi);

/*
 * IRKA-style outer loop with computed shifts (Algorithm 2 without its
 * bilinear terms), SISO: b, c (dev) are n-vectors.  Round z solves the r
 * shifted pairs at the current shifts (morx_solve_shifts with m = 1; round 1
 * under opts->chain, RESET or NEXT_ROUND, later rounds under NEXT_ROUND, so
 * Algorithm 4's vertical link carries the first shift's factor from round to
 * round), projects with orthonormalised bases (morx_project) and takes the
 * eigenvalues lambda_i of (Ar, Er); the next shifts are -lambda_i, ascending.
 * The loop stops when the largest relative change of the shifts is <= tol
 * (MORX_OK), after max_rounds rounds (MORX_E_NOT_CONVERGED), or when the
 * reduced pencil has a complex pole pair (|Im| > 1e-10 max |lambda|) or
 * repeated mirror images (MORX_E_UNSUPPORTED: the solver takes real,
 * distinct shifts).  On return sigmas (host, r; initial shifts on entry,
 * distinct, any order) holds the ascending shifts of the last model
 * projected, Ar, Er (host, r x r column-major), Br, Cr (host, r) that model,
 * poles_re/poles_im (host, r) its poles, *rounds the rounds run, *change the
 * relative change of the poles' mirror images against sigmas, and stats (r
 * entries, may be null) the last round's solves.
 */
morx_status morx_irka(morx_system sys, int32_t r, double* sigmas, const double* b,
                      const double* c, int32_t max_rounds, double tol, const morx_opts* opts,
                      double* Ar, double* Er, double* Br, double* Cr, double* poles_re,
                      double* poles_im, int32_t* rounds, double* change, morx_col_stats* stats,
                      void* stream);

/*
 * The MIMO (tangential) form of the IRKA-style loop: Algorithm 2 (BIRKA)
 * without its bilinear terms for B (dev, n x m, ldb) and C (dev, n x q, ldc).
 * Round z solves, for each shift sigma_i and its directions bdir_i (m) and
 * cdir_i (q), (sigma_i E - A) v_i = B bdir_i and (sigma_i E - A)^T w_i =
 * C cdir_i in one batch (morx_solve_pairs; round 1 under opts->chain, RESET or
 * NEXT_ROUND, later rounds under NEXT_ROUND), projects with the
 * orthonormalised V = [v_i] and W = [w_i] (morx_project), and diagonalises
 * the reduced matrix Er^{-1} Ar = R diag(lambda) R^{-1} (line 3; eigenvalues
 * as morx_pencil_eigvals, eigenvectors by inverse iteration on the host):
 * the next shifts are -lambda_i, the next bdir_i row i of R^{-1} Er^{-1} Br
 * and cdir_i column i of Cr^T R, each scaled to unit length with its largest
 * entry positive (the scaling leaves the subspaces alone), in ascending shift
 * order.  Stopping and errors as morx_irka.  sigmas (host, r), bdir (host,
 * m x r column-major: column i for shift i) and cdir (host, q x r) hold the
 * initial shifts and directions on entry and those of the last model
 * projected on return (nonzero directions; shifts distinct); Ar, Er (host,
 * r x r), Br (host, r x m), Cr (host, r x q) that model, column-major;
 * poles_re/poles_im, rounds, change and stats (r entries, may be null) as
 * morx_irka.  r 1..64, m and q 1..64.
 */
morx_status morx_irka_tangential(morx_system sys, int32_t r, double* sigmas, int32_t m,
                                 const double* B, int64_t ldb, int32_t q, const double* C,
                                 int64_t ldc, double* bdir, double* cdir, int32_t max_rounds,
                                 double tol, const morx_opts* opts, double* Ar, double* Er,
                                 double* Br, double* Cr, double* poles_re, double* poles_im,
                                 int32_t* rounds, double* change, morx_col_stats* stats,
                                 void* stream);

/*
 * Launch shapes of a system's kernels (the batching extension: the tile and
 * row-block shapes of the multi-column iteration kernels and of the
 * least-squares factor kernel); -1 selects the built-in choice.
 *   factor_kernel    0: one wave per column, the local matrix in LDS;
 *                    1: one wave per column, the local matrix in registers
 *                    (8 or 16 column lanes; patterns with |J_k| < 16);
 *                    2: normal equations (|J_k| <= 32): per column the
 *                    m x m matrices (A^T A)(J_k, J_k) and A(J_k, J_k), then
 *                    per shift a Cholesky solve in registers; columns whose
 *                    pivots show poor conditioning are redone by kernel 0
 *                    (the built-in choice when the pattern allows it);
 *                    8 or 16: one block of 32 x 8 or 32 x 16 threads per
 *                    column, the local matrix in registers (|J_k| < 32);
 *   cols_per_wave    chain step: most right-hand-side columns one wave
 *                    carries over its rows, sharing every factor load among
 *                    them (1..16);
 *   slices_per_wave  iteration kernels: 64-row slices per wave (1..64; raised
 *                    to the least value that keeps <= 1024 row blocks);
 *   spmv_cols_per_wave  shifted pair and true residual: the same as
 *                    cols_per_wave for the operator's loads (1..16; -1
 *                    follows cols_per_wave); on the halo layout the shifted
 *                    pair runs as a pass of the chain kernel, a block taking
 *                    this many columns per chunk (A is read once per chunk;
 *                    a chunk's staged vectors share the L2);
 *   chain_kernel     chain step: 0 gathers the input vectors row by row; 1
 *                    copies, per block of 256 rows, the input entries at the
 *                    block's distinct columns into LDS and sums from there (the
 *                    halo layout, built by morx_system_create for rows of at
 *                    most 32 entries whose blocks touch at most 2048 columns,
 *                    1024 for rows of at most 8; MORX_E_UNSUPPORTED when the
 *                    system has none); -1 takes 1 for rows of more than 8
 *                    entries where the layout exists, else 0.  The shifted
 *                    pair follows the same choice.  Both give the same
 *                    results.  morx_system_get_tune
 *                    reports the kernel the next solve launches (0 or 1).
 * morx_system_set_tune checks the values (MORX_E_INVALID) and they apply from
 * the next call on the system.  morx_autotune times the candidates on the
 * system itself: per factor kernel one launch of min(chain_len, 16) SPAI
 * problems at `sigma` (storage prec; fewer on large systems, about 8M column
 * problems per candidate), then a few BiCG iterations of ncols column pairs
 * per iteration
 * shape (HIP events), column c preconditioned by 1 + c * chain_len / ncols
 * distinct factors of one list, as the chains of one round are
 * (chain_len 1..64: the longest chain of the solves to come); chain kernel
 * (both where the system has a halo layout), tile and row block first, then
 * the shifted pair's tile.  It keeps the
 * fastest, fills *out (factor_ms and iter_ms: the chosen build and one
 * iteration) and returns MORX_OK.  Shapes change rounding order only.  It
 * allocates its own scratch on the device.
 */
typedef struct {
  int32_t factor_kernel;
  int32_t cols_per_wave;
  int32_t slices_per_wave;
  int32_t spmv_cols_per_wave;
  int32_t chain_kernel;
  int32_t halo_stride;  /* reported only: distance of the row blocks one block
                           of the halo kernels walks (1: consecutive; the
                           detected plane distance of a lexicographically
                           ordered grid otherwise), at one column            */
  double factor_ms;
  double iter_ms;
} morx_tune;

morx_status morx_system_get_tune(morx_system sys, morx_tune* out);
/*
 * The chain-step kernel instance a solve of ncol column pairs on sys
 * launches now (for every chain step but the last of an iteration, whose
 * instance also forms the rho partial sums), with factors stored at prec and
 * applied at apply_prec, written as its demangled name, e.g.
 * "k_chain_halo<double, double, 12, 0, 32, 2048>" (host buf, cap bytes,
 * NUL-terminated; MORX_E_INVALID if it does not fit).
 */
morx_status morx_chain_kernel_name(morx_system sys, int32_t ncol, int32_t prec,
                                   int32_t apply_prec, char* buf, int32_t cap);
morx_status morx_system_set_tune(morx_system sys, const morx_tune* tune);
morx_status morx_autotune(morx_system sys, double sigma, int32_t ncols, int32_t chain_len,
                          int32_t prec, morx_tune* out, void* stream);

/*
 * Serving (continuous batching).  A server owns one scheduler thread on the
 * context's device.  Requests ask for the primal solve (sigma E - A) x = b on
 * a resident system; they are admitted while their device memory fits the
 * budget, run in column slots of a per-system batch (one stream per system),
 * and slots are refilled between iteration segments, so requests that
 * arrive while others run join the work already on the device.  Each system
 * keeps a chain of `anchors` factors (SPAI at the first anchor, column-wise
 * updates between consecutive anchors, log-spaced over [anchor_min,
 * anchor_max]); a request adds one update from its nearest anchor
 * (Section III-B, Table 2 second approach; the nearest anchor in log(sigma),
 * the first on ties).  A system is made resident (slot batch and anchors)
 * on its first admitted request; when a request's system or factor does not
 * fit the budget, idle resident systems (no request in a slot) are released,
 * least recently used first, and a request that cannot fit even then, with
 * nothing left running, finishes with MORX_E_ADMISSION.  Systems must
 * outlive the server; b and x (dev, n entries) stay owned by the caller
 * until the request is finished.  submit, poll, wait, info, counts and
 * chain are thread-safe.
 */
typedef struct morx_server_s* morx_server;

typedef struct {
  size_t hbm_budget_bytes;   /* device memory the server may hold: slot batches,
                                anchor and request factors (16 GiB)                 */
  int32_t slots_per_system;  /* concurrent requests per system, 1..64 (8)           */
  int32_t anchors;           /* anchor shifts per system, 1..31 (8)                 */
  double anchor_min;         /* anchors log-spaced over [anchor_min, anchor_max]    */
  double anchor_max;         /* (1, 1e3)                                            */
  int32_t segment_iters;     /* iterations between admissions (8)                   */
  int32_t reserved;
} morx_serve_config;

void morx_serve_config_default(morx_serve_config* cfg);
/* opts: tol, maxit, max_restarts, precond_prec, use_graph are used. */
morx_status morx_serve_start(morx_ctx ctx, const morx_serve_config* cfg, const morx_opts* opts,
                             morx_server* out);
/* sigma must be finite and > 0.  *ticket identifies the request. */
morx_status morx_serve_submit(morx_server srv, morx_system sys, double sigma, const double* b,
                              double* x, uint64_t* ticket);
/*
 * MORX_E_PENDING while the request runs; otherwise the request's status
 * (MORX_E_ADMISSION if it can never fit the budget), *st and the latency
 * (submit to completion, seconds) are filled and the ticket is released.
 */
morx_status morx_serve_poll(morx_server srv, uint64_t ticket, morx_col_stats* st,
                            double* latency_s);
/* Like poll, but blocks until the request is finished. */
morx_status morx_serve_wait(morx_server srv, uint64_t ticket, morx_col_stats* st,
                            double* latency_s);
morx_status morx_serve_info(morx_server srv, uint64_t* submitted, uint64_t* completed,
                            int32_t* running, int32_t* queued, int64_t* bytes_in_use);

/*
 * Device bytes a server with this configuration and these options counts
 * against its budget for sys: *system_bytes when the system is made
 * resident (its slot batch and anchor factors), *request_bytes per admitted
 * request (its update factor).  cfg and opts may be NULL for the defaults.
 */
morx_status morx_serve_footprint(const morx_serve_config* cfg, const morx_opts* opts,
                                 morx_system sys, size_t* system_bytes, size_t* request_bytes);

/* Scheduler counters since morx_serve_start. */
typedef struct {
  uint64_t admitted;        /* requests given a slot                                  */
  uint64_t joined_running;  /* of those, admitted while another request of the same
                               system was already iterating on the device (the
                               continuous-batching case)                              */
  uint64_t segments;        /* iteration segments launched (one per busy system and
                               scheduler pass)                                        */
  uint64_t systems_made;    /* systems made resident (slot batch and anchors built)   */
  uint64_t systems_evicted; /* idle resident systems released, least recently used
                               first, to admit a request that did not fit             */
  int32_t resident;         /* systems resident now                                   */
  int32_t max_running;      /* most requests running at once                          */
} morx_serve_counts;
morx_status morx_serve_counts_get(morx_server srv, morx_serve_counts* out);

/*
 * The preconditioner chain of an admitted request, in application order:
 * the system's anchor factors up to its nearest anchor (SPAI at the first
 * anchor, then the updates between consecutive anchors) and the request's
 * own update from that anchor to its shift.  MORX_E_PENDING until the
 * request is admitted; valid until the ticket is taken by poll or wait.
 * *len receives the chain length and specs (host) its first min(len, cap)
 * factors.
 */
morx_status morx_serve_chain(morx_server srv, uint64_t ticket, int32_t cap, int32_t* len,
                             morx_factor_spec* specs);
/* Finishes every submitted request, then frees the server (and the slot
   batches and anchor factors it holds). */
morx_status morx_serve_stop(morx_server srv);

/*
 * Kernel tracing (measurement only).  While enabled on a context, solves do
 * not use graphs; every launch of the listed kernel classes is bracketed by
 * HIP events on the library's stream and the algorithmic bytes each launch
 * must move (matrix or factor values and indices once per launch, each
 * vector it reads or writes once) are added up on the device.  Enabling
 * resets the totals.  Classes: "chain_step" (one factor of every
 * preconditioner chain, forward and transposed), "spmv_pair" (shifted
 * operator and its transpose), "form_p" (search directions p = z + beta p
 * of both recurrences), "update" (iterate and residual update),
 * "factor_ls" (least-squares factor construction; no byte count).
 */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;   /* sum of event-bracketed launch durations */
  double alg_bytes;  /* algorithmic bytes over those launches   */
} morx_trace_entry;

morx_status morx_trace_enable(morx_ctx ctx, int32_t enable);
/* Fill up to cap entries (host); *count receives the number of classes. */
morx_status morx_trace_read(morx_ctx ctx, morx_trace_entry* out, int32_t cap, int32_t* count);

#ifdef __cplusplus
}
#endif

#endif /* MORX_H */
