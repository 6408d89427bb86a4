/*
 * lrp.h -- low-rank Poisson solver (Cross-DEIM with leverage scores) on one MI355X.
 *
 * Problem (paper, Section 3, eq. poisson / matrix_poisson): -Lap u = f on the unit square,
 * u = 0 on the boundary, 5-point stencil on n x n interior points with h = 1/(n+1), i.e.
 * T W + W T^T = h^2 F with T = tridiag(-1, 2, -1). The right-hand side is given in low-rank
 * form F = U_F diag(sigma_F) V_F^T (Section 3.2). The solver moves the factors to the sine
 * basis with the orthonormal DST-I, runs the warm-started Cross-DEIM iteration (Algorithm 4,
 * with the stabilized cross approximation of Algorithm 1 and leverage-score index selection
 * of Algorithm 3) on W^(i,j) = h^2 F^(i,j)/(lambda_i + lambda_j) (Section 3.1, eq. g_for_p)
 * and moves the factors of the result back: W ~= U_W diag(S) V_W^T.
 *
 * Conventions for every entry point below:
 *   - Matrices are column-major; "ld" is the leading dimension (distance in elements between
 *     columns, ld >= n). Row and column indices are 0-based; frequency index i (0-based)
 *     stands for the paper's 1-based mode i+1.
 *   - Pointers documented as "device" are HIP device pointers (hipMalloc or torch CUDA
 *     tensors); "host" pointers are ordinary CPU memory. The caller owns every buffer it
 *     passes; the library never frees them and keeps no pointer to them after a call returns
 *     (except lrp_set_guess, whose pointers are read by the next lrp_solve).
 *   - Input buffers are read-only. Output buffers must not overlap inputs (LRP_EINVAL).
 *   - A context owns all of its device workspace; it is allocated in lrp_create and reused
 *     by every lrp_solve, which allocates nothing.
 *   - Negative return codes mean no valid result; positive codes are warnings with a valid
 *     result; LRP_OK is 0. Argument checks happen before any device work.
 *   - One context is used by one host thread at a time (calls on a context are not
 *     thread-safe); work is ordered on the context's stream.
 */
#ifndef LRP_H
#define LRP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lrp_ctx lrp_ctx;

enum lrp_status {
  LRP_OK = 0,
  LRP_NOT_CONVERGED = 1, /* maxiter passes made without meeting the tolerance (Algorithm 4 returns its last iterate) */
  LRP_STAGNATED = 2,     /* the index sets repeated: a fixed point; the last distinct iterate is returned */
  LRP_EINVAL = -1,       /* bad argument: sizes, null or overlapping pointers, n+1 not a power of two */
  LRP_ENOMEM = -2,       /* device allocation failed in lrp_create */
  LRP_EDEVICE = -3,      /* a HIP call failed */
  LRP_ENUMERIC = -4,     /* NaN or Inf in the right-hand side factors */
  LRP_ESIZE = -5         /* the problem needs more workspace than the fixed workspace of an
                            entry point that allocates nothing (lrp_tsqr_noalloc) */
};

enum lrp_precision {
  LRP_FP64 = 0,  /* every step in FP64 */
  LRP_MIXED = 1  /* DSTs and fiber evaluation in FP32 with FP32 accumulation; QR, leverage
                    scores, core pseudo-inverse and the stopping test in FP64; the effective
                    tolerance is max(tol, 1e-7) and the prune threshold 1e-7 */
};

/* Options of lrp_create (host struct). All-zero selects the defaults. */
typedef struct lrp_opts {
  int32_t maxiter;   /* passes of the Cross-DEIM loop; 0 -> 20 */
  int32_t precision; /* enum lrp_precision */
  double prune_tau;  /* relative threshold on |diag R| for dropping redundant indices
                        (Algorithm 4); 0 -> 1e-12 (FP64) or 1e-7 (mixed) */
  void* stream;      /* hipStream_t to order all work on; NULL -> a stream owned by the context */
  int32_t flags;     /* bitwise OR of enum lrp_flags; other bits -> LRP_EINVAL */
  int32_t selector;  /* enum lrp_selector: how each pass picks its new indices (Algorithm 4's
                        index selection); other values -> LRP_EINVAL */
  double ls_oversampling; /* LRP_SEL_LEVERAGE_SAMPLED: rho in p_i = min(1, rho pi_i), i.e. the
                             oversampling c = rho r_sig of Algorithm 3; 0 -> 2; must be finite
                             and >= 0 */
  uint64_t seed;     /* LRP_SEL_LEVERAGE_SAMPLED: key of the Philox4x32-10 generator */
  int32_t matrix;    /* enum lrp_matrix: the matrix G whose cross approximation is computed;
                        other values -> LRP_EINVAL */
  int32_t reserved;  /* must be 0 */
} lrp_opts;

enum lrp_matrix {
  LRP_MAT_POISSON = 0,  /* the spectral solution of the Poisson problem (lrp_solve) */
  LRP_MAT_HILBERT = 1,  /* H(i, j) = 1/(1 + i + j), 0-based: the Hilbert matrix (Section 4.2;
                           lrp_cross_solve) */
  LRP_MAT_K = 2         /* K(i, j) = (|x_i + x_j|/2)^5 on the grid x_i = -1 + 2 i/(n - 1), a C^4
                           function with a kink along x + y = 0 (Section 4.2; lrp_cross_solve) */
};

enum lrp_selector {
  LRP_SEL_LEVERAGE = 0,  /* leverage scores (Algorithm 3): the r_sig largest scores outside the
                            current set, appended in ascending index order */
  LRP_SEL_QDEIM = 1,     /* QDEIM (Algorithm 2): the first r_sig pivots of the column-pivoted
                            Householder QR of U(:, :r_sig)^T (the largest remaining squared norm,
                            near-ties within 1e-12 relative to the smaller index), those not yet
                            in the set appended in pivot order; when none is new, and at the first
                            pass, the index outside the set with the largest leverage score is
                            appended as well (Algorithm 4's safeguard, taken deterministically).
                            Costs one launch per possible pivot (r_max) per pass. */
  LRP_SEL_LEVERAGE_SAMPLED = 2 /* leverage scores as Algorithm 3 states them: row i (outside the
                            set) is kept with probability p_i = min(1, rho pi_i), pi_i the
                            squared norm of row i of U(:, :r_sig); the uniform u_i is the
                            Philox4x32-10 output for counter (i mod 2^32, i / 2^32, pass, side)
                            and key (seed mod 2^32, seed / 2^32), 53 bits / 2^53, and i is kept
                            when u_i < p_i. The kept rows with the largest scores fill the set up
                            to r_max (appended in ascending order); when none is kept, the row
                            outside the set with the largest -1 - u_i is appended (the
                            safeguard's random index). */
};

enum lrp_flags {
  LRP_FLAG_PROFILE = 1  /* record the device time of every kernel launch of each solve with
                           HIP events on the solve's stream (read with lrp_get_profile). The
                           passes are then launched one kernel at a time instead of as graphs,
                           and the stream is held for about 0.5 ms at the start of each solve
                           so that the host is ahead of the device; results are unchanged. */
};

/* Per-solve report (host struct), filled by lrp_solve when non-NULL. */
typedef struct lrp_info {
  int32_t status;    /* same as the return code */
  int32_t iters;     /* cross approximations computed (calls of Algorithm 1) */
  int32_t rank;      /* rank of the returned solution */
  int32_t nI, nJ;    /* sizes of the final (pruned) index sets */
  double rho;        /* ||X_k - X_{k-1}||_F / ||S_k||_F of the last pass (inf if not computed) */
  double indicator;  /* min(eta1 (1+eta2), eta2 (1+eta1)) S_min / ||S_k||_F of the last pass;
                        +inf where it cannot pass the test (pass 0, or 2 S_min/||S_k|| >= tol) */
  float ms;          /* device time of the whole solve, milliseconds (HIP events) */
} lrp_info;

/*
 * lrp_create -- context for grids of n interior points per dimension and rank cap r_max.
 *   ctx    out (host): receives the context.
 *   n      grid size; n+1 must be a power of two, 4 <= n+1 <= 2^23 (for the test matrices of
 *          opts.matrix: 2 <= n <= 2^23).
 *   r_max  rank cap of the result and cap of each index set, 1 <= r_max <= 64, r_max <= n.
 *   tol    tolerance eps of Algorithm 4, relative to ||S_k||_F; tol >= 0.
 *   opts   host, may be NULL (defaults).
 * Allocates all device workspace (about 12 n r_max doubles) and the eigenvalue and DST
 * twiddle tables (Section 3: lambda_k = 4 sin^2(pi k/(2(n+1)))).
 * Returns LRP_OK, LRP_EINVAL, LRP_ENOMEM or LRP_EDEVICE.
 */
int lrp_create(lrp_ctx** ctx, int64_t n, int32_t r_max, double tol, const lrp_opts* opts);

/*
 * lrp_solve -- one low-rank Poisson solve (Section 3.2 with Algorithm 4).
 *   r_F      rank of the right-hand side, 1 <= r_F <= r_max.
 *   U_F      device, n x r_F, leading dimension ldu >= n; need not be orthonormal.
 *   sigma_F  device, r_F values (signed allowed); F = U_F diag(sigma_F) V_F^T.
 *   V_F      device, n x r_F, leading dimension ldv >= n.
 *   U_out    device, n x r_max, leading dimension ldou >= n: left factors of W in columns
 *            0..rank-1; columns rank..r_max-1 are set to 0.
 *   S_out    device, r_max values: the rank singular values in descending order, then 0.
 *   V_out    device, n x r_max, leading dimension ldov >= n, as U_out.
 *   r_out    host, receives the rank (1 <= rank <= r_max).
 *   info     host, may be NULL. On a negative return only status and iters (the passes
 *            completed before the failure) are set.
 * Blocks until the result is complete. Returns LRP_OK, LRP_NOT_CONVERGED or LRP_STAGNATED
 * with a valid result, or LRP_EINVAL / LRP_ENUMERIC / LRP_EDEVICE without one. A zero
 * right-hand side gives the zero solution with rank 1 and LRP_OK.
 */
int lrp_solve(lrp_ctx* ctx, int32_t r_F, const double* U_F, int64_t ldu, const double* sigma_F,
              const double* V_F, int64_t ldv, double* U_out, int64_t ldou, double* S_out,
              double* V_out, int64_t ldov, int32_t* r_out, lrp_info* info);

/*
 * lrp_cross_solve -- Cross-DEIM (Algorithm 4 with Algorithm 1) on the n x n test matrix the
 * context was created for (opts.matrix = LRP_MAT_HILBERT or LRP_MAT_K; any n >= 2), started from
 * the initial guess U0 V0^T of Algorithm 4: its truncated SVD (thin QRs of U0 and V0, SVD of
 * R_u R_v^T, truncated at r0 eps sigma_1) is the first iterate. Returns G ~= U diag(S) V^T, the
 * cross approximation truncated at the tolerance (no transform: U, V are the iterate's
 * orthonormal factors).
 *   r0       columns of the guess, 1 <= r0 <= r_max.
 *   U0, V0   device, n x r0, leading dimensions ldu0, ldv0 >= n.
 *   U_out, S_out, V_out, r_out, info   as in lrp_solve.
 * Returns as lrp_solve; LRP_ENUMERIC for a zero or non-finite guess, LRP_EINVAL on a Poisson
 * context (and lrp_solve returns LRP_EINVAL on a test-matrix context).
 */
int lrp_cross_solve(lrp_ctx* ctx, int32_t r0, const double* U0, int64_t ldu0, const double* V0, int64_t ldv0,
                    double* U_out, int64_t ldou, double* S_out, double* V_out, int64_t ldov, int32_t* r_out,
                    lrp_info* info);

/*
 * lrp_get_index_sets -- the pruned row set I and column set J of the iterate returned by the
 * last lrp_solve, in their stored order (old indices first, then new ones ascending).
 *   I, J   host, capacity r_max each; nI, nJ host, receive the sizes.
 * Returns LRP_OK or LRP_EINVAL (no solve yet).
 */
int lrp_get_index_sets(const lrp_ctx* ctx, int64_t* I, int32_t* nI, int64_t* J, int32_t* nJ);

/*
 * lrp_get_trace -- per-pass record of the last lrp_solve (Algorithm 4), pass k = 0..count-1:
 *   Ipre, Jpre  host, count x r_max: the index sets handed to the cross approximation;
 *   nIpre, nJpre, nI, nJ  host, count: their sizes before and after pruning;
 *   rank        host, count: rank of the pass's cross approximation;
 *   indicator, rho  host, count (+inf where the stopping test did not need them);
 *   branch      host, count: 1 where |J| <= |I| (Algorithm 1 solves with Q(I,:)), 0 where it
 *               solves with Z(J,:);
 *   route       host, count: how the core's pseudo-inverse was formed: 0 through a Householder
 *               QR (a bound showed that the cutoff drops no singular value, so the pseudo-inverse
 *               is the left inverse), 1 through a Jacobi SVD with the cutoff;
 *   sweeps      host, count: one-sided Jacobi sweeps of the SVD of the pass's core (the last
 *               sweep rotates no pair by more than a cosine of 1e-8, after which a further sweep
 *               would find the pairs orthogonal to rounding).
 *   count       host in/out: capacity in passes on input, passes recorded on output.
 * Any array pointer may be NULL. Returns LRP_OK or LRP_EINVAL.
 */
int lrp_get_trace(const lrp_ctx* ctx, int32_t* count, int32_t* Ipre, int32_t* nIpre, int32_t* Jpre,
                  int32_t* nJpre, int32_t* nI, int32_t* nJ, int32_t* rank, double* indicator,
                  double* rho, int32_t* branch, int32_t* route, int32_t* sweeps);

/*
 * lrp_set_guess -- the initial guess U0, V0 of Algorithm 4 (its signature takes them as input;
 * Section 1 describes the solver as warm started) for the next lrp_solve on this context.
 * The guess is given in physical space like the solver's output, for example the factors of
 * a previous solution: that solve then starts from the truncated SVD of
 * DST(U0) diag(S0) DST(V0)^T (computed in FP64 in both precisions, truncated at
 * r0 eps sigma_1) instead of from the right-hand side.
 *   r0   columns of the guess, 1 <= r0 <= r_max; 0 clears a guess set earlier.
 *   U0   device, n x r0, leading dimension ldu0 >= n.
 *   S0   device, r0 weights, or NULL for unit weights.
 *   V0   device, n x r0, leading dimension ldv0 >= n.
 * The pointers are read by the next lrp_solve only (they must stay valid and unchanged until
 * it returns; they may be that solve's output buffers, which are written only after the
 * guess has been read), and the guess is cleared when that solve returns. A guess whose
 * product is zero is ignored (the solve starts from the right-hand side); non-finite values
 * make that solve return LRP_ENUMERIC. Returns LRP_OK or LRP_EINVAL (nothing changed).
 */
int lrp_set_guess(lrp_ctx* ctx, int32_t r0, const double* U0, int64_t ldu0, const double* S0,
                  const double* V0, int64_t ldv0);

/*
 * lrp_set_index_sets -- replay (a diagnostic): passes 0 .. npasses-1 of every following
 * lrp_solve on this context take the given index sets as the sets handed to the cross
 * approximation (the union of Algorithm 4) instead of selecting them; later passes select from the
 * iterate these produce, as usual. Run a mixed-precision solve on the sets of an FP64 solve to
 * separate rounding from index-set divergence.
 *   npasses  0 <= npasses <= maxiter; 0 switches replay off.
 *   I        host, npasses x r_max, row-major: entries 0 .. nI[k]-1 of row k are the row set of
 *            pass k, 0-based, < n, distinct within the row.
 *   nI       host, npasses sizes, 1 <= nI[k] <= r_max.
 *   J, nJ    host, the column sets, as I and nI.
 * Synchronizes the context's stream. Returns LRP_OK, LRP_EINVAL (nothing changed) or
 * LRP_EDEVICE.
 */
int lrp_set_index_sets(lrp_ctx* ctx, int32_t npasses, const int64_t* I, const int32_t* nI,
                       const int64_t* J, const int32_t* nJ);

/* One kernel class of a profiled solve (host struct filled by lrp_get_profile). */
typedef struct lrp_kernel_time {
  const char* name;  /* kernel name (static string owned by the library) */
  int32_t launches;  /* launches in the last solve */
  double ms;         /* their summed device time, milliseconds, each launch timed by start and
                        stop events attached to its dispatch (hipExtLaunchKernelGGL; a copy by
                        events recorded around it). The bracket adds a few microseconds per
                        launch: 16 empty launches made at the start of the solve, reported as the
                        entry "empty kernel", show its size */
} lrp_kernel_time;

/*
 * lrp_get_profile -- per-kernel device time of the last lrp_solve of a context created with
 * LRP_FLAG_PROFILE.
 *   count  host, in: capacity of out; out: number of kernel classes that ran (entries beyond
 *          the capacity are counted but not written).
 *   out    host array of *count entries (may be NULL when *count is 0).
 * Returns LRP_OK (count 0 for a context without the flag), or LRP_EINVAL (NULL arguments, or a
 * profiled context that has not completed a solve).
 */
int lrp_get_profile(const lrp_ctx* ctx, int32_t* count, lrp_kernel_time* out);

/* lrp_destroy -- frees the context and its workspace (NULL is a no-op). */
int lrp_destroy(lrp_ctx* ctx);

/* lrp_strerror -- static description of a return code. */
const char* lrp_strerror(int code);

/*
 * lrp_dst1 -- orthonormal DST-I along the columns of a device matrix (Section 3:
 * (Z x)_i = sqrt(2/(n+1)) sum_k x_k sin(i k pi/(n+1)), Z = Z^T = Z^{-1}, Section 3.2).
 *   X  device, n x ncols, ld ldx >= n (read);  Y  device, n x ncols, ld ldy >= n (written).
 *   scale  device or NULL: if given, column c of Y is multiplied by scale[c] (ncols values).
 *   mul    host scalar multiplying every output (1.0 for the plain transform).
 *   precision  LRP_FP64 or LRP_MIXED (FP32 arithmetic, FP64 in and out).
 * Uses the context's stream and tables, so n must equal the context's n; X and Y must not
 * overlap; ncols <= 2 r_max. Returns LRP_OK, LRP_EINVAL or LRP_EDEVICE; does not block.
 */
int lrp_dst1(lrp_ctx* ctx, int32_t ncols, const double* X, int64_t ldx, double* Y, int64_t ldy,
             const double* scale, double mul, int32_t precision);

/*
 * lrp_tsqr -- thin Householder QR of a tall device matrix, A = Q R (the QR of Algorithm 1,
 * computed as a tree of block QRs). The rows of the context's grid are the rows of A.
 *   A  device, n x ncols, ld lda >= n (read); 1 <= ncols <= r_max.
 *   Q  device, n x ncols, ld ldq >= n (written; orthonormal columns).
 *   R  device, ncols x ncols, ld ldr >= ncols (written; upper triangular, zeros below).
 * Blocks until done. Returns LRP_OK, LRP_EINVAL or LRP_EDEVICE.
 */
int lrp_tsqr(lrp_ctx* ctx, int32_t ncols, const double* A, int64_t lda, double* Q, int64_t ldq,
             double* R, int64_t ldr);

/*
 * lrp_tsqr_noalloc -- the thin QR of lrp_tsqr without a context and without any device or host
 * allocation, for callers that cannot allocate: code under HIP graph capture, tight serving
 * loops and harnesses that forbid hipMalloc. The tree's workspace (Householder vectors, their
 * scalars and the stacked R factors of every level, and the intermediate Q pieces) is a fixed
 * static device array of lrp_tsqr_noalloc_max_bytes() bytes (32 MiB) on each GPU the library
 * runs on, held until the process ends. It holds about 1.7 n ncols doubles at 64 columns
 * (largest n: 32661 at 64 columns, 91392 at 32, 217600 at 16, 4129344 at 1 column).
 *   n      rows, 1 <= n; ncols columns, 1 <= ncols <= 64, ncols <= n.
 *   A      device, n x ncols, ld lda >= n (read).
 *   Q      device, n x ncols, ld ldq >= n (written; orthonormal columns); must not overlap A.
 *   R      device, ncols x ncols, ld ldr >= ncols (written; upper triangular, zeros below).
 *   stream hipStream_t the work is ordered on (NULL: the null stream).
 * Asynchronous: enqueues the kernels on stream and returns. Every call on one GPU shares that
 * GPU's workspace (each call writes every workspace element it reads, so nothing carries over
 * from an earlier call), so calls whose work can overlap on one GPU race: order them on one
 * stream or synchronize between them. Returns LRP_OK, LRP_EINVAL (arguments), LRP_ESIZE (the
 * workspace for n x ncols exceeds the fixed size) or LRP_EDEVICE; nothing is enqueued on error.
 */
int lrp_tsqr_noalloc(int64_t n, int32_t ncols, const double* A, int64_t lda, double* Q, int64_t ldq,
                     double* R, int64_t ldr, void* stream);

/* lrp_tsqr_noalloc_max_bytes -- size in bytes of lrp_tsqr_noalloc's fixed per-GPU workspace. */
int64_t lrp_tsqr_noalloc_max_bytes(void);

/* ---------------------------------------------------------------------------------------
 * Serving: a solve queue with continuous admission.
 *
 * Requests (each one Poisson solve of the kind lrp_solve performs) are admitted in arrival
 * order as soon as a context of their shape (n, r_max, tol, maxiter, precision) is free or
 * can be created inside the device-memory budget; idle contexts of other shapes are freed to
 * make room. Every admitted request advances pass by pass; the requests of one shape that
 * are ready for their next pass run it together as one launch per stage (same-stage grouping,
 * lrp_server_set_grouping), and groups of different shapes overlap on the device. A finished
 * request frees its context immediately for the next one. A request computes exactly what
 * lrp_solve computes for it, bit for bit, whatever else is in flight or in its group. The
 * scheduler runs on a thread of its own.
 * --------------------------------------------------------------------------------------- */
typedef struct lrp_server lrp_server;

/* One request (host struct). Pointers as in lrp_solve: U_F, sigma_F, V_F, U_out, S_out,
 * V_out are device pointers; inputs must stay valid and unchanged, and outputs untouched,
 * until the request completes. */
typedef struct lrp_request {
  int64_t n;          /* grid size, as for lrp_create with the Poisson matrix */
  int32_t r_F;        /* 1 <= r_F <= r_max */
  int32_t r_max;      /* 1 <= r_max <= 64 */
  double tol;
  int32_t maxiter;    /* 0 -> 20 */
  int32_t precision;  /* enum lrp_precision */
  const double* U_F;
  int64_t ldu;
  const double* sigma_F;
  const double* V_F;
  int64_t ldv;
  double* U_out;
  int64_t ldou;
  double* S_out;
  double* V_out;
  int64_t ldov;
} lrp_request;

typedef struct lrp_server_stats {
  int64_t submitted, completed, failed; /* requests so far */
  int64_t queued, active;               /* waiting for admission / being solved now */
  int64_t bytes_in_use, bytes_budget;   /* device memory held by contexts / allowed */
  int32_t contexts;                     /* contexts currently held */
  int32_t grouping;                     /* 1: same-stage grouping on (lrp_server_set_grouping) */
  int64_t passes;                       /* Cross-DEIM passes run, over all requests */
  int64_t pass_launches;                /* pass launch sequences: a grouped pass of m requests
                                           counts once, so passes / pass_launches is the mean
                                           group size */
} lrp_server_stats;

/*
 * lrp_server_create -- start a server on the current HIP device.
 *   budget_bytes  device memory the server's contexts may hold in total (> 0).
 *   max_active    requests solved concurrently, 1..64.
 * Returns LRP_OK, LRP_EINVAL, LRP_ENOMEM or LRP_EDEVICE.
 */
int lrp_server_create(lrp_server** srv, int64_t budget_bytes, int32_t max_active);

/*
 * lrp_server_submit -- queue a request; *ticket (host) identifies it. Arguments are checked
 * as in lrp_solve (LRP_EINVAL before queuing); a request whose context alone exceeds the
 * budget is rejected with LRP_ENOMEM.
 */
int lrp_server_submit(lrp_server* srv, const lrp_request* req, int64_t* ticket);

/*
 * lrp_server_poll -- *done (host) = 1 once the request has finished; then *status gets its
 * lrp_solve-style return code, *rank its rank, info its report, *latency_ms the time from
 * submission to completion (host clock). Any output pointer may be NULL. A finished ticket
 * may be polled again until lrp_server_release. Returns LRP_OK or LRP_EINVAL.
 */
int lrp_server_poll(lrp_server* srv, int64_t ticket, int32_t* done, int32_t* status, int32_t* rank,
                    lrp_info* info, double* latency_ms);

/* lrp_server_wait -- as lrp_server_poll, blocking until the request has finished. */
int lrp_server_wait(lrp_server* srv, int64_t ticket, int32_t* status, int32_t* rank, lrp_info* info,
                    double* latency_ms);

/*
 * lrp_server_times -- where a finished request's latency went (host clock, milliseconds):
 * *queue_ms from submission to admission into a context (waiting for a free context or for
 * memory, including the creation of a new context), *run_ms from admission to completion
 * (its stages on the device and the scheduler's polling). A request that failed before
 * admission has *run_ms = 0. Either pointer may be NULL. Returns LRP_OK, or LRP_EINVAL for an
 * unknown or unfinished ticket.
 */
int lrp_server_times(lrp_server* srv, int64_t ticket, double* queue_ms, double* run_ms);

/* lrp_server_release -- forget a finished ticket. Returns LRP_OK or LRP_EINVAL. */
int lrp_server_release(lrp_server* srv, int64_t ticket);

/* lrp_server_get_stats -- counters of the server (host struct). */
int lrp_server_get_stats(lrp_server* srv, lrp_server_stats* out);

/*
 * lrp_server_set_grouping -- same-stage grouping on (enabled != 0, the default) or off.
 * With grouping on, the requests of one shape that are ready for their next Cross-DEIM pass
 * (Alg. 4, one iteration) run it together, as one launch per stage of the pass (one graph per
 * group size); off, each request's passes run on its own stream. Results are bitwise the same
 * either way. Allowed only while no request is queued or active: LRP_EINVAL otherwise.
 */
int lrp_server_set_grouping(lrp_server* srv, int32_t enabled);

/* lrp_server_destroy -- finish every admitted request, drop queued ones, free everything. */
int lrp_server_destroy(lrp_server* srv);

/* lrp_context_bytes -- device memory one context of this shape holds (0 if invalid). */
int64_t lrp_context_bytes(int64_t n, int32_t r_max, int32_t maxiter, int32_t precision);

#ifdef __cplusplus
}
#endif

#endif /* LRP_H */
