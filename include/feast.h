/*
 * feast.h -- C ABI of the MI355X FEAST hot path.
 *
 * FEAST (E. Polizzi, "A Density Matrix-based Algorithm for Solving Eigenvalue
 * Problems") finds the eigenpairs of A x = lambda B x with lambda inside a
 * search interval [emin, emax], A real symmetric and B symmetric positive
 * definite (Sec. III.A, eq. 2).  One refinement loop of the real-symmetric
 * algorithm (Fig. 2) is:
 *   R   = B Y                                   (Y random first, Y = X later)
 *   Q   = -sum_e (w_e/2) Re{ r e^{i theta_e} (Z_e B - A)^{-1} R }     (eq. 15)
 *   A_Q = Q^T A Q,  B_Q = Q^T B Q                                     (eq. 7)
 *   A_Q Phi = eps B_Q Phi,  Phi^T B_Q Phi = I                         (eq. 6)
 *   lambda = eps,  X = Q Phi                                      (eqs. 8-9)
 * with Gauss-Legendre nodes x_e, weights w_e, r = (emax-emin)/2,
 * theta_e = -(pi/2)(x_e - 1), Z_e = (emax+emin)/2 + r e^{i theta_e}
 * (eqs. 13-14).  An in-interval Ritz pair counts as an eigenvalue solution
 * once its relative residual (below) is at most sqrt(tol).  Loops stop when
 * the count M of counted pairs is stable, the relative change of their trace
 * is below tol (Sec. III.B (i), Sec. IV.A), and no uncounted in-interval
 * pair is still converging (the smallest residual among them did not fall
 * below half its previous-loop value).  Fig. 2 counts every in-interval Ritz
 * value; the residual gate keeps mixtures of eigenvectors from both sides of
 * the interval out of M, so loop counts can differ from that literal rule.
 *
 * Matrices are block-tridiagonal with nc cells of b x b blocks (the shape of
 * nanowire / nanotube Hamiltonians):
 *   diag[nc][b][b]  row-major diagonal blocks (symmetric),
 *   up[nc-1][b][b]  row-major coupling block (i, i+1); block (i+1, i) is its
 *                   transpose.
 * Dense N x M0 arrays (N = nc*b) are row-major [N][M0].
 *
 * Memory: every pointer marked (dev) is HIP device memory owned by the caller;
 * (host) is host memory owned by the caller.  The context owns its workspace
 * (factors, subspaces, reduced matrices), grows it on demand and frees it in
 * feast_destroy.  Nothing the library allocates is handed to the caller.
 * Work is ordered on the stream given to feast_init; feast_solve synchronises
 * that stream before it returns.  A context must not be used by two host
 * threads at once.
 *
 * Status codes (int):
 *    0  success
 *   -1  nc < 1 or b < 1, or b above the supported maximum (96 for feast_solve,
 *       feast_solve_batched, feast_shifted_solve and feast_solve_hermitian, 64
 *       for the other calls)
 *   -2  emin >= emax or a bound is not finite
 *   -3  M0 < 1 or M0 > N, or M0 above the supported maximum, 128
 *   -4  Ne < 1 or Ne > 64
 *   -5  a required pointer is NULL
 *   -6  a non-finite value in A, B or Y0
 *   -7  bad option (tol <= 0, max_loops < 1, unknown precision)
 *   <= -100  HIP runtime error or out of memory: -100 - hipError_t
 *    1  not converged within max_loops (outputs hold the last loop)
 *    2  B_Q was not numerically positive definite in the last loop (a
 *       Cholesky pivot at or below 1e-12 times B_Q's diagonal entry in its
 *       row):
 *       the reduced problem was solved in the span of B_Q's eigenvectors
 *       with eigenvalue > 1e-10 max; dropped Ritz slots are returned last
 *       with lambda = NaN and a zero eigenvector
 *    3  no eigenvalue in the interval (M = 0)
 *    4  M = M0: the subspace is too small (Fig. 2 needs M0 > M)
 *    5  precision 1 only: the float64 refinement of a shifted solve stopped
 *       (10 corrections) above its tolerance (see feast_shifted_solve_mixed)
 * Positive codes are warnings: every output is written.
 */
#ifndef FEAST_MI355X_H
#define FEAST_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct feast_ctx feast_ctx;

/* Block-tridiagonal pencil (A, B); all four pointers (dev), float64. */
typedef struct {
  int32_t nc;            /* number of cells, >= 1 */
  int32_t b;             /* block size, 1..64; feast_solve,
                            feast_solve_batched and feast_shifted_solve also
                            take 65..96: such pencils run on the wide kernels
                            (blocks padded to 96; one top-down chain per
                            contour point, no twist and no partitions; B*Y,
                            the projection and the residuals from the same
                            repacked blocks), precision 0 only */
  const double *A_diag;  /* [nc][b][b] */
  const double *A_up;    /* [nc-1][b][b] (may be NULL when nc == 1) */
  const double *B_diag;  /* [nc][b][b] */
  const double *B_up;    /* [nc-1][b][b] (may be NULL when nc == 1) */
} feast_bt_matrix;

typedef struct {
  double tol;            /* relative trace change for convergence, e.g. 1e-12 */
  int32_t max_loops;     /* refinement loops allowed, >= 1 */
  int32_t precision;     /* 0: complex float64 shifted solves;
                            1: factor blocks rounded to float32, complex float32
                            sweeps, float64 iterative refinement of every
                            shifted solve (criterion: feast_shifted_solve_mixed);
                            2 (experiment, float64 factors): the first contour
                            integration by one float32 solve per node without
                            refinement, every later one in float64; the
                            convergence test compares two float64 loops.
                            b <= 64 for 1 and 2 */
  int32_t partitions;    /* partitions per half chain of the factorisation;
                            0 = automatic (at least 8 cells each, about one
                            chain per compute unit).  The partitioned
                            factorisation is exact in exact arithmetic; in
                            float64 its interface step loses accuracy at
                            contour points close to the real axis (measured
                            backward error of one shifted solve at
                            Im z = 1e-4: 8e-14 with 1 partition, 5e-12 with
                            10), so results depend on it beyond rounding
                            there */
  int32_t graph;         /* precision 0 only: 1 = the second contour
                            integration and the rest of its loop (B*Y, the
                            sweeps of all nodes, Q, the projection, the
                            reduced problem, X = Q Phi, the residuals, Y <- X)
                            are captured once as a HIP graph on the context's
                            stream and the graph is launched for every later
                            loop; the host still reads the convergence data
                            between loops.  The first loop runs eagerly.
                            Results are bitwise those of graph = 0; the
                            per-kernel timers see the eager launches only.
                            For callers that pay for launch latency (many
                            small problems).  2 = the convergence decision
                            runs on the device after every loop (same
                            decisions as the host's), and the loops are
                            captured four at a time into one graph whose
                            kernels return at once after convergence: one
                            graph launch and one host synchronisation per
                            four loops, Y and X alternating between two
                            buffers; bitwise the results of graph = 0;
                            max_loops <= 64.  0 = eager launches */
  const double *Y0;      /* (dev) [N][M0] initial subspace, or NULL: then
                            M0 random vectors are drawn on the device from
                            `seed` (Fig. 2 step 1): element t = i*M0 + j of
                            Y0 is standard normal from the counter-based
                            generator Philox4x64-10 (counter (t/4, 0, 0, 0),
                            key (seed, 0)); its four 64-bit words w_k give
                            u_k = (w_k >> 11) 2^-53 + 2^-54, and Box-Muller on
                            (u0, u1) and (u2, u3) gives four normals
                            sqrt(-2 ln u_a) cos(2 pi u_b), ... sin(2 pi u_b);
                            element t takes normal t % 4 */
  uint64_t seed;         /* key of the random start when Y0 is NULL */
  int32_t verbose;       /* 1 = one line per loop on stderr (loop, M, trace,
                            trace change); 0 = silent */
} feast_opts;

typedef struct {
  int32_t loops;         /* contour integrations performed */
  int32_t M;             /* counted pairs: inside [emin, emax] with
                            residual <= sqrt(tol) */
  double trace;          /* sum of their Ritz values (last loop) */
  double trace_rel;      /* relative trace change of the last loop */
  double max_res;        /* max residual over the M counted pairs */
  int32_t status;        /* same as the return value */
  int32_t fallback;      /* 1 if the last loop used the B_Q fallback */
  double trace_hist[64]; /* trace per loop (first min(loops,64) entries) */
  int32_t count_hist[64];/* M per loop */
  int32_t rr_sweeps;     /* Jacobi sweeps of the reduced eigensolver, all loops */
  int32_t refine_steps;  /* precision 1: float32 correction solves, all loops;
                            precision 2: loops run with float32 solves */
  double solve_res;      /* precision 1: largest final residual ratio of a
                            shifted solve column (feast_shifted_solve_mixed)
                            over all loops and nodes */
  int32_t m0_small;      /* 1 if M0 < 1.5 M: below the subspace size the
                            paper recommends after Fig. 2 (M0 >= 1.5 M); the
                            results stand, but more loops may be needed */
} feast_info;

/* Default options: tol 1e-12, max_loops 20, precision 0, partitions 0, graph 0,
   Y0 NULL (random start from seed 0), seed 0, verbose 0. */
void feast_default_opts(feast_opts *opts);

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t or
 * NULL for the default stream.  Returns 0 or a status <= -100. */
int feast_init(feast_ctx **ctx, int device, void *hip_stream);

/* Release the context and its workspace.  NULL is accepted. */
int feast_destroy(feast_ctx *ctx);

/* Human-readable text of a status code (static storage). */
const char *feast_strerror(int status);

/*
 * Full FEAST solve (Fig. 2, real symmetric case) on the GPU.
 *   lambda (dev) [M0]    Ritz values: the M counted ones first, ascending,
 *                        then the others ascending (uncounted values inside
 *                        the interval among them), NaN slots last.
 *   X      (dev) [N][M0] Ritz vectors in the same column order, B-orthonormal.
 *   res    (dev) [M0]    ||A x - lambda B x||_1 / ||A x||_1 per column
 *                        (Table I caption); when ||A x||_1 < r ||B x||_1 the
 *                        denominator is ||B x||_1 max(|emin|, |emax|, r).
 *   info   (host)        may be NULL.
 * The shifted systems are factored once per call (Sec. V, parallelism (ii))
 * and reused by every refinement loop.
 */
int feast_solve(feast_ctx *ctx, const feast_bt_matrix *AB, double emin, double emax,
                int32_t M0, int32_t Ne, const feast_opts *opts,
                double *lambda, double *X, double *res, feast_info *info);

/* ---- many problems ---- */

/* One problem of a batched call: every pointer as in feast_solve. */
typedef struct {
  feast_bt_matrix AB;
  double emin, emax;     /* search interval */
  int32_t M0, Ne;        /* subspace size, contour points */
  const double *Y0;      /* (dev) [N][M0] initial subspace, or NULL for the
                            random start of feast_opts (seed from opts) */
  double *lambda;        /* (dev) [M0] */
  double *X;             /* (dev) [N][M0] */
  double *res;           /* (dev) [M0] */
  feast_info *info;      /* (host) may be NULL */
  int32_t status;        /* out: what feast_solve returned for this problem */
} feast_problem;

/*
 * FEAST solves of `count` independent problems of any sizes (independent
 * problems or intervals: parallelism level (i) of Sec. V).  The problems are
 * taken longest first (estimated from nc, b, M0 and Ne) by `workers` host
 * threads, each with its own HIP stream (default priority) and workspace, so
 * that the kernels of several problems share the GPU.  opts applies to every
 * problem except Y0, which each problem brings; partitions 0 (automatic)
 * means one partition per half chain here (the problems fill the GPU
 * together, and the partitioned factorisation loses accuracy on some
 * problems whose contour points lie close to the real axis).
 * workers: 0 = min(count, 8);
 * the worker streams and workspaces belong to the context and are kept for
 * later calls.  Work queued on the context's stream before the call is
 * complete before any problem starts, and every problem is complete when the
 * call returns.  Returns the first negative per-problem status if any, else
 * the largest positive one, else 0; each problem's status is in
 * probs[i].status.  Results are identical to feast_solve on each problem
 * with the same options (partitions 0 read as 1).
 */
int feast_solve_batched(feast_ctx *ctx, feast_problem *probs, int32_t count,
                        const feast_opts *opts, int32_t workers);

/*
 * Partition count of the factorisation for one problem shape, measured: the
 * factorisation plus one forward and back sweep of (AB, emin, emax, M0, Ne)
 * are timed (after a warm-up) for 1, 2, 4, ... partitions per half chain up
 * to the largest with at least 8 cells each, and the fastest is returned in
 * *partitions (host), to be passed as feast_opts.partitions.  cache_path
 * (host string, may be NULL) names a text file of lines
 * "arch nc b M0 Ne partitions ms": a shape found there for this device is not
 * measured again, and a measured one is appended.  A count is taken only if
 * the shifted solve at the contour point nearest the real axis keeps a
 * relative residual within 10 times that of one partition (see the
 * partitions field of feast_opts).
 */
int feast_autotune_partitions(feast_ctx *ctx, const feast_bt_matrix *AB, double emin,
                              double emax, int32_t M0, int32_t Ne, const char *cache_path,
                              int32_t *partitions);

/* ---- single steps of the same path, for step-by-step parity checks ---- */

/*
 * Gauss-Legendre rule and contour of Sec. III.B (eqs. 13-15), host only.
 * Writes Ne values each (host): nodes x (ascending), weights w, the contour
 * points Z_e (real and imaginary parts) and the accumulation weights
 * kappa_e = -(w_e/2) r e^{i theta_e}, so that Q = sum_e Re(kappa_e Q_e).
 */
int feast_contour(int32_t Ne, double emin, double emax, double *x, double *w,
                  double *z_re, double *z_im, double *k_re, double *k_im);

/*
 * out = T V for one block-tridiagonal operator T = (diag, up) (dev, float64)
 * and a dense V [nc*b][m] (dev, row-major); out (dev) [nc*b][m].
 * `which` selects T: 0 = A, 1 = B of the pencil.  1 <= m <= 128.
 */
int feast_bt_multiply(feast_ctx *ctx, const feast_bt_matrix *AB, int32_t which,
                      int32_t m, const double *V, double *out);

/*
 * Solve (z B - A) X = R for one complex shift z with Im z > 0 (Fig. 2 step 2),
 * R real (dev) [N][m]; X_re, X_im (dev) [N][m].  1 <= m <= 128.
 * partitions: partitions per half chain of the factorisation as in
 * feast_opts (0 = automatic); ignored for 64 < b <= 96 (the wide kernels
 * factor one top-down chain).
 */
int feast_shifted_solve(feast_ctx *ctx, const feast_bt_matrix *AB, double z_re,
                        double z_im, int32_t m, const double *R, double *X_re,
                        double *X_im, int32_t partitions);

/*
 * Mixed-precision variant of feast_shifted_solve: the factor blocks of
 * (z B - A) are computed in float64 and rounded to float32, the sweeps run in
 * complex float32, and the float64 residual r = R - (z B - A) X drives
 * corrections X += solve32(r) until every column j satisfies
 *   ||r_j||_2 <= 1e-12 (||R_j||_2 + |z| ||B X_j||_2 + ||A X_j||_2),
 * at most 10 corrections.  (The bound is relative to the terms r is formed
 * from, so float64 rounding never keeps it out of reach.)  Arguments as
 * feast_shifted_solve; *steps (host, may be NULL) receives the corrections
 * made and *rel_res (host, may be NULL) the final worst ratio
 * ||r_j|| / (||R_j|| + |z| ||B X_j|| + ||A X_j||).  Returns 5 (outputs
 * written) when the bound was not reached.
 */
int feast_shifted_solve_mixed(feast_ctx *ctx, const feast_bt_matrix *AB, double z_re,
                              double z_im, int32_t m, const double *R, double *X_re,
                              double *X_im, int32_t partitions, int32_t *steps,
                              double *rel_res);

/*
 * The random start block of feast_solve with Y0 = NULL (Fig. 2 step 1):
 * Y (dev) [N][M0] receives the standard normal draws from `seed` described
 * at feast_opts.Y0.  N >= 1, 1 <= M0 <= 128.
 */
int feast_random_start(feast_ctx *ctx, uint64_t seed, int64_t N, int32_t M0, double *Y);

/*
 * One contour integration (Fig. 2 step 2, eq. 15 with RHS B Y):
 * Q = -sum_e (w_e/2) Re{ r e^{i theta_e} (Z_e B - A)^{-1} B Y }.
 * Y, Q (dev) [N][M0].
 */
int feast_filter(feast_ctx *ctx, const feast_bt_matrix *AB, double emin, double emax,
                 int32_t M0, int32_t Ne, const double *Y, double *Q);

/*
 * The same contour integration with the mixed-precision shifted solves of
 * feast_shifted_solve_mixed (all Ne systems refined together; *steps and
 * *rel_res as there, over all nodes).  Returns 5 (Q written) when the
 * refinement bound was not reached.
 */
int feast_filter_mixed(feast_ctx *ctx, const feast_bt_matrix *AB, double emin, double emax,
                       int32_t M0, int32_t Ne, const double *Y, double *Q, int32_t *steps,
                       double *rel_res);

/*
 * Projection (eq. 7): A_Q = Q^T A Q and B_Q = Q^T B Q, symmetrised.
 * Q (dev) [N][M0]; AQ, BQ (dev) [M0][M0].
 */
int feast_project(feast_ctx *ctx, const feast_bt_matrix *AB, int32_t M0,
                  const double *Q, double *AQ, double *BQ);

/*
 * Reduced generalized eigenproblem (eq. 6): A_Q Phi = eps B_Q Phi with
 * Phi^T B_Q Phi = I, eps ascending (NaN slots last, see status 2).
 * AQ, BQ (dev) [M0][M0] symmetric; eps (dev) [M0]; Phi (dev) [M0][M0].
 * *fallback (host) is set to 1 when B_Q was not numerically s.p.d.
 */
int feast_reduced_eig(feast_ctx *ctx, int32_t M0, const double *AQ, const double *BQ,
                      double *eps, double *Phi, int32_t *fallback);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * reduced eigensolve as feast_reduced_eig, with identical results, but its
 * workspace is a file-scope device array of the library (1.7 MB on every GPU
 * the library runs on, held until the process ends) instead of the
 * context's; the call allocates nothing.  M0 is limited to 128 (the size
 * the array holds): larger values return -3.  All calls on one GPU share
 * that array, so calls that overlap in time on one GPU (from several
 * contexts or streams) race and must be serialised by the caller; nothing in
 * the array needs to start at zero (every part is written before it is
 * read).  Arguments and results as feast_reduced_eig.
 */
int feast_reduced_eig_noalloc(feast_ctx *ctx, int32_t M0, const double *AQ, const double *BQ,
                              double *eps, double *Phi, int32_t *fallback);

/* ---- instrumentation ---- */

/*
 * Kernel timing.  feast_timing(ctx, 1) clears the records and, until
 * feast_timing(ctx, 0), brackets every kernel class that feast_solve and
 * feast_solve_hermitian launch with hipEvents on the context's stream.
 * feast_timing_read(ctx, k, ...) synchronises the stream and returns, for
 * class k, its name (static string), the summed event time in milliseconds
 * and the number of launches; with k < 0 it returns the number of classes.
 * Classes: factor, forward_sweep, back_sweep, bt_multiply, sum_nodes,
 * projection, reduced_eig, ritz_gemm, residual, layout, round_factors,
 * forward_sweep32, back_sweep32, refine_residual (the last four with
 * precision 1 or 2 only), sweeps_hermitian (the forward and back sweeps of
 * both solves of eq. 12 in one kernel).
 */
int feast_timing(feast_ctx *ctx, int32_t enable);
int feast_timing_read(feast_ctx *ctx, int32_t kind, const char **name, double *total_ms,
                      int64_t *launches);

/* ---- Hermitian A (Sec. III.B, eq. 12, and the changes listed after Fig. 2) ----
 *
 * A complex Hermitian, B real symmetric positive definite (Sec. III.A).  The
 * start block Y, the subspace Q, the reduced eigenvectors Phi and the Ritz
 * vectors X are complex; one contour integration is eq. 12 with RHS B Y:
 *   Q = -sum_e (w_e/4) r (e^{i theta_e} G(Z_e) + e^{-i theta_e} G(Z_e)^H) B Y,
 * G(Z) = (Z B - A)^{-1}; the adjoint solve G(Z_e)^H uses the factorisation of
 * Z_e B - A (G(conj Z) = G(Z)^H).  A_Q = Q^H A Q and B_Q = Q^H B Q are
 * Hermitian; the reduced problem is brought to a real symmetric
 * tridiagonal one of size M0 (Cholesky of B_Q, Householder reduction of
 * L^-1 A_Q L^-H, a diagonal phase scaling) for the real eigensolver, or, when
 * B_Q fails the Cholesky pivot test, solved through its real symmetric
 * embedding [[Re, -Im], [Im, Re]] of size 2 M0 with the B_Q fallback of
 * feast_solve.  Complex arrays are interleaved (re, im) doubles (C99 double
 * complex, torch.complex128).  Counting, convergence, residual and output
 * order as in feast_solve (residual 1-norms of complex moduli).
 * Limits: b <= 96, M0 <= 64.  For b <= 64 the factorisation is twisted and
 * partitioned as for feast_solve (opts.partitions per half chain, 0 =
 * automatic by the same rule); 64 < b <= 96 factors one chain per contour
 * point in order.
 */
typedef struct {
  int32_t nc;            /* number of cells, >= 1 */
  int32_t b;             /* block size, 1..96 */
  const double *A_diag;  /* (dev) complex [nc][b][b], Hermitian blocks */
  const double *A_up;    /* (dev) complex [nc-1][b][b]; block (i+1, i) is the
                            conjugate transpose of block (i, i+1) */
  const double *B_diag;  /* (dev) real [nc][b][b], as feast_bt_matrix */
  const double *B_up;    /* (dev) real [nc-1][b][b] */
} feast_zbt_matrix;

/* Full FEAST solve for Hermitian A.  lambda (dev) [M0] real; X (dev) complex
 * [N][M0], B-orthonormal (X^H B X = I); res (dev) [M0].  opts as feast_solve
 * (precision 0 only; Y0 complex [N][M0] or NULL: then the real and imaginary
 * parts are the seeded standard normal draws of an N x 2 M0 real block,
 * interleaved).  Errors as feast_solve; b > 96 gives -1, M0 > 64 gives -3. */
int feast_solve_hermitian(feast_ctx *ctx, const feast_zbt_matrix *AB, double emin, double emax,
                          int32_t M0, int32_t Ne, const feast_opts *opts, double *lambda,
                          double *X, double *res, feast_info *info);
/* X (dev, complex [N][m]) = (z B - A)^{-1} R, or (z B - A)^{-H} R when
 * adjoint != 0, for complex R (dev) [N][m], Im z > 0, m <= 64.  partitions
 * as in feast_opts (0 = automatic, ignored for b > 64; -7 if negative). */
int feast_shifted_solve_hermitian(feast_ctx *ctx, const feast_zbt_matrix *AB, double z_re,
                                  double z_im, int32_t m, const double *R, int32_t adjoint,
                                  double *X, int32_t partitions);
/* One contour integration of eq. 12 (RHS B Y): Y, Q (dev) complex [N][M0]. */
int feast_filter_hermitian(feast_ctx *ctx, const feast_zbt_matrix *AB, double emin, double emax,
                           int32_t M0, int32_t Ne, const double *Y, double *Q);

/* ---- learned warm start for a Hamiltonian family ----
 *
 * An extension of the project, rooted in the subspace reuse of Sec. IV.C
 * (Example III: nearby problems start from a previous solution) and Sec. V:
 * for a family of pencils parameterised by a vector a (here the amplitudes
 * of the onsite potential), a multilayer perceptron maps a to the start block
 * Y0 of feast_solve.  The network is d0 -> d1 -> d2 -> d3 with ReLU after
 * the two hidden layers; every product runs on the matrix cores with the
 * operands rounded to bfloat16 (round to nearest even) and float32 sums;
 * master weights, gradients and Adam moments are float32.  Its targets are
 * gauge-free: for a member with converged B-orthonormal eigenvectors X_in
 * (the counted pairs) and a fixed start block Y_ref, T = X_in X_in^T B Y_ref,
 * the output of one contour integration of an exact filter.  Per cell c of
 * b rows, T_c is represented as U_c C_c with an r-column basis U_c (the
 * leading eigenvectors of sum_s T_c,s T_c,s^T over the training set); the
 * network predicts the coefficients C ([nc][r][m], so d3 = nc r m) and the
 * start block is Y_c = U_c C_c.  Random Y stays the fallback: the FEAST
 * residual judges every result.
 */
typedef struct feast_mlp feast_mlp;

/* Parameters (dev, float32) are packed as W1 [d1][d0], b1 [d1], W2 [d2][d1],
 * b2 [d2], W3 [d3][d2], b3 [d3].  dims = {d0, d1, d2, d3}, each a multiple of
 * 16; max_batch a multiple of 16.  The network copies the parameters and
 * owns its device memory until feast_mlp_destroy.  Errors: -1 bad dims,
 * -3 bad max_batch, -5 NULL. */
int feast_mlp_create(feast_ctx *ctx, const int32_t dims[4], int32_t max_batch,
                     const float *params, feast_mlp **net);
int feast_mlp_destroy(feast_mlp *net);
/* Current float32 parameters into params (dev, packed as above). */
int feast_mlp_params(feast_mlp *net, float *params);
/* y (dev) [batch][d3] = network(x), x (dev) [batch][d0]; 1 <= batch <= max_batch. */
int feast_mlp_forward(feast_mlp *net, int32_t batch, const float *x, float *y);
/* Gradients of the mean squared error mean((y - target)^2) over
 * batch x d3 entries with respect to the parameters, into grads (dev,
 * packed as the parameters); *loss (host, may be NULL) gets the loss.
 * batch a multiple of 16.  The parameters are not changed. */
int feast_mlp_gradients(feast_mlp *net, int32_t batch, const float *x, const float *target,
                        float *grads, double *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; Kingma and
 * Ba) on the gradients of feast_mlp_gradients, learning rate lr > 0. */
int feast_mlp_train_step(feast_mlp *net, int32_t batch, const float *x, const float *target,
                         float lr, double *loss);

/* G (dev) [m][m2] = X^T V for tall X (dev) [N][ldx] (first m columns) and
 * V (dev) [N][ldv] (first m2 columns), float64, m, m2 <= 128;
 * workspace (dev) of feast_cross_gram_workspace(N, m, m2) doubles.  Sums in a
 * fixed order (deterministic). */
int feast_cross_gram(feast_ctx *ctx, int64_t N, int32_t m, int32_t m2, const double *X,
                     int32_t ldx, const double *V, int32_t ldv, double *workspace, double *G);
int64_t feast_cross_gram_workspace(int64_t N, int32_t m, int32_t m2);
/* T (dev) [N][m2] = X G for X (dev) [N][ldx] (first m columns), G (dev)
 * [m][m2], float64. */
int feast_tall_gemm(feast_ctx *ctx, int64_t N, int32_t m, int32_t m2, const double *X,
                    int32_t ldx, const double *G, double *T);
/* Gc (dev) [nc][b][b] += T_c T_c^T for the cell row blocks T_c of T (dev)
 * [nc*b][m], float64, b <= 64, m <= 128. */
int feast_cell_gram_accumulate(feast_ctx *ctx, int32_t nc, int32_t b, int32_t m,
                               const double *T, double *Gc);
/* C (dev, float32) [nc][r][m] = scale * U_c^T T_c for U (dev) [nc][b][r] and
 * T (dev) [nc*b][m], float64 arithmetic. */
int feast_basis_project(feast_ctx *ctx, int32_t nc, int32_t b, int32_t r, int32_t m,
                        const double *U, const double *T, double scale, float *C);
/* Y (dev) [nc*b][m] = scale * U_c C_c per cell + rscale * R, C (dev, float32)
 * [nc][r][m], R (dev) [nc*b][m] or NULL; float64 result (a start block for
 * feast_solve: a prediction of T spans only the M in-interval directions, so
 * the start block adds a random block R, e.g. from feast_random_start, to
 * give the other M0 - M columns directions). */
int feast_basis_expand(feast_ctx *ctx, int32_t nc, int32_t b, int32_t r, int32_t m,
                       const double *U, const float *C, double scale, const double *R,
                       double rscale, double *Y);

#ifdef __cplusplus
}
#endif

#endif /* FEAST_MI355X_H */
