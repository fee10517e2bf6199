/*
 * gsi -- gradient-type subspace iteration on MI355X (gfx950).
 *
 * Computes an orthonormal basis X (n x p) of the dominant invariant subspace of a sparse
 * symmetric matrix A by minimizing phi(X) = -1/2 Tr(X^T A X) over X^T X = I
 * (Sec. 2.2, eq. phi) with Riemannian steepest descent (Algorithm 2) or Riemannian
 * nonlinear conjugate gradients with Polak-Ribiere directions (Sec. 5.1, Algorithm 4),
 * each step using the polar retraction (Sec. 3.1 eq. Ynew, Sec. 5.2 eq. Xnew_P) and the
 * exact line search on the p x p projected problem (Sec. 3.2, Algorithm 3; Sec. 5.2
 * eq. phi_P / deriv_P; Sec. 6.1). A X is carried by the recursion of Sec. 6.1
 * (eq. save_matvec) so that one block product A*P is formed per iteration.
 * The smallest eigenvalues are targeted by running on -A (Sec. 2.2).
 *
 * Conventions for every entry point:
 *  - All n x p blocks are row-major with leading dimension p (no padding), in device
 *    memory owned by the caller. Matrix arrays passed to gsi_create are device pointers
 *    owned by the caller; gsi_create copies what it needs, the caller may free them after.
 *  - All work is ordered on the HIP stream given to gsi_create (NULL = default stream).
 *    Calls marked "syncs" wait for that stream before returning.
 *  - No exceptions or aborts cross this interface. Every call returns a gsi_status; the
 *    text of the last error of a handle is returned by gsi_last_error.
 *  - A handle must not be used from two host threads at once.
 */
#ifndef GSI_H
#define GSI_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsi_ctx* gsi_handle;

typedef enum {
  GSI_OK = 0,
  GSI_EINVAL = 1,         /* invalid argument (sizes, pointers, options, CSR structure) */
  GSI_ENOMEM = 2,         /* device allocation failed */
  GSI_EDEVICE = 3,        /* a HIP call failed (text in gsi_last_error) */
  GSI_NOT_CONVERGED = 4,  /* max_iter reached; the iterate stays valid */
  GSI_BREAKDOWN = 5,      /* non-finite values or a rank-deficient block */
  GSI_EUNSUPPORTED = 6    /* option combination not built (e.g. p above the supported maximum) */
} gsi_status;

typedef enum {
  GSI_RSD = 1,  /* Riemannian steepest descent with exact line search (Algorithm 2) */
  GSI_RCG = 2,  /* Riemannian nonlinear CG, Polak-Ribiere, exact line search (Algorithm 4) */
  GSI_SI = 3    /* subspace iteration with a polynomial filter (Algorithm 1): per iteration
                   X_hat = p_d(A) X, Cholesky QR, Rayleigh-Ritz X <- Q U, A X <- (A Q) U; the
                   filter is the monomial (cheb_degree 0) or the Chebyshev polynomial of
                   eq. optimal_poly over [cheb_lo, cheb_hi] normalized at cheb_top. Float64,
                   stopping test as for the other methods; gsi_step runs outer iterations
                   synchronously */
} gsi_method;

typedef enum {
  GSI_FP64 = 0,        /* every step in float64 */
  GSI_MIXED_FP32 = 1,  /* SpMM, Gram and update passes in float32 (float32 accumulation) with
                          float64 small solves, until rho <= switch_tol or rho stops halving
                          for stall_window iterations; then the float64 phase continues the
                          conjugate-gradient recursion to tol. Its SpMM reads float32 copies
                          of A and P with float64 products and sums (the rounding of A and P
                          enters the A X recursion at u32 times the step, which shrinks with
                          the gradient); gsi_solve confirms convergence with A X and X^T A X
                          formed in float64 before it returns */
  GSI_MIXED_BF16 = 2   /* as GSI_MIXED_FP32, but the iteration's SpMM reads bfloat16 matrix
                          values and a bfloat16 copy of P (written by the direction pass,
                          rounded to nearest even) with float32 accumulation and a float32
                          result: half the gather bytes of float32 (the explicit A X
                          refreshes keep float32 values) */
} gsi_precision;

/* Full symmetric CSR (both triangles stored), int32 row pointers and column indices,
 * float64 values, all device pointers. Column indices must be sorted within a row. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t* rowptr; /* n + 1 */
  const int32_t* colind; /* nnz */
  const double* vals;    /* nnz */
} gsi_csr;

/* A complex Hermitian matrix in CSR form: vals holds nnz complex values as interleaved
 * (real, imaginary) float64 pairs; the full matrix is stored (both triangles). */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t* rowptr; /* n + 1 */
  const int32_t* colind; /* nnz, sorted within each row */
  const double* vals;    /* 2 nnz */
} gsi_zcsr;

/* A 5- or 7-point stencil operator on an nx x ny x nz grid of nodes in lexicographic order
 * (x fastest; ny = nz = 1 for a 1D grid, nz = 1 for 2D), applied without index or value
 * arrays: row r has diag + diag_vec[r] on the diagonal and off at each neighbour inside the
 * grid (r -+ 1, r -+ nx, r -+ nx ny). The Dirichlet Laplacians and Schroedinger operators
 * -Laplacian + V of the test problems (Sec. 6) are of this form: diag = 2 d / h^2, off =
 * -1 / h^2, diag_vec = V (d the dimension). */
typedef struct {
  int64_t nx, ny, nz;      /* grid sides, >= 1, n = nx ny nz < 2^31 */
  double diag;             /* constant part of the diagonal */
  double off;              /* weight of every neighbour */
  const double* diag_vec;  /* nullable device array of n values added to the diagonal */
} gsi_stencil;

typedef struct {
  int32_t p;            /* block size, 1 <= p < n; p <= 128 for RCG / RSD on a CSR matrix with
                           explicit_c = 0 (any precision), p <= 64 otherwise (GSI_EUNSUPPORTED) */
  int32_t which;        /* +1 largest eigenvalues, -1 smallest (the solver runs on -A) */
  int32_t method;       /* gsi_method */
  int32_t precision;    /* gsi_precision */
  int32_t recompute_ax; /* 0: A X by the recursion of Sec. 6.1; 1: A X formed every iteration
                           (the RCG(+) variant of Sec. 6.4); -1: automatic, each solve times
                           a few iterations of both on the device and keeps the faster
                           (gsi_recompute_choice reports the outcome) */
  int32_t k_restart;    /* restart the CG direction every k_restart iterations (0 = never) */
  int32_t max_iter;     /* iteration cap (accepted steps) */
  double tol;           /* stop when rho = ||G||_F / (sqrt(p) ||A||_inf) <= tol */
  double switch_tol;    /* mixed precision: rho at which the float64 refinement phase starts */
  int32_t check_every;  /* gsi_solve polls the convergence flag every this many iterations */
  int32_t use_graph;    /* capture the per-iteration launch sequence in a HIP graph */
  int32_t explicit_c;   /* 1: form C = X^T A X and W = X^T P_old by Gram passes in the retraction
                           pass; 0: carry them by the p x p recursion C <- M (C - mu (P^T Y +
                           Y^T P) + mu^2 P^T Z) M, W <- -mu M P^T P */
  int32_t stall_window; /* mixed precision: the low-precision phase also ends when rho has not
                           halved for this many iterations (its rounding floor); >= 1 */
  int32_t cheb_degree;  /* GSI_SI: 0 monomial filter p(t) = t; d >= 1 Chebyshev filter of degree d
                           (d products with A per outer iteration) */
  double cheb_lo;       /* GSI_SI with d >= 1: interval [cheb_lo, cheb_hi] of the unwanted
                           eigenvalues of the operator solved (-A when which = -1), i.e.
                           [lambda_n, lambda_{p+1}] of eq. optimal_poly, and an estimate */
  double cheb_hi;       /* cheb_top > cheb_hi of its largest eigenvalue (the normalization */
  double cheb_top;      /* point that keeps the filtered block bounded) */
  int32_t check_symmetric; /* 1: gsi_create also verifies that A equals its transpose (every
                              stored a_ij has a stored a_ji of the same value; GSI_EINVAL
                              otherwise); 0: not checked (the methods assume it, Sec. 2) */
  uint64_t x0_seed;     /* seed of the start block drawn on the device when X0 == NULL */
} gsi_options;

/* Fill *opt with defaults: p=8, which=+1, RCG, FP64, recursion, no restart, max_iter=10000,
 * tol=1e-8, switch_tol=1e-5, check_every=25, use_graph=1, explicit_c=0, stall_window=60,
 * cheb_degree=0, check_symmetric=0, x0_seed=0. */
void gsi_options_default(gsi_options* opt);

/* Create a solver for A with options opt, starting block X0 (n x p float64, device; its
 * columns need not be orthonormal: the library orthonormalizes them by two passes of
 * Cholesky QR). X0 == NULL: the start block is drawn on the device, entries i.i.d. N(0,1)
 * (the random start of the experiments, Sec. 6) from opt->x0_seed by a counter-based
 * generator: entry e = i p + j of the row-major block is sqrt(-2 ln u1) cos(2 pi u2) (Box
 * and Muller 1958) with u1, u2 = ((o >> 11) + 1/2) 2^-53 for the outputs o number 2e and
 * 2e + 1 of SplitMix64 (Steele, Lea and Flood 2014) started at state x0_seed, output k being
 * mix(x0_seed + (k + 1) 0x9E3779B97F4A7C15), mix(z): z ^= z >> 30, z *= 0xBF58476D1CE4E5B9,
 * z ^= z >> 27, z *= 0x94D049BB133111EB, z ^= z >> 31 (mod 2^64). Validates sizes and CSR
 * structure (monotone rowptr, column indices in range). On success *h owns device copies of
 * A and X0 and all workspace; gsi_step / gsi_solve never allocate. Syncs. */
gsi_status gsi_create(gsi_handle* h, const gsi_csr* A, const gsi_options* opt, const double* X0,
                      void* hip_stream);

/* As gsi_create for a matrix-free stencil operator: every product with A reads the block
 * once (the neighbours from the caches) and the n diagonal values, and no index or value
 * arrays (Sec. 6.4 observes that the cost of a product with a very sparse A relative to the
 * rest of the iteration decides between RCG and RCG(+); a stencil makes that product as
 * cheap as a streaming pass). The results equal those of gsi_create on the same matrix in
 * CSR form (same arithmetic, same order). diag_vec is copied; gsi_set_values on such a
 * handle takes n new diag_vec values. GSI_MIXED_BF16 is not supported (GSI_EUNSUPPORTED). */
gsi_status gsi_create_stencil(gsi_handle* h, const gsi_stencil* S, const gsi_options* opt, const double* X0,
                              void* hip_stream);

/* Complex Hermitian variant (the extension the paper notes for Hermitian A: the iteration
 * with conjugate transposes on phi(X) = -1/2 Re Tr(X^H A X), X^H X = I). A is held as its
 * real symmetric embedding [[Re A, -Im A], [Im A, Re A]] (2n x 2n) and X as the 2n x 2p real
 * block [[Re X, -Im X], [Im X, Re X]]: the real iteration on this block spans the embedding
 * of the complex iterate at every step (phi and the real inner product of the embedding are
 * twice the complex ones, so the step sizes and Polak-Ribiere coefficients are the same), at
 * twice the memory traffic of native complex arithmetic. opt->p is the number of complex
 * columns, 1 <= p <= 32; X0: device array of n x p complex values (interleaved, row-major).
 * The stopping test uses ||A_emb||_inf (the max over rows of sum |Re a| + |Im a|). Other
 * calls (gsi_solve, gsi_step, gsi_history, gsi_counters) act on the embedded problem; read
 * results with gsi_hermitian_results. Builds the embedding on the host (copies A and X0 out
 * and back); syncs. Errors as gsi_create; p > 32 gives GSI_EUNSUPPORTED. */
gsi_status gsi_create_hermitian(gsi_handle* h, const gsi_zcsr* A, const gsi_options* opt, const double* X0,
                                void* hip_stream);

/* Rayleigh-Ritz of a Hermitian handle's iterate: ritz (host, p; nullable) the Ritz values
 * of A, largest first for which = +1, smallest first for -1; Xc (device, n x p complex
 * interleaved; nullable) the Ritz vectors; rho (host, nullable) the residual measure. Each
 * eigenvalue of the embedding is a complex eigenvalue twice, with the pair's real vectors
 * spanning one complex vector; column j of Xc is the first vector of pair j read as
 * complex. A complex eigenvalue of multiplicity above one inside the block has a
 * four-dimensional real eigenspace whose Ritz vectors need not pair up this way, so such
 * blocks should be cut between distinct eigenvalues. Syncs. */
gsi_status gsi_hermitian_results(gsi_handle h, double* ritz, double* Xc, double* rho);

/* The variant an automatic solve (recompute_ax = -1) chose: *recompute_ax 0 (recursion) or
 * 1 (RCG(+)), and the measured milliseconds per iteration of each (0 until a solve ran the
 * trial; a handle created with recompute_ax >= 0 reports its fixed choice). Sec. 6.4 finds
 * RCG(+) the cheaper one when a product with A costs less than the recursion's extra block
 * traffic, i.e. for very sparse A; the trial measures that on the actual matrix. */
gsi_status gsi_recompute_choice(gsi_handle h, int32_t* recompute_ax, double* ms_recursion, double* ms_recompute);

/* Enqueue n_iter iterations (fewer if the convergence flag is raised on the device;
 * the remaining launches return immediately). Asynchronous. */
gsi_status gsi_step(gsi_handle h, int32_t n_iter);

/* Iterate until rho <= tol or max_iter accepted steps. *iters_out (nullable) receives the
 * number of accepted steps. Returns GSI_OK, GSI_NOT_CONVERGED or GSI_BREAKDOWN. Syncs. */
gsi_status gsi_solve(gsi_handle h, int32_t* iters_out);

/* Rayleigh-Ritz on the current X (Sec. 2.3, eq. rr1): Ritz values of A (host array of p,
 * largest first for which=+1, smallest first for which=-1), per-column residual norms
 * ||A u_i - theta_i u_i|| (host array of p), rho and phi (host scalars). Any output may be
 * NULL. Replaces X by the Ritz vectors X U (same span). Syncs. */
gsi_status gsi_residuals(gsi_handle h, double* ritz, double* col_res, double* rho, double* phi);

/* Copy the current X (n x p, row-major, float64) to the device pointer X_out. Syncs. */
gsi_status gsi_get_x(gsi_handle h, double* X_out);

/* Replace the iterate by span(X0) (n x p float64 device block; orthonormalized inside) and
 * reset the iteration state: a warm start (Sec. 2.3: restarting from a previous subspace). */
gsi_status gsi_set_x0(gsi_handle h, const double* X0);

/* Subspace tracking (Sec. 1 and 2.3: sequences of related eigenproblems, where a method that
 * can start from the previous subspace pays only for the change): replace the matrix values
 * by vals (device array of nnz float64 in the CSR order and sparsity pattern given at
 * creation; for a stencil handle, n float64 values that take the place of diag_vec, the
 * diagonal term added to diag), recompute ||A||_inf, and restart the iteration from the current basis, which
 * stays the iterate (orthonormalized again; the solver state is reset as by gsi_set_x0).
 * Errors: GSI_EINVAL (null), GSI_BREAKDOWN (a non-finite value; the handle keeps the old
 * values), GSI_EDEVICE. */
gsi_status gsi_set_values(gsi_handle h, const double* vals);

/* Z = A_op W for the handle's operator (A, or -A when which = -1), W and Z n x p float64
 * device blocks. The same SpMM kernel the iteration uses. It stages through the handle's
 * gradient buffer: called between steps, the next step forms the gradient again and restarts
 * the conjugate direction. Asynchronous. */
gsi_status gsi_spmm(gsi_handle h, const double* W, double* Z);

/* Z = A W (device, n x p float64 row-major in and out) in the handle's low-phase precision:
 * float32 values, W rounded to float32, float32 accumulation (GSI_MIXED_FP32), or bfloat16
 * values and W rounded to bfloat16 (nearest even), float32 accumulation (GSI_MIXED_BF16);
 * A is the operator solved (negated for which = -1). GSI_EUNSUPPORTED for a float64
 * handle. For checking the low-precision SpMM; uses the handle's scratch blocks, so call it
 * between solves (a following step restarts as after gsi_spmm). */
gsi_status gsi_spmm_lowp(gsi_handle h, const double* W, double* Z);

/* Per-iteration history, host arrays of length >= count (nullable): rho, phi, mu, beta_pr
 * and ||G||_inf / ||G_0||_inf per recorded iterate. Returns the number of records in
 * *count (at most the capacity passed in *count). Syncs. */
gsi_status gsi_history(gsi_handle h, int32_t* count, double* rho, double* phi, double* mu,
                       double* beta_pr, double* ginf_rel);

/* Counters: accepted iterations, block products with A, restarts, explicit A X refreshes,
 * null steps (line search or descent test failed: the next step restarts), low-precision
 * iterations (mixed mode), Jacobi sweeps of the P^T P eigendecompositions (summed). Any
 * pointer may be NULL. Syncs. */
gsi_status gsi_counters(gsi_handle h, int32_t* iters, int32_t* spmm, int32_t* restarts,
                        int32_t* refreshes, int32_t* null_steps, int32_t* low_iters, int32_t* eig_sweeps);

/* Per-pass kernel timing with HIP events recorded on the handle's stream around every
 * launch of the iteration. Indices of ms[] / counts[] (arrays of GSI_NPASS, nullable): */
enum {
  GSI_PASS_GRAD = 0,       /* gradient pass */
  GSI_PASS_DIR = 1,        /* direction pass */
  GSI_PASS_SPMM = 2,       /* block SpMM A P */
  GSI_PASS_UPDATE = 3,     /* retraction pass; for the float64 gradient-type iterations with C
                              and W carried by the recursion (explicit_c = 0) the retraction
                              pass also forms the next gradient and its sums, and GSI_PASS_GRAD
                              then counts the gradient passes launched at the top of every
                              iteration, which run only after an explicit A X, a void step or
                              a restart of the state (the others return at once) */
  GSI_PASS_REDUCE = 4,     /* fixed-order reductions of partial sums */
  GSI_PASS_SMALL = 5,      /* p x p kernels other than the line search */
  GSI_PASS_LINESEARCH = 6, /* line-search diagonals, Get_Mu, M and the next C, W */
  GSI_PASS_REFRESH = 7,    /* explicit A X (launched every iteration, runs when requested) */
  GSI_PASS_EIG = 8,        /* eigendecomposition of P^T P (second stream, overlaps the SpMM) */
  GSI_PASS_GRAM = 9,       /* Gram pass P^T A P, P^T A X after the SpMM */
  GSI_NPASS = 10
};
/* Returns the accumulated milliseconds and launch counts since the last reset, then, if
 * enable >= 0, resets them and turns timing on (1) or off (0). While timing is on, gsi_solve
 * launches without the graph and polls every iteration. Syncs. */
gsi_status gsi_pass_times(gsi_handle h, int32_t enable, double* ms, int32_t* counts);

/* Orthonormalize a caller's block in place by two passes of Cholesky QR: X <- X R^{-1} with
 * R^T R = X^T X (R upper triangular with a positive diagonal), twice; the result spans the
 * same space as X with X^T X = I to rounding. This is the re-orthonormalization step the
 * solver applies to its start block (the paper assumes an orthonormal X0, Sec. 3 and
 * Algorithm 2; Cholesky QR is one of the admissible ways to produce it), offered as a call of
 * its own. X: device array, n x p float64, row-major with leading dimension p, owned by the
 * caller. 1 <= p <= 64 (GSI_EUNSUPPORTED above), n >= p (GSI_EINVAL otherwise, and for a null
 * X). GSI_BREAKDOWN when a pivot of the factorization is not above 1e-13 times the largest
 * diagonal entry of X^T X or is not finite (rank deficient or non-finite X): X then holds the
 * input (first pass failed) or the result of the first pass. Work is ordered on hip_stream
 * (NULL = default stream); allocates a 4.3 MB scratch buffer for the call and frees it; the
 * Gram sums are added in a fixed order, so results repeat bit for bit. Syncs. */
gsi_status gsi_orthonormalize(double* X, int64_t n, int32_t p, void* hip_stream);

/* gsi_orthonormalize for callers that cannot allocate device memory (code under HIP graph
 * capture aside, tight serving loops, harnesses that forbid allocation): the same kernels,
 * results and errors, with the scratch buffer in a file-scope device array of 4.3 MB that
 * every device the library runs on holds until the process ends (its address is looked up
 * once per device, on the first call made with that device current). Calls no hipMalloc or
 * hipFree. The limit is the same, 1 <= p <= 64 (any n >= p). Every call on a device shares that
 * device's array and overwrites what it reads, so calls that overlap on one device (two
 * streams or two host threads) race and must be serialized by the caller. Syncs. */
gsi_status gsi_orthonormalize_noalloc(double* X, int64_t n, int32_t p, void* hip_stream);

/* Measurement aid (no part of the method): the device's streaming rates with the access
 * pattern of the solver's streaming passes (16-byte loads and non-temporal stores per lane,
 * grid-stride over contiguous memory), the ceiling the kernels' HBM rates are compared with next to the
 * published peak. a and b: device buffers of `bytes` bytes each (16-byte aligned, bytes a
 * multiple of 16), owned by the caller; a is only read, b is written (it ends equal to a).
 * us (host, 3 doubles) receives the mean time per launch over `reps` launches after one
 * untimed launch, timed with HIP events on hip_stream, of: us[0] copy a -> b (2 x bytes
 * moved), us[1] read a, us[2] write b (run first). GSI_EINVAL for null or misaligned pointers
 * or sizes, GSI_EDEVICE for a HIP error. Syncs. */
gsi_status gsi_stream_rates(void* a, void* b, int64_t bytes, int32_t reps, double* us, void* hip_stream);

void gsi_destroy(gsi_handle h);
const char* gsi_status_str(gsi_status s);
const char* gsi_last_error(gsi_handle h);

/* ------------------------------------------------------------------------------------------
 * Batched solve: count independent problems (A[i], p[i], X0[i]) of different sizes solved by
 * one persistent kernel launch, captured in a HIP graph. Each workgroup takes problems from
 * an atomic queue (largest n*p first) and runs the whole iteration of one problem (Sec. 5,
 * Algorithm 4, with the same readings as gsi_solve) with workgroup barriers only. Options
 * shared by all problems: which, method, precision, recompute_ax, k_restart, max_iter, tol,
 * switch_tol, stall_window. GSI_FP64: float64 blocks throughout. GSI_MIXED_FP32: float32
 * blocks with float64 p x p solves until rho <= max(switch_tol, tol) or until rho has not
 * halved for stall_window iterations, then the iterate, previous gradient and previous direction are widened to
 * float64 and the iteration continues to tol without a restart. 1 <= p[i] <= 32, p[i] < n.
 * Arrays A, p, X0 are host arrays of count entries; the CSR arrays (float64 values) and
 * X0[i] (n x p float64, row-major) are device pointers owned by the caller and copied.
 * Errors: GSI_EINVAL (bad sizes, invalid CSR, non-finite values, problem index reported by
 * gsi_batched_last_error), GSI_ENOMEM, GSI_EDEVICE. The handle is returned even on failure
 * (for the message) and must be destroyed. */
typedef struct gsi_batch* gsi_batch_handle;
gsi_status gsi_create_batched(gsi_batch_handle* h, int32_t count, const gsi_csr* A, const int32_t* p,
                              const gsi_options* opt, const double* const* X0, void* hip_stream);
/* Runs the persistent launch; every call solves from the X0 given at creation. iters /
 * status: host arrays of count (nullable); iters counts all iterations of both phases;
 * status per problem: 1 converged (rho <= tol), 2 max_iter, 3 breakdown. Returns
 * GSI_BREAKDOWN if any problem broke down, else GSI_NOT_CONVERGED if any reached max_iter,
 * else GSI_OK; GSI_EDEVICE if a team barrier waited longer than the wait limit (30 s unless
 * gsi_batched_set_wait_limit changed it): the launch is then abandoned by every team, whose
 * problems get status 5, while problems solved by one workgroup finish normally. Syncs. */
gsi_status gsi_solve_batched(gsi_batch_handle h, int32_t* iters, int32_t* status);
/* Ritz values of problem i (host array of p[i], of A: largest first for which = +1, of -A
 * for which = -1, i.e. the negated smallest eigenvalues of A, largest first), its final rho
 * and restart count (any output nullable). Syncs. */
gsi_status gsi_batched_results(gsi_batch_handle h, int32_t i, double* ritz, double* rho, int32_t* restarts);
/* Copy the basis of problem i (n x p float64 row-major) to the device pointer X_out. Syncs. */
gsi_status gsi_batched_get_x(gsi_batch_handle h, int32_t i, double* X_out);
/* Per-problem timeline of the last solve, read from the device wall clock, in microseconds
 * from the earliest start: start, switch to float64 (= start without a float32 phase) and
 * end; iters_low: iterations of the float32 phase; team: workgroups that worked on the
 * problem at the end (1 unless idle workgroups were recruited, see below). Host arrays of
 * count, each nullable. Syncs.
 *
 * Teams: once every problem has started, a running problem recruits idle workgroups by
 * the team policy of gsi_batched_set_tuning (by default every 32 iterations, up to 4 at a
 * time, up to 16 members with at least 16 row tiles of 64 rows each). The members split the tiles, add their partial
 * Grams and sums in member order and repeat the p x p work, so all hold the same state.
 * Float64 results of a problem that stayed with one workgroup repeat bit for bit; with a
 * team they depend on the team size, which depends on timing, and agree to rounding. */
gsi_status gsi_batched_timeline(gsi_batch_handle h, double* begin_us, double* switch_us, double* end_us,
                                int32_t* iters_low, int32_t* team);
/* Team policy of the following solves (defaults 16, 4, 32): a problem recruits idle
 * workgroups every check_every iterations, at most recruit_step at a time, up to one member
 * per tiles_per_member row tiles of 64 rows (and at most 16 members). tiles_per_member >= 4,
 * 1 <= recruit_step <= 15, check_every >= 1, else GSI_EINVAL. The values are what
 * paper_2306_10379_amd/tuning.py measures and picks per batch shape. Syncs. */
gsi_status gsi_batched_set_tuning(gsi_batch_handle h, int32_t tiles_per_member, int32_t recruit_step,
                                  int32_t check_every);
/* Per-problem tile shapes of the batched passes, the knobs the tuner
 * (paper_2306_10379_amd/tuning.py) picks per (size band, block width, precision): shapes is a
 * host array of count int32 codes with 4-bit fields, bits 0-3 u (row tiles whose loads are
 * issued together in the gradient, direction and product passes: 1, 2 or 4), bits 4-7 uu
 * (the retraction pass: 1 or 2), bits 8-11 ug (the Gram passes: 1, 2 or 4), bits 12-15 ch
 * (nonzeros whose indices and gathers are issued together in the SpMM: 4, 8, or 15 for 16);
 * a field 0 keeps the built default (all zero: the defaults everywhere). The shape changes
 * only the schedule of loads, not the arithmetic or its order: float64 results of a problem
 * solved by one workgroup repeat bit for bit under any shape. GSI_EINVAL for other codes
 * (nothing is changed then). Applies to the following solves. Syncs. */
gsi_status gsi_batched_set_shapes(gsi_batch_handle h, const int32_t* shapes);
/* Longest wait of a workgroup at a team barrier, or for a team entry it has reserved, in the
 * following solves (default 30 s; 0 < seconds <= 3600, else GSI_EINVAL). Every wait of the
 * persistent launch is bounded by it, so a team whose member never arrives ends the launch
 * with GSI_EDEVICE instead of holding the GPU. A very small limit forces that path from the
 * host, which is how the abort handling is tested. Syncs. */
gsi_status gsi_batched_set_wait_limit(gsi_batch_handle h, double seconds);
/* Per-problem time per pass of the last solve in microseconds: host array of count x
 * GSI_NPASS, entry [i * GSI_NPASS + GSI_PASS_*] (GSI_PASS_REFRESH also holds the Cholesky
 * QR of the start block and the first A X, GSI_PASS_SMALL the p x p work outside the
 * eigendecomposition and line search). Syncs. */
gsi_status gsi_batched_pass_times(gsi_batch_handle h, double* us);
const char* gsi_batched_last_error(gsi_batch_handle h);
void gsi_destroy_batched(gsi_batch_handle h);

#ifdef __cplusplus
}
#endif
#endif /* GSI_H */
