/*
 * chfsi.h -- C ABI of libchfsi: residual-based Chebyshev filtered subspace
 * iteration (R-ChFSI) for the lowest eigenpairs of a symmetric-definite pencil
 *
 *        A u = lambda B u,   A symmetric, B symmetric positive definite
 *
 * (Kodali, Ramakrishnan, Motamarri, arXiv 2503.22652, Section 2, eq. ghep),
 * on one AMD Instinct MI355X (gfx950).
 *
 * Conventions for every call:
 *  - "device" pointers are HIP device memory on the context's device; "host"
 *    pointers are ordinary host memory.  Nothing in this header takes a
 *    framework (e.g. PyTorch) type; a stream is passed as `void*` and is a
 *    hipStream_t (NULL = the default stream).
 *  - Blocks of vectors are column-major, N rows, leading dimension ld >= N
 *    (the LAPACK convention).  Dense operators are column-major N x N with
 *    leading dimension ld >= N and must be symmetric.
 *  - Functions return a chfsi_status and never throw.  On error, output
 *    buffers are left untouched except where a function says otherwise, and a
 *    message is available from chfsi_last_error() (thread-local).
 *  - Complex Hermitian problems (the paper's Section 4.3): an operator of
 *    kind CHFSI_OP_DENSE_HERMITIAN or CHFSI_OP_STENCIL27_BLOCH makes a
 *    complex context.  Its blocks
 *    (X, resid, Yp of chfsi_filter) are interleaved complex -- (re, im) pairs
 *    of doubles, column-major, leading dimensions counted in complex
 *    elements -- while Ritz values and d_inv stay real.  Such a context runs
 *    the residual filter (Algorithm 3) in FP64, FP32 or BF16 and an FP64
 *    Rayleigh-Ritz on the real embedding [[G_r, -G_i], [G_i, G_r]] of the
 *    projected Hermitian pencil.  A singular Gram matrix takes the SVQB
 *    fallback of real blocks on the embedding, keeping and refilling whole
 *    complex directions (chfsi_report.flags bit 0).  Equal Ritz values get
 *    a B-orthonormal basis of their eigenspace.
 */
#ifndef CHFSI_H_
#define CHFSI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CHFSI_OK = 0,
  CHFSI_ERR_ARG = 1,        /* invalid argument (message says which) */
  CHFSI_ERR_NOMEM = 2,      /* device allocation failed */
  CHFSI_ERR_DEVICE = 3,     /* HIP runtime / kernel launch error */
  CHFSI_ERR_NOT_SPD = 4,    /* B (or the Gram matrix Y^T B Y) is not positive definite */
  CHFSI_ERR_NOCONV = 5,     /* max_iter reached; best pairs so far are returned */
  CHFSI_ERR_NUMERIC = 6,    /* NaN/Inf met in Ritz values or residual norms */
  CHFSI_ERR_BUSY = 7,       /* server queue full / admission refused */
  CHFSI_ERR_CANCELLED = 8,  /* request was cancelled */
  CHFSI_ERR_TIMEOUT = 9     /* chfsi_wait timed out; the request is still live */
} chfsi_status;

/* Operator kinds. */
typedef enum {
  CHFSI_OP_IDENTITY = 0,        /* B = I (standard problem) */
  CHFSI_OP_DENSE = 1,           /* dense symmetric matrix in device memory */
  CHFSI_OP_STENCIL27 = 2,       /* periodic 27-point grid operator (see chfsi_operator) */
  CHFSI_OP_DENSE_HERMITIAN = 3, /* dense complex Hermitian matrix (Section 4.3; see below) */
  CHFSI_OP_STENCIL27_BLOCH = 4, /* grid operator with Bloch phases, complex (Section 4.3) */
  CHFSI_OP_CSR = 5              /* sparse symmetric matrix in CSR form (see chfsi_operator) */
} chfsi_op_kind;

/* Storage / arithmetic precision of the filter's bulk work (the residual
 * filter's reduced-precision product of Section 3.2).  FP32: blocks and the
 * operator copy are FP32 and products accumulate in FP32 on MFMA.  BF16,
 * stencil operators: filter blocks are stored in bfloat16 and all arithmetic
 * is FP32.  BF16, dense operators (residual filter only): the product's
 * inputs -- an owned bfloat16 copy of A and D^{-1} R_Y, both rounded to
 * nearest-even -- run on bfloat16 MFMA with FP32 accumulation; the filter
 * blocks and the three-term update stay FP32.  The Rayleigh-Ritz step,
 * reconstruction and residual norms are always FP64. */
typedef enum { CHFSI_PREC_FP64 = 0, CHFSI_PREC_FP32 = 1, CHFSI_PREC_BF16 = 2 } chfsi_prec;

/* Filter algorithm: Algorithm 2 (three-term recurrence on the block, with
 * H = D^{-1} A) or Algorithm 3 (residual-based recurrence). */
typedef enum { CHFSI_METHOD_CHFSI = 0, CHFSI_METHOD_RCHFSI = 1 } chfsi_method;

/*
 * A symmetric operator.
 *  kind = CHFSI_OP_DENSE: `dense` (device, n x n, column-major, leading
 *    dimension `ld`, symmetric; borrowed: must outlive the context).
 *  kind = CHFSI_OP_DENSE_HERMITIAN: `dense` (device) holds an n x n complex
 *    Hermitian matrix, interleaved (entry (i, j) at dense[2 (i + j ld)] and
 *    dense[2 (i + j ld) + 1]), `ld` in complex elements; borrowed.  With a
 *    Hermitian A, B is NULL / the identity or Hermitian dense of A's size,
 *    params.method must be CHFSI_METHOD_RCHFSI and params.memory_mode 0.  The
 *    context keeps a planar copy [Re A | Im A] in the filter precision (2 n^2
 *    elements) and runs each recurrence step as one real MFMA product of
 *    2n x 2b operands (Section 4.3's complex product, 8 n^2 b flops).
 *  kind = CHFSI_OP_STENCIL27: periodic grid nx*ny*nz = n, vector index
 *    x + nx*(y + ny*z).  y = S z + potential term, where S has coefficients
 *    coef[(dz+1)*9 + (dy+1)*3 + (dx+1)] for the 27 offsets (dx,dy,dz) in
 *    {-1,0,1}^3.  field_mode 0: no potential; 1: diag(V) z; 2: the
 *    mass-weighted 1/2 (diag(V) M + M diag(V)) z with M given by coef_mass.
 *    `field` (device, length n) holds V; borrowed.
 *  kind = CHFSI_OP_STENCIL27_BLOCH: the grid operator above on cell-periodic
 *    complex vectors at wave vector k = (bloch[0], bloch[1], bloch[2]) (kx,
 *    ky, kz in radians per grid step): the coefficient of offset (dx,dy,dz)
 *    is multiplied by exp(i (kx dx + ky dy + kz dz)), in S and in the mass
 *    stencil of field_mode 2 alike; field_mode 1 is unchanged.  The result
 *    is Hermitian (the k-point problems of Section 4.3 on a grid).  It makes
 *    a complex context like CHFSI_OP_DENSE_HERMITIAN (interleaved blocks,
 *    the residual filter only, memory_mode 0, FP64/FP32/BF16 filter); B is
 *    NULL / the identity or of this kind on A's grid with the same k and
 *    field_mode 0; block <= 65535.  The context runs in the frame twisted
 *    by D = diag(exp(i k.r)): the real z-marching kernels on the planar real
 *    and imaginary parts plus a correction at the boundary points for the
 *    phase of wrapped neighbours.  bloch[] is ignored for other kinds.
 *  kind = CHFSI_OP_CSR: a real symmetric n x n matrix (the sparse
 *    finite-element operators of Section 4.2) in compressed sparse row form,
 *    device arrays, borrowed: rowptr (int64, n + 1 entries, rowptr[0] = 0,
 *    non-decreasing, rowptr[n] = nnz), colind (int32, nnz entries in
 *    [0, n)), val (double, nnz entries).  Both triangles are stored; the
 *    library does not check symmetry.  chfsi_create checks the structure
 *    (CHFSI_ERR_ARG if invalid), keeps an FP32 copy of val for FP32 / BF16
 *    filters and requires n < 2^31 and memory_mode 0.  B may be NULL / the
 *    identity, CSR or dense of A's size.  The filter's products run in the
 *    context's filter precision (FP64, FP32, or BF16-stored blocks with FP32
 *    arithmetic).
 */
typedef struct {
  int32_t kind;
  int64_t n;
  const double* dense;
  int64_t ld;
  int32_t nx, ny, nz;
  double coef[27];
  double coef_mass[27];
  const double* field;
  int32_t field_mode;
  double bloch[3];
  const int64_t* rowptr;   /* CHFSI_OP_CSR */
  const int32_t* colind;
  const double* val;
  int64_t nnz;
} chfsi_operator;

/* Solver parameters (Algorithm 1 inputs: n, p, bounds, tau). */
typedef struct {
  int64_t n_wanted;     /* number of wanted eigenpairs n (stopping test uses j < n) */
  int64_t block;        /* block size b >= n (columns filtered per iteration) */
  int32_t degree;       /* Chebyshev degree p >= 1 */
  int32_t max_iter;     /* outer iterations of Algorithm 1 */
  double tol;           /* tau: stop when max_{j<n} ||A x_j - eps_j B x_j||_2 < tau */
  int32_t method;       /* chfsi_method */
  int32_t filter_prec;  /* chfsi_prec */
  /* Filter bounds (Section 2.1: estimates).  lambda_max: an upper bound of
   * the spectrum of B^{-1}A, or NaN: chfsi_solve then estimates it once per
   * context with chfsi_estimate_bounds (lanczos_steps steps from an N(0,1)
   * start of seed `seed`) and uses its `upper`.  lambda_min / lambda_T may be
   * NaN: then each iteration uses lambda_T = largest Ritz value of the block
   * and lambda_min = eps_1 - 0.05 (eps_b - eps_1).  Infinite values are
   * rejected. */
  double lambda_min, lambda_max, lambda_T;
  uint64_t seed;        /* seed of the random start block when init_random != 0 */
  int32_t init_random;  /* chfsi_solve: 1 = fill X with N(0,1) (Philox-4x32-10), 0 = X holds the start */
  int32_t profile;      /* 1 = time every filter operator-product kernel with HIP events */
  /* 0: Rayleigh-Ritz keeps A Y and B Y as full n x b FP64 blocks.
   * 1: slab-wise Rayleigh-Ritz for stencil operators with tensor-product
   *    coefficients and the residual filter: Gram matrices are accumulated over
   *    z-slabs, the rotation X = Y E is done slab by slab in place and the
   *    residual in one fused stencil pass, so the context holds only the
   *    residual block, the filter blocks and two slabs (chfsi_solve then works
   *    in the caller's X). */
  int32_t memory_mode;
  /* 1: the plain filter (CHFSI_METHOD_CHFSI, FP64) uses the exact inverse,
   * H = B^{-1} A (Algorithm 2 with the generalized problem's own operator),
   * for dense A and dense B.  chfsi_create forms H once from the Cholesky
   * factor of B (B = L L^T, B^{-1} = L^{-T} L^{-1}, kept as A B^{-1} = H^T)
   * and owns it (n^2 doubles); d_inv is not used by the filter then.
   * 0: H = D^{-1} A. */
  int32_t binv_exact;
  /* Lanczos steps of the lambda_max estimate (0: 12). */
  int32_t lanczos_steps;
  /* Stagnation: chfsi_solve stops with CHFSI_ERR_NOCONV once the lowest max
   * residual so far has not halved for stall_iters consecutive iterations
   * (0: run to max_iter). */
  int32_t stall_iters;
  /* 1: keep a copy of the Ritz block of the lowest max residual (one more
   * n x b FP64 block, allocated by chfsi_create) and return those pairs on
   * CHFSI_ERR_NOCONV; 0: return the last pairs. */
  int32_t keep_best;
  /* 1: precision escalation for a BF16 filter on a real operator (dense,
   * grid or CSR): when the max residual stagnates for stall_iters passes
   * (which must be > 0), the remaining passes filter in FP32 (FP32 blocks;
   * dense: FP32 products) instead of stopping (report flags bit 3,
   * escalation_iteration).  A reduced-precision filter has a largest usable
   * degree (Section 3.1's condition); past it the BF16 iteration stalls.  The
   * context then holds FP32 filter blocks from the start (dense: also an FP32
   * copy of A), as an FP32 context does. */
  int32_t escalate;
  /* Amplification guard.  A pass filters the unwanted end of the spectrum by
   * up to T_p(|L(lambda_min)|) relative to the damped interval (L maps
   * [lambda_T, lambda_max] onto [-1, 1]); rounding in a reduced-precision
   * filter is amplified by that much (Section 3.1's condition), and past
   * ~1e12 a pass is likely to lose the wanted columns' accuracy.  Every pass
   * reports it (report max_amplification; flags bit 4 when it exceeds 1e12).
   * amp_cap > 0 caps it: a pass then filters at the largest degree
   * p' <= degree with T_p'(|L(lambda_min)|) <= amp_cap (at least 1; flags
   * bit 5, report min_degree_used).  0: no cap. */
  double amp_cap;
} chfsi_params;

/* Per-solve report (host). */
#define CHFSI_MAX_HISTORY 512
typedef struct {
  int32_t iterations;          /* filter + Rayleigh-Ritz passes performed */
  int32_t converged;           /* 1 if max residual < tol */
  double max_residual;         /* final max_{j<n} r_j */
  double time_total_ms;        /* wall time of chfsi_solve (device-synchronous) */
  double time_filter_ms;       /* sum of filter times (HIP events) */
  double time_rr_ms;           /* sum of Rayleigh-Ritz + residual times (HIP events) */
  double filter_flops;         /* algorithmic flops of all filter products */
  int32_t jacobi_sweeps;       /* sum of eigensolver sweeps */
  int32_t kernel_launches;     /* profile: filter operator-product kernels timed */
  double kernel_ms;            /* profile: their summed durations (HIP events) */
  int32_t flags;               /* bit 0: a Gram matrix took the SVQB fallback;
                                  bit 1: a Jacobi eigensolve reached its cap of 40 sweeps
                                  with rotations still applied (not fully diagonalised);
                                  bit 2: the solve stopped on stagnation (stall_iters);
                                  bit 3: the filter precision was escalated to FP32;
                                  bit 4: a pass's amplification T_p(|L(lambda_min)|)
                                  exceeded 1e12;
                                  bit 5: amp_cap lowered a pass's degree */
  double history[CHFSI_MAX_HISTORY]; /* max residual after each pass (entry 0: initial RR) */
  int32_t svqb_events;         /* Rayleigh-Ritz passes that took the SVQB fallback */
  int32_t svqb_dropped;        /* directions dropped (and refilled) by those passes, summed */
  double lambda_max_used;      /* the filter's upper bound (given, or the Lanczos estimate) */
  double time_bounds_ms;       /* time of the Lanczos estimate in this solve (0 if none) */
  int32_t best_iteration;      /* pass with the lowest max residual (0: initial RR) */
  double best_residual;        /* that lowest max residual */
  int32_t escalation_iteration;/* params.escalate: pass after which FP32 took over (0: none) */
  double max_amplification;    /* largest T_p(|L(lambda_min)|) of the passes, at the degree used */
  int32_t min_degree_used;     /* smallest filter degree of the passes (params.degree unless
                                  amp_cap lowered it; 0 if no pass ran) */
} chfsi_report;

typedef struct chfsi_ctx chfsi_ctx;

/*
 * Create a solver context for the pencil (A, B) with approximate inverse
 * D^{-1} = diag(d_inv) of B (paper Section 3.2: D^{-1} replaces B^{-1} in the
 * filter only).  B == NULL or B->kind == CHFSI_OP_IDENTITY means B = I.
 * d_inv: device, length n, or NULL for D^{-1} = I.
 * The context borrows A, B and d_inv (they must outlive it) and owns every
 * workspace and precision-converted copy it makes (all allocated here, once;
 * chfsi_workspace_bytes() reports the size).  stream: hipStream_t or NULL.
 * Errors: CHFSI_ERR_ARG (inconsistent sizes/kinds/params), CHFSI_ERR_NOMEM,
 * CHFSI_ERR_DEVICE.
 */
chfsi_status chfsi_create(chfsi_ctx** out, const chfsi_operator* A, const chfsi_operator* B,
                          const double* d_inv, const chfsi_params* params, void* stream);

/* Device bytes chfsi_create would allocate for these arguments (0 on invalid input). */
size_t chfsi_workspace_bytes(const chfsi_operator* A, const chfsi_operator* B,
                             const chfsi_params* params);

/*
 * One Chebyshev filter pass, stream-ordered and asynchronous.
 * method CHFSI (Algorithm 2): Yp = C_p(D^{-1} A) X; ritz and resid ignored.
 * method RCHFSI (Algorithm 3): inputs X (Ritz vectors), ritz (host, b Ritz
 *   values Lambda^(i)) and resid (device, Y = A X - B X Lambda^(i)); output
 *   Yp = D^{-1} R_Y + X Lambda_Y after `degree` steps of the residual
 *   recurrence (eq. rChFSIrecurrenceMP), computed in the context's
 *   filter precision.
 * X, resid: device, n x b (ld >= n).  Yp: device, n x b; may alias X.
 * lmin, lmax, lT: the filter bounds (Section 2.1); lmin < lT < lmax.
 * degree: p >= 1 (0 means the context's degree).
 */
chfsi_status chfsi_filter(chfsi_ctx* ctx, const double* X, int64_t ldx, const double* ritz,
                          const double* resid, int64_t ldr, double* Yp, int64_t ldy, double lmin,
                          double lmax, double lT, int32_t degree);

/*
 * Rayleigh-Ritz on a filtered block (Algorithm 1, steps 2-3) and residuals.
 * Solves (Y^T A Y) E = (Y^T B Y) E Lambda through the Cholesky factor of the
 * column-scaled Gram matrix (CholQR) and a Jacobi eigensolver, then writes
 * X = Y E (B-orthonormal Ritz vectors, ascending Ritz values), R = A X - B X
 * Lambda and r_j = ||R_j||_2.  Y, X, R: device n x b; X must not alias Y.
 * ritz, resnorm: host, length b.  Synchronises the stream once.
 * A numerically singular Gram matrix takes the SVQB fallback: the directions
 * above 1e-14 of its largest eigenvalue are kept, the others refilled with
 * N(0,1) values, and Rayleigh-Ritz repeated once (chfsi_report.flags bit 0).
 * Errors: CHFSI_ERR_NOT_SPD if the Gram matrix has a zero or non-finite
 * column, or is not positive definite after the refill; CHFSI_ERR_NUMERIC on
 * NaN/Inf.
 */
chfsi_status chfsi_rayleigh_ritz(chfsi_ctx* ctx, const double* Y, int64_t ldy, double* X,
                                 int64_t ldx, double* R, int64_t ldr, double* ritz,
                                 double* resnorm);

/*
 * Estimates of the spectrum bounds of B^{-1} A (Section 2.1 treats the
 * filter's bounds as estimates).  A k-step Lanczos process on B^{-1} A in the
 * B-inner product from v0 (each step: one product with A and a
 * preconditioned conjugate-gradient solve with B to relative residual 1e-10,
 * preconditioner D^{-1}; no solve when B = I), in FP64 on the device.  With
 * theta_1 <= theta_k the extreme eigenvalues of the k x k tridiagonal matrix
 * and beta_k the B-norm of the last Lanczos residual (the "Ritz value +
 * |beta_k|" safeguard of Zhou, Saad, Tiago and Chelikowsky, J. Comput. Phys.
 * 219 (2006)): *upper = theta_k + |beta_k|, *lower = theta_1 - |beta_k|.
 * v0: device, length n (interleaved complex for a complex context), or NULL
 * for N(0,1) values (Philox-4x32-10, seed params.seed).  steps: k >= 1 (0 =
 * params.lanczos_steps or 12); fewer steps are taken if the Krylov space is
 * exhausted.  theta: optional host array of 2 (theta_1, theta_k).  The first
 * call on a context allocates its Lanczos vectors (12 n doubles, complex: 24
 * n) unless chfsi_create did (lambda_max = NaN).  Synchronises the stream.
 * Errors: CHFSI_ERR_ARG, CHFSI_ERR_NOMEM, CHFSI_ERR_NOT_SPD (B not positive
 * definite on the Krylov space), CHFSI_ERR_DEVICE.
 */
chfsi_status chfsi_estimate_bounds(chfsi_ctx* ctx, const double* v0, int32_t steps,
                                   double* lower, double* upper, double* theta);

/*
 * Full eigensolve (Algorithm 1 with the context's filter).  X (device, n x b,
 * ld >= n): on entry the start block (or overwritten with N(0,1) values when
 * params.init_random), on exit the Ritz vectors.  evals, resnorms: host,
 * length b (ascending Ritz values and their residual norms).  rep: optional.
 * Returns CHFSI_OK on convergence, CHFSI_ERR_NOCONV after max_iter passes or
 * on stagnation (params.stall_iters; report flags bit 2); the outputs then hold
 * the pairs of the lowest max residual when params.keep_best, else the last
 * pairs (as LAPACK's INFO > 0).  Other errors as above.
 */
chfsi_status chfsi_solve(chfsi_ctx* ctx, double* X, int64_t ldx, double* evals, double* resnorms,
                         chfsi_report* rep);

/*
 * Profiling (params.profile = 1): total duration (ms, HIP events recorded on
 * the context's stream immediately around each step) and count of the
 * filter's recurrence steps -- every kernel of the step's fused operator
 * product: the GEMM with its split-K reduction (which carries the three-term
 * epilogue), the BF16 product's operand rounding, or the stencil kernel --
 * since the previous call.
 * Synchronises the stream.  Returns CHFSI_ERR_ARG when profiling is off.
 */
chfsi_status chfsi_filter_kernel_time(chfsi_ctx* ctx, double* total_ms, int32_t* launches);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * residual filter of chfsi_filter (method CHFSI_METHOD_RCHFSI, filter_prec
 * CHFSI_PREC_FP64) without a context and without any allocation.
 *
 * A: CHFSI_OP_DENSE (device, symmetric, ld >= n) or CHFSI_OP_STENCIL27
 *    (any field_mode), borrowed for the call.  d_inv: device, length n, or
 *    NULL for D^{-1} = I.  b: number of columns (b = 0: only binds the
 *    scratch array on the current device and returns; do this once before a
 *    stream capture).  X, resid (Y = A X - B X Lambda), Yp: device, n x b,
 *    column-major (ld >= n); Yp may alias X.  ritz: DEVICE array of the b
 *    Ritz values (unlike chfsi_filter, so that the call records no host
 *    copy).  lmin < lT < lmax, degree p >= 1, stream: as chfsi_filter.
 *    Result: Yp = D^{-1} R_Y + X diag(Lambda_Y) after p - 1 steps, computed by
 *    the same kernels as chfsi_filter with an FP64 context.
 *
 * Every intermediate (the Lambda_Y table, R_X, R_Y, split-K partial sums)
 * lives in one static device array of CHFSI_STATIC_SCRATCH_BYTES per GPU,
 * held from its first use on that GPU until the process ends.  The
 * call needs chfsi_filter_static_bytes(n, b, degree) of it and returns
 * CHFSI_ERR_ARG, with a message, when that exceeds the maximum; split-K
 * partials use what is left (fewer or no k-splits when little is).  The call
 * makes no hipMalloc / hipFree or other allocating call; it is
 * stream-ordered and asynchronous.  All calls on one GPU share the array:
 * calls that overlap in time on one GPU (different streams or threads
 * without ordering) race and give undefined results.
 * Errors: CHFSI_ERR_ARG, CHFSI_ERR_DEVICE.
 */
#define CHFSI_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
size_t chfsi_filter_static_bytes(int64_t n, int64_t b, int32_t degree);
chfsi_status chfsi_filter_static(const chfsi_operator* A, const double* d_inv, int64_t b,
                                 const double* X, int64_t ldx, const double* ritz,
                                 const double* resid, int64_t ldr, double* Yp, int64_t ldy,
                                 double lmin, double lmax, double lT, int32_t degree,
                                 void* stream);

/* Release the context and everything it owns (borrowed arrays untouched). */
void chfsi_destroy(chfsi_ctx* ctx);

/* Message of the last error on the calling thread ("" if none). */
const char* chfsi_last_error(void);

/* Library version string. */
const char* chfsi_version(void);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of eigensolves on one GPU.
 *
 * A server owns a scheduler thread and up to `slots` concurrent solves, each
 * on its own HIP stream.  Requests that arrive while others run are admitted
 * as soon as a slot is free and the request's workspace (chfsi_workspace_bytes)
 * fits in the device-memory budget; their kernels then overlap on the device.
 * Requests of one sequence (same seq_id) run in submission order, and the
 * server keeps the sequence's last Ritz vectors on the device to warm-start
 * the next one (the evolving-matrix setting of the paper's introduction).
 * Every request runs exactly the same kernels with the same launch shapes
 * whether it runs alone or mixed with others, so results are bitwise equal.
 * ------------------------------------------------------------------------- */
typedef struct chfsi_server chfsi_server;

typedef struct {
  int32_t slots;            /* concurrent solves (>= 1) */
  int32_t queue_capacity;   /* pending requests before chfsi_submit returns BUSY */
  size_t memory_budget;     /* device bytes for workspaces; 0 = 90% of free memory */
} chfsi_server_config;

typedef struct {
  chfsi_operator A;         /* borrowed device arrays: must stay valid until completion */
  chfsi_operator B;         /* kind CHFSI_OP_IDENTITY for a standard problem */
  const double* d_inv;      /* device length n, or NULL */
  chfsi_params params;
  int64_t seq_id;           /* sequence id for warm starts; < 0: independent request */
  const double* X0;         /* device n x b start block (ld n) when the sequence has none;
                               NULL: random start from params.seed; interleaved complex
                               (2 n b doubles) for a complex A */
  double* X_out;            /* optional device n x b (ld n) output of the Ritz vectors,
                               interleaved complex for a complex A */
} chfsi_request;

typedef struct {
  chfsi_status status;
  int32_t iterations;
  double max_residual;
  double submit_ms, start_ms, finish_ms;   /* server-clock timestamps */
  int64_t n, block;
  double* evals;            /* host array of `block` Ritz values, owned by the result */
  double* resnorms;         /* host array of `block` residual norms, owned by the result */
} chfsi_result;

chfsi_status chfsi_server_create(chfsi_server** out, const chfsi_server_config* cfg);
/* Thread-safe and non-blocking: enqueue a request, return its ticket. */
chfsi_status chfsi_submit(chfsi_server* s, const chfsi_request* req, uint64_t* ticket);
/* Block until the request finishes (timeout_ms < 0: forever).  On success the
 * result is moved into *res (free it with chfsi_result_free). */
chfsi_status chfsi_wait(chfsi_server* s, uint64_t ticket, int32_t timeout_ms, chfsi_result* res);
/* Cancel a pending request (a running one finishes its current pass first). */
chfsi_status chfsi_cancel(chfsi_server* s, uint64_t ticket);
void chfsi_result_free(chfsi_result* res);
/* Server memory.  Every context, working block and warm-start block of the
 * server's requests is drawn from two pools (device memory, pinned host
 * memory) that grow by whole chunks (hipMalloc / hipHostMalloc) only when no
 * free range fits, and that are released only by chfsi_server_destroy, so a
 * server in steady state allocates and frees nothing per request (hipFree
 * would synchronise the whole device).  The budget charges a running request
 * its workspace plus working block, and each sequence its warm-start block
 * from allocation to replacement or server destruction. */
typedef struct {
  size_t budget;             /* device bytes admission may charge */
  size_t used;               /* charged now: running requests + warm-start blocks */
  size_t sequence_bytes;     /* of which warm-start blocks of live sequences */
  int32_t device_pool_chunks;/* hipMalloc calls made by the device pool so far */
  int32_t host_pool_chunks;  /* hipHostMalloc calls made by the pinned pool so far */
} chfsi_server_stats_t;
chfsi_status chfsi_server_stats(chfsi_server* s, chfsi_server_stats_t* out);

/* Drain running requests and stop the scheduler. */
void chfsi_server_destroy(chfsi_server* s);

#ifdef __cplusplus
}
#endif

#endif /* CHFSI_H_ */
