// Internal declarations shared by the HIP translation units of libchfsi.
// Not part of the public C ABI (that is include/chfsi.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <atomic>
#include <functional>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/chfsi.h"

struct chfsi_ctx;

namespace chfsi {

// roctx range over a phase of the solver (filter, Rayleigh-Ritz, CholQR,
// eigensolve, residual, bound estimate), visible with rocprofv3 --marker-trace
// and free when no tool is attached.
class TraceRange {
 public:
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// Memory source of a context (the server's pools): device and pinned host
// allocations; frees return memory to the source.  A context without one
// allocates with hipMalloc / hipHostMalloc.
struct Allocator {
  void* self = nullptr;
  void* (*dev_alloc)(void* self, size_t bytes) = nullptr;
  void (*dev_free)(void* self, void* p) = nullptr;
  void* (*host_alloc)(void* self, size_t bytes) = nullptr;
  void (*host_free)(void* self, void* p) = nullptr;
};
// chfsi_create with every allocation of the context drawn from `al`
// (chfsi_destroy returns it there).
chfsi_status create_with_allocator(chfsi_ctx** out, const chfsi_operator* A,
                                   const chfsi_operator* B, const double* d_inv,
                                   const chfsi_params* params, void* stream,
                                   const Allocator* al);

// Sets the calling thread's message returned by chfsi_last_error().
void set_error_message(const char* msg);

// ---------------------------------------------------------------------------
// GEMM: C(m,n) = epilogue( sum_k A(m,k) * B(k,n) )
//   A(m,k) = A[m*sam + k*sak]   (exactly one of sam, sak equals 1)
//   B(k,n) = B[k*sbk + n*sbn]   (exactly one of sbk, sbn equals 1)
//   optional kscale: B(k,n) is multiplied by kscale[k] as it is loaded
//   C is column-major: C(m,n) = C[m + n*ldc]
// Epilogue (all terms optional):
//   v = alpha * rowscale[m] * acc + beta * C1(m,n) + gamma * C2(m,n)
//       + delta * colscale3[n] * C3(m,n)
// C may alias C1, C2 or C3 (each element is read before it is written by the
// same thread).
// ---------------------------------------------------------------------------
template <typename T>
struct Epilogue {
  T alpha = T(1);
  const T* rowscale = nullptr;
  T beta = T(0);
  const T* C1 = nullptr;
  int64_t ldc1 = 0;
  T gamma = T(0);
  const T* C2 = nullptr;
  int64_t ldc2 = 0;
  T delta = T(0);
  const T* colscale3 = nullptr;
  const T* C3 = nullptr;
  int64_t ldc3 = 0;
};

template <typename T>
struct GemmDesc {
  int64_t M = 0, N = 0, K = 0;
  const T* A = nullptr;
  int64_t sam = 0, sak = 0;
  const T* B = nullptr;
  int64_t sbk = 0, sbn = 0;
  const T* kscale = nullptr;
  T* C = nullptr;
  int64_t ldc = 0;
  // batched problems (blockIdx decodes the batch index); only the plain
  // alpha/beta*C1 epilogue is supported when batch > 1
  int batch = 1;
  int64_t bsA = 0, bsB = 0, bsC = 0, bsC1 = 0;
  // symmetric result: only tiles that reach the diagonal or below are formed
  // (tiles strictly above it are left unwritten; mirror the lower part after)
  bool lower_only = false;
  Epilogue<T> epi;
  // optional: events recorded on the stream right before the first kernel and
  // right after the last one of the product (the tile kernel and, with split-K,
  // the reduction that carries the epilogue)
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
};

// Scratch the GEMM may use for deterministic split-K partial sums.
struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Launch a GEMM on `stream`.  `force_splits` > 0 pins the split-K factor
// (results then do not depend on the heuristic).  Returns hipSuccess or the
// first launch error.  Throws nothing.
template <typename T>
hipError_t gemm(const GemmDesc<T>& d, hipStream_t stream, const Workspace& ws,
                int force_splits = 0, int force_config = -1);

// Bytes of split-K scratch the heuristic may ask for at most for an M x N
// output with reduction length K (per batch entry).
size_t gemm_workspace_bytes(int64_t M, int64_t N, int64_t K, size_t elem);
// BF16 filter product: C = epilogue(A16 * bf16(kscale .* B)), A16 the
// k-contiguous bfloat16 copy of the operator (ld lda16), B FP32 k-contiguous;
// B16 (K x N bfloat16, ld K) receives the rounded right operand; FP32
// accumulation and epilogue.  Split-K partials need at most
// gemm_bf16_workspace_bytes(M, N) of ws.
// Chained steps (M == K): b16_ready says B16 already holds bfloat16(kscale .*
// B) and skips the rounding pass; with next16, the split-K reduction (when the
// product takes it) also writes next16 (M x N, ld M) = bfloat16(next_scale .*
// C) and sets *next_ready -- the next step's right operand, rounded from the
// values just formed.  next16 may be B16: the reduction runs after the product.
hipError_t gemm_bf16_filter(const GemmDesc<float>& d, const uint16_t* A16, int64_t lda16,
                            uint16_t* B16, hipStream_t st, const Workspace& ws,
                            int force_splits = 0, bool b16_ready = false,
                            uint16_t* next16 = nullptr, const float* next_scale = nullptr,
                            bool* next_ready = nullptr);
size_t gemm_bf16_workspace_bytes(int64_t M, int64_t N);
// split-K partial bytes the BF16 product will use for this shape (0: no split)
size_t gemm_bf16_plan_bytes(int64_t M, int64_t N, int64_t K, int force_splits);

// Which tile configuration/split the heuristic picks (for reports and tests).
template <typename T>
void gemm_plan(int64_t M, int64_t N, int64_t K, int batch, int* config, int* splits);

// ---------------------------------------------------------------------------
// Complex Hermitian layouts (complex.hip).  Interleaved complex data are
// (re, im) double pairs with leading dimensions in complex elements; planar
// blocks are n x 2b (real parts, then imaginary parts), ld n.
// ---------------------------------------------------------------------------
// L (n x 2n, row m at L + m*2n) = [Re A(:,m), -Im A(:,m)]: the left operand of
// the planar real product (F = float, double or uint16_t bfloat16)
template <typename F>
hipError_t herm_to_planar(const double* A, int64_t lda, int64_t n, F* L, hipStream_t st);
// out[0..n) = out[n..2n) = dinv (1 when null)
template <typename F>
hipError_t dup_dinv(const double* dinv, int64_t n, F* out, hipStream_t st);
// planar RY = scale * R, RX = 0, Yc = R from the interleaved residual
template <typename F>
hipError_t cplx_init(const double* R, int64_t ldr, int64_t n, int64_t b, double scale, F* RY,
                     F* RX, F* Yc, hipStream_t st);
// Zt (2n x 2b, ld 2n) = [[Z_r, Z_i], [-Z_i, Z_r]] from the planar Z
template <typename F>
hipError_t cplx_rhs(const F* Z, int64_t n, int64_t b, F* Zt, hipStream_t st);
// interleaved Yp = dinv .* RY + X diag(lamY)
template <typename F>
hipError_t cplx_reconstruct(const F* RY, const double* dinv, const double* X, int64_t ldx,
                            const double* lamY, double* Yp, int64_t ldy, int64_t n, int64_t b,
                            hipStream_t st);

// planar P (n x 2b, ld n) <-> interleaved Z (n x b, ld ldz)
hipError_t cplx_to_planar(const double* Z, int64_t ldz, int64_t n, int64_t b, double* P,
                          hipStream_t st);
hipError_t planar_to_cplx(const double* P, int64_t n, int64_t b, double* Z, int64_t ldz,
                          hipStream_t st);
// M (2b x 2b, ld 2b) = the real embedding [[G_r, -G_i], [G_i, G_r]] of the
// Hermitian G = Y^H W from the lower triangles of the four b x b blocks
// P11 = Y_r^T W_r, P22 = Y_i^T W_i, P12 = Y_r^T W_i, P21 = Y_i^T W_r of
// [Y_r Y_i]^T [W_r W_i] (consecutive in P4, ld b)
hipError_t embed_gram_lower(const double* P4, int64_t b, double* M, hipStream_t st);
// Zx (b x 2b planar, ld b): column j = T(0:b, 2j), column b+j = T(b:2b, 2j)
// for the first k eigenvalue pairs of the eigenvector matrix T (2b rows, ld
// ldt) of an embedded problem; columns k..b-1 of Zx are zero
hipError_t select_pairs_n(const double* T, int64_t ldt, int64_t b, int64_t k, double* Zx,
                          hipStream_t st);
// SVQB on the embedded Gram matrix: planar W (b x 2k) from the first vector of
// the eigenvalue pairs first, first + 2, ..., first + 2(k-1) of E (ld lde),
// column j scaled by gs[j] and row i by s[i] (device arrays)
hipError_t pairs_to_planar(const double* E, int64_t lde, int64_t b, int64_t first, int64_t k,
                           const double* gs, const double* s, double* W, hipStream_t st);
// Equal complex Ritz values: overwrite the 2 ncl columns of E (each [Re u;
// Im u], 2 cd rows, ld lde) with the pairs [Re q; Im q], [-Im q; Re q] of ncl
// G-orthonormal complex vectors q spanning the candidates, by pivoted
// Gram-Schmidt (one workgroup).  G: identity (Mg null) or G(i, j) = Mg(i, j)
// + i Mg(cd + i, j) (ld ldm).  *status (device): 0, or 1 if fewer than ncl
// independent directions exist (E then untouched).
size_t cluster_gs_work_bytes(int64_t cd, int64_t ncl);
hipError_t cluster_orthonormalize(double* E, int64_t lde, int64_t cd, int64_t ncl,
                                  const double* Mg, int64_t ldm, double* work, int* status,
                                  hipStream_t st);
// M(W) = [[W_r, -W_i], [W_i, W_r]] (2b x 2k, ld ldm) from planar W (b x 2k)
hipError_t embed_block(const double* W, int64_t b, int64_t k, double* M, int64_t ldm,
                       hipStream_t st);

// ---------------------------------------------------------------------------
// Bloch-phase grid operators in the twisted frame (bloch.hip).  D =
// diag(exp(i k.r)), r = (x, y, z) of grid point x + nx (y + ny z); planar
// blocks as above.
// ---------------------------------------------------------------------------
struct Twist {
  double kx, ky, kz;
  int64_t nx, ny;
};
// number of grid points with a neighbour across a periodic face
int64_t bloch_boundary_points(int nx, int ny, int nz);
// planar RY = scale D R, RX = 0, Yc = D R from the interleaved residual; E
// (may be null) receives RY's x = 0 and x = nx-1 values, ((z ny + y) 2 +
// (x == nx-1)) per column, ld 2 n / nx
template <typename F>
hipError_t bloch_init(const double* R, int64_t ldr, int64_t n, int64_t b, double scale, F* RY,
                      F* RX, F* Yc, const Twist& tw, hipStream_t st, F* E = nullptr);
// interleaved Yp = D^* (dinv .* RY) + X diag(lamY)
template <typename F>
hipError_t bloch_reconstruct(const F* RY, const double* dinv, const double* X, int64_t ldx,
                             const double* lamY, double* Yp, int64_t ldy, int64_t n, int64_t b,
                             const Twist& tw, hipStream_t st);
// planar P = D Z from interleaved Z, and interleaved Z = D^* P
hipError_t bloch_to_planar(const double* Z, int64_t ldz, int64_t n, int64_t b, double* P,
                           const Twist& tw, hipStream_t st);
hipError_t bloch_from_planar(const double* P, int64_t n, int64_t b, double* Z, int64_t ldz,
                             const Twist& tw, hipStream_t st);
// (the boundary correction kernels are declared with the grid kernels, stencil_api.h)

// ---------------------------------------------------------------------------
// Spectrum-bound estimates by a k-step Lanczos process on B^{-1} A in the
// B-inner product (lanczos.hip).  Vectors are FP64 of length L.
// ---------------------------------------------------------------------------
struct LanczosOps {
  std::function<hipError_t(const double*, double*)> apply_A;  // y = A x
  std::function<hipError_t(const double*, double*)> apply_B;  // y = B x; empty: B = I
  const double* dinv = nullptr;   // CG preconditioner (length L; null: none)
  const double* v0 = nullptr;     // start vector (device, length L)
  int steps = 12;
  double cg_tol = 1e-10;          // relative residual of the inner B-solves
  int cg_max_iter = 1000;
};
struct LanczosResult {
  int steps = 0, cg_iterations = 0;
  double theta_min = 0.0, theta_max = 0.0, beta_last = 0.0;
  double lower = 0.0, upper = 0.0;   // theta_min - |beta_k|, theta_max + |beta_k|
};
// device scratch for vectors of length L
size_t lanczos_workspace_bytes(int64_t L);
// y = A x, A dense symmetric n x n (ld), FP64; one wave per row
hipError_t gemv_rows_f64(const double* A, int64_t ld, int64_t n, const double* x, double* y,
                         hipStream_t st);
// host_scalars: pinned host memory for 8 doubles.  Synchronises the stream
// once per Lanczos step and once per batch of CG iterations.  Returns hipErrorInvalidValue if B is not positive
// definite on the Krylov space (a non-positive B-norm).
hipError_t lanczos_bounds(const LanczosOps& ops, int64_t L, double* work, double* host_scalars,
                          hipStream_t st, LanczosResult* res);

// ---------------------------------------------------------------------------
// Elementwise / reduction kernels (blas1.hip)
// ---------------------------------------------------------------------------
// out32[i,j] = (float)(s * in64[i,j]); optional second output copy32 = (float)in64
hipError_t rchfsi_init_f32(const double* R, int64_t ldr, int64_t n, int64_t b, double scale,
                           float* RY, float* RX, float* Ycopy, int64_t ld32, hipStream_t st);
hipError_t rchfsi_init_f64(const double* R, int64_t ldr, int64_t n, int64_t b, double scale,
                           double* RY, double* RX, int64_t ld, hipStream_t st);
// Per-column Lambda recurrence of the residual filter from the Ritz values
// (device, b): coefficient rows k - 2 = Lambda_Y before step k (FP64 table
// and/or FP32 table, each b per row, either may be null) and the final
// Lambda_Y in lamY.  e, c, sigma1 as in the filter's first line.
hipError_t rchfsi_coef(const double* ritz, int64_t b, double e, double c, double sigma1, int p,
                       double* coef64, float* coef32, double* lamY, hipStream_t st);
// Yp[i,j] = dinv[i] * RY[i,j] + X[i,j] * lamY[j]   (dinv may be null => 1)
hipError_t rchfsi_reconstruct_f32(const float* RY, int64_t ldry, const double* dinv,
                                  const double* X, int64_t ldx, const double* lamY, double* Yp,
                                  int64_t ldy, int64_t n, int64_t b, hipStream_t st);
hipError_t rchfsi_reconstruct_f64(const double* RY, int64_t ldry, const double* dinv,
                                  const double* X, int64_t ldx, const double* lamY, double* Yp,
                                  int64_t ldy, int64_t n, int64_t b, hipStream_t st);
// column 2-norms of an n x b FP64 block, deterministic order
hipError_t column_norms(const double* R, int64_t ldr, int64_t n, int64_t b, double* out,
                        hipStream_t st);
// FP64 -> FP32 copy of an n x m column-major matrix
hipError_t convert_f64_f32(const double* in, int64_t ldi, float* out, int64_t ldo, int64_t n,
                           int64_t m, hipStream_t st);
hipError_t convert_f64_bf16(const double* in, int64_t ldi, uint16_t* out, int64_t ldo, int64_t n,
                            int64_t m, hipStream_t st);
// copy an n x b block between leading dimensions
hipError_t copy_block(const double* in, int64_t ldi, double* out, int64_t ldo, int64_t n,
                      int64_t b, hipStream_t st);
// B <- diag(s) A diag(s) with s = 1/sqrt(diag(G)); writes s
hipError_t scale_gram(const double* G, int64_t ldg, int64_t b, double* Gs, int64_t lds,
                      double* s, int* bad_flag, hipStream_t st);
hipError_t scale_sym(const double* G, int64_t ldg, int64_t b, const double* s, double* out,
                     int64_t ldo, hipStream_t st);
// out = 0.5 (A + A^T) in place on a b x b matrix
hipError_t symmetrize(double* A, int64_t lda, int64_t b, hipStream_t st);
// completes a symmetric matrix of which the lower block panels of width w were
// formed (w = 1: copies the strictly lower part to the upper part)
hipError_t symmetrize_panels(double* A, int64_t lda, int64_t b, int64_t w, hipStream_t st);
// columns of M scaled by v: M[:,j] *= v[j]
hipError_t scale_columns(double* M, int64_t ldm, int64_t n, int64_t b, const double* v,
                         hipStream_t st);
// rows of M scaled by v: M[i,:] *= v[i]
hipError_t scale_rows(double* M, int64_t ldm, int64_t n, int64_t b, const double* v,
                      hipStream_t st);
hipError_t set_identity(double* M, int64_t ldm, int64_t n, hipStream_t st);
hipError_t fill_zero(void* p, size_t bytes, hipStream_t st);
// random N(0,1) block from a counter-based generator (Philox-4x32-10 + Box-Muller)
hipError_t fill_gaussian(double* X, int64_t ldx, int64_t n, int64_t b, uint64_t seed,
                         hipStream_t st);
// any NaN/Inf in a vector -> *flag = 1
hipError_t check_finite(const double* v, int64_t n, int* flag, hipStream_t st);

// ---------------------------------------------------------------------------
// Small dense FP64 linear algebra (dense_small.hip)
// ---------------------------------------------------------------------------
// In-place lower Cholesky of a b x b SPD matrix (upper part zeroed). Sets
// *info = j+1 at the first non-positive pivot (0 on success).
// scratch of potrf_lower / trsm_lower_left: inverses of the diagonal blocks
// and one block row or column of temporaries
size_t tri_workspace_bytes(int64_t b, int64_t nrhs);
// lower Cholesky factor in place (upper part zeroed); info: first pivot
// (1-based) that is not above piv_tol (or not finite), or 0
hipError_t potrf_lower(double* A, int64_t lda, int64_t b, int* info, hipStream_t st,
                       const Workspace& ws, double* tri, double piv_tol = 0.0);
// X <- L^{-1} X (L lower b x b, X b x nrhs); inverses_ready: tri holds the
// diagonal blocks' inverses of this L (left by potrf_lower)
hipError_t trsm_lower_left(const double* L, int64_t ldl, double* X, int64_t ldx, int64_t b,
                           int64_t nrhs, hipStream_t st, const Workspace& ws, double* tri,
                           bool inverses_ready);
// Symmetric eigensolver (parallel block Jacobi).  A (b x b) is destroyed.
// w: ascending eigenvalues (device, b); V: eigenvectors (device, b x b, ldv).
// scratch from ws; sweeps reported through *sweeps_out (host) if non-null;
// *unconverged_out (host, if non-null) = 1 when the sweep cap was reached with
// rotations still being applied (the result is then not fully diagonalised).
// pinned_flags (two ints of pinned host memory) and ev (an event of the
// stream's device): optional; with both, the next sweep's first launches are
// queued before each convergence read-back
hipError_t syev_jacobi(double* A, int64_t lda, int64_t b, double* w, double* V, int64_t ldv,
                       hipStream_t st, const Workspace& ws, int* sweeps_out,
                       int* unconverged_out = nullptr, int* pinned_flags = nullptr,
                       hipEvent_t ev = nullptr);
size_t syev_workspace_bytes(int64_t b);
size_t potrf_workspace_bytes(int64_t b);

// ---------------------------------------------------------------------------
// 27-point periodic stencil operators (stencil.hip)
// ---------------------------------------------------------------------------
struct StencilOp {
  int nx = 0, ny = 0, nz = 0;
  double coef[27];        // S1 coefficients, index (dz+1)*9 + (dy+1)*3 + (dx+1)
  double coefM[27];       // mass coefficients used by the field term
  const double* field = nullptr;  // V (length n) or null
  int field_mode = 0;     // 0 none, 1 lumped diag(V), 2 mass weighted 1/2(VM + MV)
};

// Cooperative cancellation used by the serving scheduler: chfsi_solve checks
// *flag before every outer iteration and returns CHFSI_ERR_CANCELLED once set.
void ctx_set_cancel_flag(chfsi_ctx* c, const std::atomic<int>* flag);

}  // namespace chfsi
