// Host driver and C ABI of libchfsi (see include/chfsi.h).
//
// Implements Algorithm 1 (outer subspace iteration), Algorithm 2 (Chebyshev
// filter) and Algorithm 3 (residual-based Chebyshev filter) of
// arXiv 2503.22652 on one GPU.  Every numerical step runs in the HIP kernels of
// this library; the host only sequences launches, computes the O(b)
// recurrence scalars of the filter (Section 2.1, eq. ChFSIrecurrence; the
// diagonal recurrence eq. ChFSIrecurrenceEigval) and reads back b Ritz values
// and residual norms once per outer iteration.
#include "../../include/chfsi.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "stencil_api.h"

using namespace chfsi;

namespace {

// The CholQR factorisation of a column-scaled (unit-diagonal) Gram matrix
// under a roctx range.  A pivot at or below the SVQB drop tolerance 1e-14 counts
// as a breakdown: the smallest eigenvalue is then below 1e-14 times the largest
// (which is at least 1), so the SVQB reading would drop a direction.
constexpr double kGramPivotTol = 1e-14;
hipError_t potrf_traced(double* A, int64_t lda, int64_t b, int* info, hipStream_t st,
                        const Workspace& ws, double* tri) {
  TraceRange tr("chfsi cholqr factor");
  return potrf_lower(A, lda, b, info, st, ws, tri, kGramPivotTol);
}

// the eigensolver under a roctx range; pinned (two ints of pinned host memory)
// and ev let it queue the next sweep's first launches before each read-back
hipError_t syev_traced(double* A, int64_t lda, int64_t b, double* w, double* V, int64_t ldv,
                       hipStream_t st, const Workspace& ws, int* sweeps, int* unconverged,
                       int* pinned = nullptr, hipEvent_t ev = nullptr) {
  TraceRange tr("chfsi jacobi eigensolve");
  return syev_jacobi(A, lda, b, w, V, ldv, st, ws, sweeps, unconverged, pinned, ev);
}

thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

}  // namespace

// the calling thread's error message, for the other translation units
void chfsi::set_error_message(const char* msg) { g_last_error = msg; }

namespace {

#define CK(expr)                                                                        \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess) {                                                             \
      set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
      return CHFSI_ERR_DEVICE;                                                          \
    }                                                                                   \
  } while (0)

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

template <typename T>
size_t plan_bytes(int64_t M, int64_t N, int64_t K) {
  int cfg, splits;
  gemm_plan<T>(M, N, K, 1, &cfg, &splits);
  return splits > 1 ? size_t(splits) * size_t(M) * size_t(N) * sizeof(T) : 0;
}

bool is_identity(const chfsi_operator* op) { return op == nullptr || op->kind == CHFSI_OP_IDENTITY; }

// Tuning knobs for the filter's operator-product GEMMs (tile shape index and
// split-K factor); unset or negative = the planner's choice.  Results do not
// depend on them beyond floating-point summation order.
int env_int(const char* name) {
  const char* v = std::getenv(name);
  return v && *v ? std::atoi(v) : -1;
}
int filter_gemm_cfg() { return env_int("CHFSI_FILTER_GEMM_CFG"); }
// CHFSI_PROGRESS=1: chfsi_solve prints one line per outer iteration to stderr
bool progress_log() {
  static const bool v = env_int("CHFSI_PROGRESS") > 0;
  return v;
}
int filter_gemm_splits() {
  const int s = env_int("CHFSI_FILTER_GEMM_SPLITS");
  return s > 0 ? s : 0;
}

}  // namespace

struct chfsi_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  chfsi_operator A{};
  chfsi_operator B{};
  bool B_identity = true;
  const double* dinv = nullptr;
  chfsi_params prm{};
  int64_t n = 0, b = 0;

  std::vector<void*> allocs;  // everything owned
  size_t bytes = 0;
  const Allocator* al = nullptr;   // memory source (null: hipMalloc / hipHostMalloc)

  // filter precision copies / buffers
  float* A32 = nullptr;
  uint16_t* A16 = nullptr;        // bfloat16 copy of a dense operator (BF16 residual filter)
  float* dinv32 = nullptr;        // FP32 D^{-1} (dense: always; stencil: only when given)
  float* Vf = nullptr;            // FP32 potential of a stencil operator (FP32/BF16 filter)
  double* Ht = nullptr;           // exact-inverse filter operator, stored as H^T = A B^{-1} (n x n)
  // complex Hermitian operator (residual filter only): planar left operand
  // L = [A_r | A_i] (n x 2n, filter precision), [d; d], the materialised right
  // operand Z~ (2n x 2b, FP32/FP64) and its bfloat16 copy (BF16)
  bool cplx = false;
  bool bloch = false;             // Bloch-phase grid operator (twisted frame, planar blocks)
  void* bcorr = nullptr;          // its filter step's boundary correction (nbnd x 2b)
  int64_t nbnd = 0;               // boundary points rounded up to a multiple of 4
  void* bedge[2] = {nullptr, nullptr};   // row-end values of the filter blocks (2 ny nz x 2b)
  double* redge = nullptr;                 // row-end values of a Rayleigh-Ritz block (FP64)
  void* Lc = nullptr;
  void* dinv2 = nullptr;
  void* Zt = nullptr;
  double* f64_c = nullptr;        // planar FP64 copy of the residual (complex FP64 filter)
  // complex Rayleigh-Ritz: FP64 planar A and B, planar n x 2b blocks, the
  // 2n x 2b right operand, the 2b x 2b rotation operand and pair selection
  double *LA64 = nullptr, *LB64 = nullptr;
  double *Ypl = nullptr, *AYpl = nullptr, *BYpl = nullptr, *Xpl = nullptr, *Rpl = nullptr;
  double *Yt = nullptr, *Xt = nullptr, *Zx = nullptr, *wdup = nullptr;
  double* tri = nullptr;          // Cholesky / triangular-solve scratch
  float *f32_a = nullptr, *f32_b = nullptr, *f32_c = nullptr;     // RX, RY, Y copy (n x b)
  double *f64_a = nullptr, *f64_b = nullptr;                        // RX, RY (FP64 filter)
  void *bf_a = nullptr, *bf_b = nullptr, *bf_c = nullptr;           // BF16 stencil filter blocks
  float* coef32 = nullptr;        // per-step column coefficients, (p-1) x b
  double* coef64 = nullptr;
  double* lamY = nullptr;         // final Lambda_Y (device, b)
  double* ritz_d = nullptr;       // Ritz values staged for the residual filter (device, b)
  std::vector<float> h_coef32;
  std::vector<double> h_coef64;
  int coef_cap = 0;               // steps the coefficient tables hold

  // Rayleigh-Ritz buffers
  double *Yw = nullptr, *Xw = nullptr, *AY = nullptr, *BY = nullptr, *R = nullptr;
  double *Ga = nullptr, *Gb = nullptr, *Gs = nullptr, *Linv = nullptr, *Tmp = nullptr;
  double *Hp = nullptr, *E = nullptr, *T = nullptr, *TL = nullptr;
  double *svec = nullptr, *w = nullptr, *norms = nullptr;
  int* dflags = nullptr;          // [0] potrf info, [1] bad diag, [2] non-finite
  Workspace ws;
  Workspace ws_eig;

  // pinned host staging
  double* h_w = nullptr;
  double* h_norms = nullptr;
  int* h_flags = nullptr;
  void* h_stage = nullptr;
  size_t h_stage_bytes = 0;

  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_stage = nullptr;   // last copy out of h_stage (reuse waits on it)
  hipEvent_t ev_jac = nullptr;     // the eigensolver's read-back of its sweep flags (h_flags[8..9])
  int last_sweeps = 0;
  int flags = 0;
  int jacobi_unconv = 0;          // the last eigensolve reached its sweep cap
  double* Xbest = nullptr;        // keep_best: Ritz block of the lowest max residual
  double* gs_work = nullptr;      // complex contexts: scratch of the equal-Ritz-value Gram-Schmidt
  // CSR operators: longest rows (checked at create) and FP32 value copies
  int csrA_kmax = 0, csrB_kmax = 0;
  float* val32 = nullptr;
  int svqb_events = 0;            // Rayleigh-Ritz passes that took the SVQB fallback
  int svqb_dropped = 0;           // directions those passes dropped and refilled
  // Lanczos bound estimate: vectors (lanczos_ctx_bytes), pinned scalars, the
  // estimate once made
  double* lz_work = nullptr;
  double* h_lz = nullptr;
  bool have_lmax = false;
  double lmax_est = 0.0;
  // second stream (default priority) for the estimate overlapped with the
  // first Rayleigh-Ritz pass, and the event that orders it after the caller's work
  hipStream_t aux_stream = nullptr;
  hipEvent_t ev_aux = nullptr;
  const std::atomic<int>* cancel = nullptr;
  uint64_t refill_seed = 0;
  // slab-wise Rayleigh-Ritz (memory_mode 1)
  int slab_planes = 0;
  double* S1 = nullptr;
  double* S2 = nullptr;
  // profiling: event pairs around the filter's operator-product kernels
  std::vector<hipEvent_t> pev;
  int pused = 0;
  double pacc_ms = 0.0;
  int pacc_n = 0;
};

void chfsi::ctx_set_cancel_flag(chfsi_ctx* c, const std::atomic<int>* flag) { c->cancel = flag; }

namespace {

chfsi_status check_params(const chfsi_operator* A, const chfsi_operator* B,
                          const chfsi_params* p) {
  if (!A || !p) {
    set_error("A and params must be non-null");
    return CHFSI_ERR_ARG;
  }
  if (A->n <= 0) {
    set_error("operator size must be positive");
    return CHFSI_ERR_ARG;
  }
  if (A->kind == CHFSI_OP_STENCIL27_BLOCH) {
    // complex grid problems at a wave vector k (Section 4.3): the residual filter only
    if (int64_t(A->nx) * A->ny * A->nz != A->n || A->nx < 3 || A->ny < 3 || A->nz < 3) {
      set_error("stencil grid nx*ny*nz must equal n with every side >= 3");
      return CHFSI_ERR_ARG;
    }
    if (A->field_mode < 0 || A->field_mode > 2 || (A->field_mode != 0 && !A->field)) {
      set_error("stencil field_mode must be 0, 1 or 2 (1/2 need a field)");
      return CHFSI_ERR_ARG;
    }
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(A->bloch[d])) {
        set_error("the Bloch vector must be finite");
        return CHFSI_ERR_ARG;
      }
    if (!is_identity(B) &&
        (B->kind != CHFSI_OP_STENCIL27_BLOCH || B->n != A->n || B->nx != A->nx ||
         B->ny != A->ny || B->nz != A->nz || B->field_mode != 0 || B->bloch[0] != A->bloch[0] ||
         B->bloch[1] != A->bloch[1] || B->bloch[2] != A->bloch[2])) {
      set_error("with a Bloch grid A, B must be the identity or a Bloch grid operator on A's grid "
                "with the same wave vector and no field");
      return CHFSI_ERR_ARG;
    }
    if (p->method != CHFSI_METHOD_RCHFSI || p->memory_mode != 0 || p->binv_exact != 0) {
      set_error("complex Hermitian operators support the residual filter with memory_mode 0");
      return CHFSI_ERR_ARG;
    }
    if (p->block <= 0 || p->n_wanted <= 0 || p->n_wanted > p->block || p->block > A->n ||
        p->block > 65535) {
      set_error("need 0 < n_wanted <= block <= min(n, 65535)");
      return CHFSI_ERR_ARG;
    }
    if (p->degree < 1 || p->degree > 1000) {
      set_error("degree must be in [1, 1000]");
      return CHFSI_ERR_ARG;
    }
    if (p->filter_prec < CHFSI_PREC_FP64 || p->filter_prec > CHFSI_PREC_BF16) {
      set_error("unknown filter precision");
      return CHFSI_ERR_ARG;
    }
    return CHFSI_OK;
  }
  if (A->kind == CHFSI_OP_DENSE_HERMITIAN) {
    // complex Hermitian problems (Section 4.3): the residual filter only
    if (!A->dense || A->ld < A->n) {
      set_error("dense A needs a device pointer and ld >= n");
      return CHFSI_ERR_ARG;
    }
    if (!is_identity(B) && (B->kind != CHFSI_OP_DENSE_HERMITIAN || B->n != A->n || !B->dense ||
                            B->ld < B->n)) {
      set_error("with a Hermitian A, B must be the identity or a Hermitian dense matrix of A's size");
      return CHFSI_ERR_ARG;
    }
    if (p->method != CHFSI_METHOD_RCHFSI || p->memory_mode != 0 || p->binv_exact != 0) {
      set_error("complex Hermitian operators support the residual filter with memory_mode 0");
      return CHFSI_ERR_ARG;
    }
    if (p->block <= 0 || p->n_wanted <= 0 || p->n_wanted > p->block || p->block > A->n) {
      set_error("need 0 < n_wanted <= block <= n");
      return CHFSI_ERR_ARG;
    }
    if (p->degree < 1 || p->degree > 1000) {
      set_error("degree must be in [1, 1000]");
      return CHFSI_ERR_ARG;
    }
    if (p->filter_prec < CHFSI_PREC_FP64 || p->filter_prec > CHFSI_PREC_BF16) {
      set_error("unknown filter precision");
      return CHFSI_ERR_ARG;
    }
    return CHFSI_OK;
  }
  if (A->kind == CHFSI_OP_DENSE) {
    if (!A->dense || A->ld < A->n) {
      set_error("dense A needs a device pointer and ld >= n");
      return CHFSI_ERR_ARG;
    }
  } else if (A->kind == CHFSI_OP_STENCIL27) {
    if (int64_t(A->nx) * A->ny * A->nz != A->n || A->nx < 3 || A->ny < 3 || A->nz < 3) {
      set_error("stencil grid nx*ny*nz must equal n with every side >= 3");
      return CHFSI_ERR_ARG;
    }
    if (A->field_mode < 0 || A->field_mode > 2 || (A->field_mode != 0 && !A->field)) {
      set_error("stencil field_mode must be 0, 1 or 2 (1/2 need a field)");
      return CHFSI_ERR_ARG;
    }
  } else if (A->kind == CHFSI_OP_CSR) {
    if (!A->rowptr || !A->colind || !A->val || A->nnz < 0 || A->n >= (int64_t(1) << 31)) {
      set_error("CSR A needs rowptr, colind and val device arrays, nnz >= 0 and n < 2^31");
      return CHFSI_ERR_ARG;
    }
  } else {
    set_error("A must be dense, a stencil or a CSR operator");
    return CHFSI_ERR_ARG;
  }
  if (!is_identity(B)) {
    if (B->n != A->n) {
      set_error("B must have the size of A");
      return CHFSI_ERR_ARG;
    }
    if (B->kind == CHFSI_OP_DENSE && (!B->dense || B->ld < B->n)) {
      set_error("dense B needs a device pointer and ld >= n");
      return CHFSI_ERR_ARG;
    }
    if (B->kind == CHFSI_OP_STENCIL27 &&
        (B->nx != A->nx || B->ny != A->ny || B->nz != A->nz || B->field_mode != 0)) {
      set_error("stencil B must share A's grid and carry no field");
      return CHFSI_ERR_ARG;
    }
    if (B->kind == CHFSI_OP_CSR && (!B->rowptr || !B->colind || !B->val || B->nnz < 0)) {
      set_error("CSR B needs rowptr, colind and val device arrays and nnz >= 0");
      return CHFSI_ERR_ARG;
    }
    if (B->kind != CHFSI_OP_DENSE && B->kind != CHFSI_OP_STENCIL27 && B->kind != CHFSI_OP_CSR) {
      set_error("unsupported B kind");
      return CHFSI_ERR_ARG;
    }
  }
  if (p->block <= 0 || p->n_wanted <= 0 || p->n_wanted > p->block || p->block > A->n) {
    set_error("need 0 < n_wanted <= block <= n");
    return CHFSI_ERR_ARG;
  }
  if (p->degree < 1 || p->degree > 1000) {
    set_error("degree must be in [1, 1000]");
    return CHFSI_ERR_ARG;
  }
  if (p->method != CHFSI_METHOD_CHFSI && p->method != CHFSI_METHOD_RCHFSI) {
    set_error("unknown method");
    return CHFSI_ERR_ARG;
  }
  if (p->filter_prec < CHFSI_PREC_FP64 || p->filter_prec > CHFSI_PREC_BF16) {
    set_error("unknown filter precision");
    return CHFSI_ERR_ARG;
  }
  if (p->filter_prec == CHFSI_PREC_BF16 && A->kind != CHFSI_OP_STENCIL27 &&
      A->kind != CHFSI_OP_DENSE && A->kind != CHFSI_OP_CSR) {
    set_error("BF16 filters are implemented for dense, stencil and CSR operators");
    return CHFSI_ERR_ARG;
  }
  if (p->filter_prec == CHFSI_PREC_BF16 && p->method != CHFSI_METHOD_RCHFSI) {
    set_error("BF16 filters are implemented for the residual filter only");
    return CHFSI_ERR_ARG;
  }
  if (p->binv_exact != 0 &&
      (p->binv_exact != 1 || A->kind != CHFSI_OP_DENSE || is_identity(B) ||
       B->kind != CHFSI_OP_DENSE || p->method != CHFSI_METHOD_CHFSI ||
       p->filter_prec != CHFSI_PREC_FP64 || p->memory_mode != 0)) {
    set_error("binv_exact needs dense A and B and the plain filter in FP64");
    return CHFSI_ERR_ARG;
  }
  if (p->memory_mode != 0) {
    if (p->memory_mode != 1 || A->kind != CHFSI_OP_STENCIL27 || !stencil_separable(*A) ||
        (!is_identity(B) && (B->kind != CHFSI_OP_STENCIL27 || !stencil_separable(*B))) ||
        p->method != CHFSI_METHOD_RCHFSI || p->filter_prec == CHFSI_PREC_FP64) {
      set_error("memory_mode 1 needs tensor-product stencil operators and the residual filter "
                "in FP32 or BF16");
      return CHFSI_ERR_ARG;
    }
  }
  return CHFSI_OK;
}

// z-planes per slab of the slab-wise Rayleigh-Ritz: about 1/16 of the grid,
// at most 2 GiB per slab block
int slab_planes_for(const chfsi_operator& A, int64_t b) {
  const double plane = double(A.nx) * A.ny * b * sizeof(double);
  int nzs = std::max(1, A.nz / 16);
  while (nzs > 1 && plane * nzs > 2.0 * 1024 * 1024 * 1024) --nzs;
  return nzs;
}

struct SizePlan {
  int slab_planes = 0;
  size_t slab = 0;
  size_t total = 0;
  size_t a32 = 0, f32blk = 0, f64blk = 0, bfblk = 0, coef = 0;
  size_t blk = 0, bb = 0, ws = 0, ws_eig = 0, tri = 0;
};

SizePlan plan_sizes_complex(const chfsi_operator* A, const chfsi_params* p) {
  SizePlan s;
  const int64_t n = A->n, b = p->block;
  const size_t el = p->filter_prec == CHFSI_PREC_FP64 ? sizeof(double) : sizeof(float);
  const size_t lel = p->filter_prec == CHFSI_PREC_BF16 ? sizeof(uint16_t) : el;
  s.a32 = size_t(n) * 2 * n * lel + size_t(2) * n * el;              // L, [d; d]
  s.f32blk = size_t(n) * 2 * b * el;                                   // one planar block
  size_t zt = size_t(2) * n * 2 * b * el;                              // Z~
  if (p->filter_prec == CHFSI_PREC_BF16) zt += size_t(2) * n * 2 * b * sizeof(uint16_t);
  s.coef = size_t(p->degree + 1) * 2 * b * sizeof(double);
  // Rayleigh-Ritz on the 2b x 2b real embedding
  const int64_t m = 2 * b;
  s.blk = size_t(n) * b * 2 * sizeof(double);                          // one complex block
  s.bb = size_t(m) * m * sizeof(double);
  s.ws_eig = syev_workspace_bytes(m) + 256;
  s.tri = tri_workspace_bytes(m, m);
  size_t rr = size_t(n) * 2 * n * sizeof(double) * (p->filter_prec == CHFSI_PREC_FP64 ? 0 : 1) +
              size_t(n) * 2 * n * sizeof(double) +                     // LA64 (FP32/BF16), LB64
              5 * s.blk + size_t(2) * n * 2 * b * sizeof(double) +     // planar blocks, Y~
              3 * s.blk + 12 * s.bb + 8 * m * sizeof(double);         // Xw, Yw, R, small
  size_t ws = p->filter_prec == CHFSI_PREC_FP64
                  ? std::max(plan_bytes<double>(n, 2 * b, 2 * n), size_t(16) * n * 2 * b * el)
                  : std::max(plan_bytes<float>(n, 2 * b, 2 * n), size_t(16) * n * 2 * b * el);
  if (p->filter_prec == CHFSI_PREC_BF16) ws = std::max(ws, gemm_bf16_workspace_bytes(n, 2 * b));
  ws = std::max(ws, plan_bytes<double>(n, m, 2 * n));
  ws = std::max(ws, plan_bytes<double>(m, m, n));
  ws = std::max(ws, 2 * gemm_workspace_bytes(b, b, n, sizeof(double)));   // batched Gram blocks
  ws = std::max(ws, plan_bytes<double>(n, m, m));
  ws = std::max(ws, plan_bytes<double>(m, m, m));
  s.ws = ws + 256;
  s.total = s.a32 + 3 * s.f32blk + zt + 2 * s.coef + b * sizeof(double) + s.ws + 64 + rr +
            s.ws_eig + s.tri;
  return s;
}

// Bloch grid contexts: three planar filter blocks (n x 2b) in the filter
// precision, FP32 copies of D^{-1} and V (FP32/BF16), and the complex
// Rayleigh-Ritz buffers without any n x n operand
SizePlan plan_sizes_bloch(const chfsi_operator* A, const chfsi_operator* B, const chfsi_params* p) {
  SizePlan s;
  const int64_t n = A->n, b = p->block, m = 2 * b;
  const size_t el = p->filter_prec == CHFSI_PREC_FP64   ? sizeof(double)
                    : p->filter_prec == CHFSI_PREC_FP32 ? sizeof(float)
                                                        : sizeof(uint16_t);
  s.f32blk = size_t(n) * 2 * b * el;
  if (p->filter_prec != CHFSI_PREC_FP64)
    s.a32 = size_t(n) * sizeof(float) * (1 + (A->field_mode != 0 ? 1 : 0));
  // the boundary correction, in the step's arithmetic type, and two copies of
  // the blocks' row ends
  s.a32 += size_t((bloch_boundary_points(A->nx, A->ny, A->nz) + 3) / 4 * 4) * 2 * b *
               (p->filter_prec == CHFSI_PREC_FP64 ? sizeof(double) : sizeof(float)) +
           size_t(2) * 2 * A->ny * A->nz * 2 * b * el +
           size_t(2) * A->ny * A->nz * 2 * b * sizeof(double);
  s.coef = size_t(p->degree + 1) * 2 * b * sizeof(double);
  s.blk = size_t(n) * b * 2 * sizeof(double);
  s.bb = size_t(m) * m * sizeof(double);
  s.ws_eig = syev_workspace_bytes(m) + 256;
  s.tri = tri_workspace_bytes(m, m);
  const size_t rr = (is_identity(B) ? 4 : 5) * s.blk + 3 * s.blk + 12 * s.bb + 8 * m * sizeof(double);
  size_t ws = plan_bytes<double>(m, m, n);
  ws = std::max(ws, 2 * gemm_workspace_bytes(b, b, n, sizeof(double)));   // batched Gram blocks
  ws = std::max(ws, plan_bytes<double>(n, m, m));
  ws = std::max(ws, plan_bytes<double>(m, m, m));
  s.ws = ws + 256;
  s.total = s.a32 + 3 * s.f32blk + 2 * s.coef + b * sizeof(double) + s.ws + 64 + rr + s.ws_eig +
            s.tri;
  return s;
}

// device bytes of the Lanczos bound estimate: its vectors plus the start
// vector, a planar copy of D^{-1} and the complex product's right operand
size_t lanczos_ctx_bytes(int64_t n, bool cplx) {
  const int64_t L = cplx ? 2 * n : n;
  return lanczos_workspace_bytes(L) + size_t(6) * L * sizeof(double) + 256;
}

SizePlan plan_sizes_kind(const chfsi_operator* A, const chfsi_operator* B, const chfsi_params* p);

SizePlan plan_sizes(const chfsi_operator* A, const chfsi_operator* B, const chfsi_params* p) {
  SizePlan s = plan_sizes_kind(A, B, p);
  if (A->kind == CHFSI_OP_DENSE_HERMITIAN || A->kind == CHFSI_OP_STENCIL27_BLOCH)
    s.total += cluster_gs_work_bytes(p->block, p->block) + 256;
  if (p->keep_best) {
    const bool cx = A->kind == CHFSI_OP_DENSE_HERMITIAN || A->kind == CHFSI_OP_STENCIL27_BLOCH;
    s.total += size_t(A->n) * (cx ? 2 : 1) * p->block * sizeof(double);
  }
  if (std::isnan(p->lambda_max))
    s.total += lanczos_ctx_bytes(A->n, A->kind == CHFSI_OP_DENSE_HERMITIAN ||
                                           A->kind == CHFSI_OP_STENCIL27_BLOCH);
  return s;
}

SizePlan plan_sizes_kind(const chfsi_operator* A, const chfsi_operator* B, const chfsi_params* p) {
  if (A->kind == CHFSI_OP_DENSE_HERMITIAN) return plan_sizes_complex(A, p);
  if (A->kind == CHFSI_OP_STENCIL27_BLOCH) return plan_sizes_bloch(A, B, p);
  SizePlan s;
  const int64_t n = A->n, b = p->block;
  const bool dense = A->kind == CHFSI_OP_DENSE;
  s.blk = size_t(n) * b * sizeof(double);
  s.bb = size_t(b) * b * sizeof(double);
  if (p->filter_prec == CHFSI_PREC_FP32) {
    s.f32blk = size_t(n) * b * sizeof(float);
    if (dense) s.a32 = size_t(n) * n * sizeof(float) + size_t(n) * sizeof(float);
  } else if (p->filter_prec == CHFSI_PREC_BF16 && dense) {
    // BF16 products on a bfloat16 copy of A, FP32 filter blocks
    s.f32blk = size_t(n) * b * sizeof(float);
    s.a32 = size_t(n) * n * sizeof(uint16_t) + size_t(n) * sizeof(float) + size_t(n) * b * 2;
  } else if (p->filter_prec == CHFSI_PREC_FP64) {
    s.f64blk = s.blk;
  } else if (p->escalate) {
    s.f32blk = size_t(n) * b * sizeof(float);   // FP32 blocks; BF16 data in their first halves
  } else {
    s.bfblk = size_t(n) * b * 2;
  }
  if (p->escalate && dense) s.a32 += size_t(n) * n * sizeof(float);   // FP32 copy of A
  // stencil filters in FP32/BF16: FP32 copies of D^{-1} and of the potential
  if (A->kind == CHFSI_OP_STENCIL27 && p->filter_prec != CHFSI_PREC_FP64)
    s.a32 += size_t(n) * sizeof(float) * (1 + (A->field_mode != 0 ? 1 : 0));
  // CSR filters in FP32/BF16: FP32 copies of D^{-1} and of the values
  if (A->kind == CHFSI_OP_CSR && p->filter_prec != CHFSI_PREC_FP64)
    s.a32 += size_t(n) * sizeof(float) + size_t(A->nnz) * sizeof(float);
  s.coef = size_t(p->degree + 1) * b * sizeof(double);
  size_t ws = 0;
  if (dense) {
    // the filter product may be run with up to 16 k-splits (tuning knob)
    if (p->filter_prec == CHFSI_PREC_FP32)
      ws = std::max(ws, std::max(plan_bytes<float>(n, b, n), size_t(16) * n * b * sizeof(float)));
    ws = std::max(ws, plan_bytes<double>(n, b, n));
    if (p->filter_prec == CHFSI_PREC_FP64)
      ws = std::max(ws, size_t(16) * n * b * sizeof(double));
    if (p->filter_prec == CHFSI_PREC_BF16) ws = std::max(ws, gemm_bf16_workspace_bytes(n, b));
  }
  ws = std::max(ws, plan_bytes<double>(b, b, n));
  ws = std::max(ws, plan_bytes<double>(n, b, b));
  if (p->memory_mode == 1) {
    const int64_t rows = int64_t(A->nx) * A->ny * slab_planes_for(*A, b);
    ws = std::max(ws, plan_bytes<double>(b, b, rows));
    ws = std::max(ws, plan_bytes<double>(rows, b, b));
  }
  ws = std::max(ws, plan_bytes<double>(b, b, b));
  s.ws = ws + 256;
  s.ws_eig = syev_workspace_bytes(b) + 256;
  s.tri = tri_workspace_bytes(b, b);
  const bool Bid = is_identity(B);
  // filter blocks: FP32 3 blocks, FP64 2 blocks, BF16 3 blocks
  size_t filt = 3 * s.f32blk + 2 * s.f64blk + 3 * s.bfblk;
  // RR: Yw, Xw, AY, R (+ BY when B != I); slab-wise: R + two slabs
  size_t rr = (Bid ? 4 : 5) * s.blk;
  if (p->memory_mode == 1) {
    s.slab_planes = slab_planes_for(*A, b);
    s.slab = size_t(A->nx) * A->ny * s.slab_planes * b * sizeof(double);
    rr = s.blk + 2 * s.slab;
  }
  s.total = s.a32 + filt + 2 * s.coef + rr + 10 * s.bb + 5 * b * sizeof(double) + 64 + s.ws +
            s.ws_eig + s.tri;
  if (p->binv_exact) s.total += size_t(n) * n * sizeof(double);   // H^T (formation: 3 more, freed)
  return s;
}

template <typename T>
T* ctx_alloc(chfsi_ctx* c, size_t bytes, chfsi_status* st) {
  if (bytes == 0) return nullptr;
  void* p = nullptr;
  if (c->al) {
    p = c->al->dev_alloc(c->al->self, (bytes + 255) / 256 * 256);
    if (!p) {
      set_error("device pool allocation of %zu bytes failed", bytes);
      *st = CHFSI_ERR_NOMEM;
      return nullptr;
    }
  } else {
    hipError_t e = hipMalloc(&p, (bytes + 255) / 256 * 256);
    if (e != hipSuccess) {
      set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
      *st = CHFSI_ERR_NOMEM;
      return nullptr;
    }
  }
  c->allocs.push_back(p);
  c->bytes += bytes;
  return static_cast<T*>(p);
}

// the kernels' view of a CSR operator of the context (FP64 values, or the
// FP32 copy of A's)
CsrMat csr_of(const chfsi_ctx* c, const chfsi_operator& op, bool f32) {
  CsrMat m;
  m.n = op.n;
  m.rowptr = op.rowptr;
  m.col = op.colind;
  m.val = f32 ? static_cast<const void*>(c->val32) : static_cast<const void*>(op.val);
  m.kmax = (&op == &c->B) ? c->csrB_kmax : c->csrA_kmax;
  return m;
}

// nominal flops per element and step of an operator product (for reporting)
double op_flops(const chfsi_operator& op) {
  if (op.kind == CHFSI_OP_CSR) return 2.0 * double(op.nnz) / double(std::max<int64_t>(op.n, 1));
  return stencil_flops(op);
}

// y = Op x for an n x b FP64 block
chfsi_status apply_op64(chfsi_ctx* c, const chfsi_operator* op, const double* X, int64_t ldx,
                        double* Y, int64_t ldy, int64_t b) {
  if (op->kind == CHFSI_OP_DENSE) {
    GemmDesc<double> g;
    g.M = c->n;
    g.N = b;
    g.K = c->n;
    g.A = op->dense;      // symmetric: A(m,k) = dense[k + m*ld]
    g.sak = 1;
    g.sam = op->ld;
    g.B = X;
    g.sbk = 1;
    g.sbn = ldx;
    g.C = Y;
    g.ldc = ldy;
    CK(gemm<double>(g, c->stream, c->ws));
    return CHFSI_OK;
  }
  if (op->kind == CHFSI_OP_STENCIL27) {
    CK(stencil_apply_f64(*op, X, ldx, Y, ldy, b, c->stream));
    return CHFSI_OK;
  }
  if (op->kind == CHFSI_OP_CSR) {
    CK(csr_apply_f64(csr_of(c, *op, false), X, ldx, Y, ldy, b, c->stream));
    return CHFSI_OK;
  }
  set_error("unsupported operator kind");
  return CHFSI_ERR_ARG;
}

// Scalars of the filter (Algorithm 2/3, first line)
struct FilterScalars {
  double e, c, sigma1;
};

// Scalar coefficients of one recurrence step: R_X <- a H R_Y + bb R_Y + cc R_X (+ forcing)
struct StepCoef {
  double a, bb, cc;
};

FilterScalars filter_scalars(double lmin, double lmax, double lT) {
  FilterScalars f;
  f.e = (lmax - lT) / 2.0;
  f.c = (lmax + lT) / 2.0;
  f.sigma1 = f.e / (lmin - f.c);
  return f;
}

// Resolve the recorded event pairs into the running totals (synchronising).
hipError_t prof_flush(chfsi_ctx* c) {
  for (int i = 0; i + 1 < c->pused; i += 2) {
    hipError_t e = hipEventSynchronize(c->pev[i + 1]);
    if (e != hipSuccess) return e;
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, c->pev[i], c->pev[i + 1]);
    if (e != hipSuccess) return e;
    c->pacc_ms += ms;
    c->pacc_n += 1;
  }
  c->pused = 0;
  return hipSuccess;
}

// Next (begin, end) event pair, or nulls when profiling is off.
hipError_t prof_pair(chfsi_ctx* c, hipEvent_t* b, hipEvent_t* e) {
  *b = *e = nullptr;
  if (!c->prm.profile || c->pev.empty()) return hipSuccess;
  if (c->pused + 2 > int(c->pev.size())) {
    hipError_t err = prof_flush(c);
    if (err != hipSuccess) return err;
  }
  *b = c->pev[c->pused];
  *e = c->pev[c->pused + 1];
  c->pused += 2;
  return hipSuccess;
}

chfsi_status ensure_coef(chfsi_ctx* c, int p) {
  if (p <= c->coef_cap) return CHFSI_OK;
  set_error("degree %d exceeds the context's degree %d", p, c->coef_cap);
  return CHFSI_ERR_ARG;
}

// Algorithm 3 with the context's filter precision.
// `ritz` is host memory, or device memory when `ritz_on_device`.
chfsi_status filter_rchfsi(chfsi_ctx* c, const double* X, int64_t ldx, const double* ritz,
                           const double* resid, int64_t ldr, double* Yp, int64_t ldy, double lmin,
                           double lmax, double lT, int p, double* flops,
                           bool ritz_on_device = false) {
  const int64_t n = c->n, b = c->b;
  chfsi_status st = ensure_coef(c, p);
  if (st != CHFSI_OK) return st;
  const FilterScalars f = filter_scalars(lmin, lmax, lT);
  const double gamma = 2.0 / f.sigma1;
  // the Lambda recurrence (eq. ChFSIrecurrenceEigval) runs on the device in FP64
  // and writes each step's forcing coefficients Lambda_Y (before the update) and
  // the final Lambda_Y for the reconstruction
  const double* ritz_d = ritz;
  if (!ritz_on_device) {
    // the staging buffer may still feed an earlier asynchronous copy
    CK(hipEventSynchronize(c->ev_stage));
    std::memcpy(c->h_stage, ritz, b * sizeof(double));
    CK(hipMemcpyAsync(c->ritz_d, c->h_stage, b * sizeof(double), hipMemcpyHostToDevice,
                      c->stream));
    CK(hipEventRecord(c->ev_stage, c->stream));
    ritz_d = c->ritz_d;
  }
  const bool f64tab = c->prm.filter_prec == CHFSI_PREC_FP64;
  CK(rchfsi_coef(ritz_d, b, f.e, f.c, f.sigma1, p, f64tab ? c->coef64 : nullptr,
                 f64tab ? nullptr : c->coef32, c->lamY, c->stream));
  // the block recurrence's scalar coefficients, step by step
  double sigma = f.sigma1;
  auto next_step = [&]() {
    const double sigma2 = 1.0 / (gamma - sigma);
    const double a = 2.0 * sigma2 / f.e;
    const StepCoef sc{a, -a * f.c, -sigma * sigma2};
    sigma = sigma2;
    return sc;
  };
  const int nsteps = p - 1;
  const double scale1 = f.sigma1 / f.e;
  double fl = 0.0;
  const bool dense = c->A.kind == CHFSI_OP_DENSE;
  if (c->prm.filter_prec == CHFSI_PREC_FP32 || (c->prm.filter_prec == CHFSI_PREC_BF16 && dense)) {
    // FP32 filter blocks; the operator product is FP32 MFMA, or BF16 MFMA on
    // the bfloat16 copy of A (dense BF16)
    float* RX = c->f32_a;
    float* RY = c->f32_b;
    float* Yc = c->f32_c;
    CK(rchfsi_init_f32(resid, ldr, n, b, scale1, RY, RX, Yc, n, c->stream));
    // dense BF16: each step's split-K reduction also rounds D^{-1} R_Y for the next
    bool b16_ready = false;
    for (int s = 0; s < nsteps; ++s) {
      const StepCoef sp = next_step();
      if (dense) {
        GemmDesc<float> g;
        g.M = n;
        g.N = b;
        g.K = n;
        g.A = c->A32;
        g.sak = 1;
        g.sam = n;
        g.B = RY;
        g.sbk = 1;
        g.sbn = n;
        g.kscale = c->dinv32;
        g.C = RX;
        g.ldc = n;
        g.epi.alpha = float(sp.a);
        g.epi.beta = float(sp.bb);
        g.epi.C1 = RY;
        g.epi.ldc1 = n;
        g.epi.gamma = float(sp.cc);
        g.epi.C2 = RX;
        g.epi.ldc2 = n;
        g.epi.delta = float(sp.a);
        g.epi.colscale3 = c->coef32 + int64_t(s) * b;
        g.epi.C3 = Yc;
        g.epi.ldc3 = n;
        CK(prof_pair(c, &g.ev_begin, &g.ev_end));
        if (c->prm.filter_prec == CHFSI_PREC_BF16) {
          uint16_t* b16 = static_cast<uint16_t*>(c->bf_a);
          bool next_ready = false;
          CK(gemm_bf16_filter(g, c->A16, n, b16, c->stream, c->ws, filter_gemm_splits(),
                              b16_ready, s + 1 < nsteps ? b16 : nullptr, c->dinv32,
                              &next_ready));
          b16_ready = next_ready;
        } else
          CK(gemm<float>(g, c->stream, c->ws, filter_gemm_splits(), filter_gemm_cfg()));
        fl += 2.0 * double(n) * double(n) * double(b);
      } else {
        StencilStep ss{sp.a, sp.bb, sp.cc, sp.a};
        {
          hipEvent_t e0, e1;
          CK(prof_pair(c, &e0, &e1));
          if (e0) CK(hipEventRecord(e0, c->stream));
          if (c->A.kind == CHFSI_OP_CSR)
            CK(csr_rchfsi_step_f32(csr_of(c, c->A, true), c->dinv ? c->dinv32 : nullptr, RY, RX,
                                   Yc, c->coef32 + int64_t(s) * b, ss, b, c->stream));
          else
            CK(stencil_rchfsi_step_f32(c->A, c->Vf, c->dinv32, RY, RX, Yc,
                                       c->coef32 + int64_t(s) * b, ss, b, c->stream));
          if (e1) CK(hipEventRecord(e1, c->stream));
        }
        fl += op_flops(c->A) * double(n) * double(b);
      }
      std::swap(RX, RY);
    }
    CK(rchfsi_reconstruct_f32(RY, n, c->dinv, X, ldx, c->lamY, Yp, ldy, n, b, c->stream));
  } else if (c->prm.filter_prec == CHFSI_PREC_FP64) {
    double* RX = c->f64_a;
    double* RY = c->f64_b;
    CK(rchfsi_init_f64(resid, ldr, n, b, scale1, RY, RX, n, c->stream));
    for (int s = 0; s < nsteps; ++s) {
      const StepCoef sp = next_step();
      if (dense) {
        GemmDesc<double> g;
        g.M = n;
        g.N = b;
        g.K = n;
        g.A = c->A.dense;
        g.sak = 1;
        g.sam = c->A.ld;
        g.B = RY;
        g.sbk = 1;
        g.sbn = n;
        g.kscale = c->dinv;
        g.C = RX;
        g.ldc = n;
        g.epi.alpha = sp.a;
        g.epi.beta = sp.bb;
        g.epi.C1 = RY;
        g.epi.ldc1 = n;
        g.epi.gamma = sp.cc;
        g.epi.C2 = RX;
        g.epi.ldc2 = n;
        g.epi.delta = sp.a;
        g.epi.colscale3 = c->coef64 + int64_t(s) * b;
        g.epi.C3 = resid;
        g.epi.ldc3 = ldr;
        CK(prof_pair(c, &g.ev_begin, &g.ev_end));
        CK(gemm<double>(g, c->stream, c->ws, filter_gemm_splits(), filter_gemm_cfg()));
        fl += 2.0 * double(n) * double(n) * double(b);
      } else {
        StencilStep ss{sp.a, sp.bb, sp.cc, sp.a};
        {
          hipEvent_t e0, e1;
          CK(prof_pair(c, &e0, &e1));
          if (e0) CK(hipEventRecord(e0, c->stream));
          if (c->A.kind == CHFSI_OP_CSR)
            CK(csr_rchfsi_step_f64(csr_of(c, c->A, false), c->dinv, RY, RX, resid, ldr,
                                   c->coef64 + int64_t(s) * b, ss, b, c->stream));
          else
            CK(stencil_rchfsi_step_f64(c->A, c->dinv, RY, RX, resid, ldr,
                                       c->coef64 + int64_t(s) * b, ss, b, c->stream));
          if (e1) CK(hipEventRecord(e1, c->stream));
        }
        fl += op_flops(c->A) * double(n) * double(b);
      }
      std::swap(RX, RY);
    }
    CK(rchfsi_reconstruct_f64(RY, n, c->dinv, X, ldx, c->lamY, Yp, ldy, n, b, c->stream));
  } else {
    // BF16-stored blocks, FP32 arithmetic (stencil operators)
    void* RX = c->bf_a;
    void* RY = c->bf_b;
    void* Yc = c->bf_c;
    CK(rchfsi_init_bf16(resid, ldr, n, b, scale1, RY, RX, Yc, c->stream));
    for (int s = 0; s < nsteps; ++s) {
      const StepCoef sp = next_step();
      StencilStep ss{sp.a, sp.bb, sp.cc, sp.a};
      {
        hipEvent_t e0, e1;
        CK(prof_pair(c, &e0, &e1));
        if (e0) CK(hipEventRecord(e0, c->stream));
        if (c->A.kind == CHFSI_OP_CSR)
          CK(csr_rchfsi_step_bf16(csr_of(c, c->A, true), c->dinv ? c->dinv32 : nullptr, RY, RX,
                                  Yc, c->coef32 + int64_t(s) * b, ss, b, c->stream));
        else
          CK(stencil_rchfsi_step_bf16(c->A, c->Vf, c->dinv32, RY, RX, Yc,
                                      c->coef32 + int64_t(s) * b, ss, b, c->stream));
        if (e1) CK(hipEventRecord(e1, c->stream));
      }
      fl += op_flops(c->A) * double(n) * double(b);
      std::swap(RX, RY);
    }
    CK(rchfsi_reconstruct_bf16(RY, c->dinv, X, ldx, c->lamY, Yp, ldy, n, b, c->stream));
  }
  if (flops) *flops += fl;
  return CHFSI_OK;
}

Twist twist_of(const chfsi_ctx* c) {
  return Twist{c->A.bloch[0], c->A.bloch[1], c->A.bloch[2], c->A.nx, c->A.ny};
}

// Algorithm 3 for a complex Hermitian A (Section 4.3).  The recurrence's
// coefficients and Lambda are real, so every step is one real product on
// planar blocks (see complex.hip): R_X <- a (L Z~) + b R_Y + c R_X + a Yc diag(Lambda_Y),
// Z~ built from D^{-1}-scaled R_Y (the product's k-scale [d; d]).  The
// per-column coefficients cover both halves of the planar block.
chfsi_status filter_rchfsi_complex(chfsi_ctx* c, const double* X, int64_t ldx, const double* ritz,
                                   const double* resid, int64_t ldr, double* Yp, int64_t ldy,
                                   double lmin, double lmax, double lT, int p, double* flops) {
  const int64_t n = c->n, b = c->b, b2 = 2 * b;
  chfsi_status st = ensure_coef(c, p);
  if (st != CHFSI_OK) return st;
  const FilterScalars f = filter_scalars(lmin, lmax, lT);
  const double gamma = 2.0 / f.sigma1;
  std::vector<double> LX(b, 1.0), LY(b), LN(b);
  for (int64_t j = 0; j < b; ++j) LY[j] = (f.sigma1 / f.e) * (ritz[j] - f.c);
  struct Step {
    double a, bb, cc;
  };
  std::vector<Step> steps;
  double sigma = f.sigma1;
  for (int k = 2; k <= p; ++k) {
    const double sigma2 = 1.0 / (gamma - sigma);
    const double a = 2.0 * sigma2 / f.e;
    steps.push_back({a, -a * f.c, -sigma * sigma2});
    for (int64_t j = 0; j < b; ++j) {
      for (int h = 0; h < 2; ++h) {
        c->h_coef64[(k - 2) * b2 + h * b + j] = LY[j];
        c->h_coef32[(k - 2) * b2 + h * b + j] = float(LY[j]);
      }
      LN[j] = a * LY[j] * ritz[j] - a * f.c * LY[j] - sigma * sigma2 * LX[j];
    }
    std::swap(LX, LY);
    std::swap(LY, LN);
    sigma = sigma2;
  }
  CK(hipEventSynchronize(c->ev_stage));
  double* h_lam = reinterpret_cast<double*>(c->h_stage);
  std::memcpy(h_lam, LY.data(), b * sizeof(double));
  CK(hipMemcpyAsync(c->lamY, h_lam, b * sizeof(double), hipMemcpyHostToDevice, c->stream));
  const int nsteps = p - 1;
  const double scale1 = f.sigma1 / f.e;
  double fl = 0.0;
  if (c->bloch) {
    // grid operator in the twisted frame: each step is the real z-march on
    // the 2b planar columns plus the boundary correction for wrapped phases
    const Twist tw = twist_of(c);
    const bool f64 = c->prm.filter_prec == CHFSI_PREC_FP64;
    if (nsteps > 0) {
      char* hs = static_cast<char*>(c->h_stage) + b * sizeof(double);
      const size_t bytes = size_t(nsteps) * b2 * (f64 ? sizeof(double) : sizeof(float));
      if (f64)
        std::memcpy(hs, c->h_coef64.data(), bytes);
      else
        std::memcpy(hs, c->h_coef32.data(), bytes);
      CK(hipMemcpyAsync(f64 ? static_cast<void*>(c->coef64) : static_cast<void*>(c->coef32), hs,
                        bytes, hipMemcpyHostToDevice, c->stream));
    }
    CK(hipEventRecord(c->ev_stage, c->stream));
    const double step_fl = (stencil_flops(c->A) * double(n) +
                            27.0 * 8.0 * double(bloch_boundary_points(c->A.nx, c->A.ny, c->A.nz))) *
                           double(b2);
    // the boundary correction goes through the z-march's epilogue when it
    // runs the step, else it is added in place after the step
    // (the row ends of R_Y come from the initialisation, then from each step)
    void* ein = c->bedge[0];
    void* eout = c->bedge[1];
    auto bstep = [&]() { return BlochStep{c->bcorr, c->nbnd, c->dinv, ein, eout}; };
    if (f64) {
      double* RX = c->f64_a;
      double* RY = c->f64_b;
      double* Yc = c->f64_c;
      CK(bloch_init<double>(resid, ldr, n, b, scale1, RY, RX, Yc, tw, c->stream,
                            static_cast<double*>(c->bedge[0])));
      for (int s = 0; s < nsteps; ++s) {
        const Step& sp = steps[s];
        StencilStep ss{sp.a, sp.bb, sp.cc, sp.a};
        hipEvent_t e0, e1;
        const BlochStep bs = bstep();
        CK(prof_pair(c, &e0, &e1));
        if (e0) CK(hipEventRecord(e0, c->stream));
        CK(stencil_rchfsi_step_f64(c->A, c->dinv, RY, RX, Yc, n, c->coef64 + int64_t(s) * b2, ss,
                                   b2, c->stream, &bs));
        if (e1) CK(hipEventRecord(e1, c->stream));
        fl += step_fl;
        std::swap(RX, RY);
        std::swap(ein, eout);
      }
      CK(bloch_reconstruct<double>(RY, c->dinv, X, ldx, c->lamY, Yp, ldy, n, b, tw, c->stream));
    } else if (c->prm.filter_prec == CHFSI_PREC_FP32) {
      float* RX = c->f32_a;
      float* RY = c->f32_b;
      float* Yc = c->f32_c;
      CK(bloch_init<float>(resid, ldr, n, b, scale1, RY, RX, Yc, tw, c->stream,
                            static_cast<float*>(c->bedge[0])));
      for (int s = 0; s < nsteps; ++s) {
        const Step& sp = steps[s];
        StencilStep ss{sp.a, sp.bb, sp.cc, sp.a};
        hipEvent_t e0, e1;
        const BlochStep bs = bstep();
        CK(prof_pair(c, &e0, &e1));
        if (e0) CK(hipEventRecord(e0, c->stream));
        CK(stencil_rchfsi_step_f32(c->A, c->Vf, c->dinv32, RY, RX, Yc,
                                   c->coef32 + int64_t(s) * b2, ss, b2, c->stream, &bs));
        if (e1) CK(hipEventRecord(e1, c->stream));
        fl += step_fl;
        std::swap(RX, RY);
        std::swap(ein, eout);
      }
      CK(bloch_reconstruct<float>(RY, c->dinv, X, ldx, c->lamY, Yp, ldy, n, b, tw, c->stream));
    } else {
      uint16_t* RX = static_cast<uint16_t*>(c->bf_a);
      uint16_t* RY = static_cast<uint16_t*>(c->bf_b);
      uint16_t* Yc = static_cast<uint16_t*>(c->bf_c);
      CK(bloch_init<uint16_t>(resid, ldr, n, b, scale1, RY, RX, Yc, tw, c->stream,
                            static_cast<uint16_t*>(c->bedge[0])));
      for (int s = 0; s < nsteps; ++s) {
        const Step& sp = steps[s];
        StencilStep ss{sp.a, sp.bb, sp.cc, sp.a};
        hipEvent_t e0, e1;
        const BlochStep bs = bstep();
        CK(prof_pair(c, &e0, &e1));
        if (e0) CK(hipEventRecord(e0, c->stream));
        CK(stencil_rchfsi_step_bf16(c->A, c->Vf, c->dinv32, RY, RX, Yc,
                                    c->coef32 + int64_t(s) * b2, ss, b2, c->stream, &bs));
        if (e1) CK(hipEventRecord(e1, c->stream));
        fl += step_fl;
        std::swap(RX, RY);
        std::swap(ein, eout);
      }
      CK(bloch_reconstruct<uint16_t>(RY, c->dinv, X, ldx, c->lamY, Yp, ldy, n, b, tw,
                                     c->stream));
    }
  } else if (c->prm.filter_prec == CHFSI_PREC_FP64) {
    if (nsteps > 0) {
      double* hs = reinterpret_cast<double*>(static_cast<char*>(c->h_stage) + b * sizeof(double));
      std::memcpy(hs, c->h_coef64.data(), size_t(nsteps) * b2 * sizeof(double));
      CK(hipMemcpyAsync(c->coef64, hs, size_t(nsteps) * b2 * sizeof(double),
                        hipMemcpyHostToDevice, c->stream));
    }
    double* RX = c->f64_a;
    double* RY = c->f64_b;
    double* Yc = c->f64_c;
    double* Zt = static_cast<double*>(c->Zt);
    CK(hipEventRecord(c->ev_stage, c->stream));
    CK(cplx_init<double>(resid, ldr, n, b, scale1, RY, RX, Yc, c->stream));
    for (int s = 0; s < nsteps; ++s) {
      const Step& sp = steps[s];
      CK(cplx_rhs<double>(RY, n, b, Zt, c->stream));
      GemmDesc<double> g;
      g.M = n;
      g.N = b2;
      g.K = 2 * n;
      g.A = static_cast<const double*>(c->Lc);
      g.sak = 1;
      g.sam = 2 * n;
      g.B = Zt;
      g.sbk = 1;
      g.sbn = 2 * n;
      g.kscale = static_cast<const double*>(c->dinv2);
      g.C = RX;
      g.ldc = n;
      g.epi.alpha = sp.a;
      g.epi.beta = sp.bb;
      g.epi.C1 = RY;
      g.epi.ldc1 = n;
      g.epi.gamma = sp.cc;
      g.epi.C2 = RX;
      g.epi.ldc2 = n;
      g.epi.delta = sp.a;
      g.epi.colscale3 = c->coef64 + int64_t(s) * b2;
      g.epi.C3 = Yc;
      g.epi.ldc3 = n;
      CK(prof_pair(c, &g.ev_begin, &g.ev_end));
      CK(gemm<double>(g, c->stream, c->ws, filter_gemm_splits(), filter_gemm_cfg()));
      fl += 8.0 * double(n) * double(n) * double(b);
      std::swap(RX, RY);
    }
    CK(cplx_reconstruct<double>(RY, c->dinv, X, ldx, c->lamY, Yp, ldy, n, b, c->stream));
  } else {
    // FP32 blocks; FP32 MFMA on the FP32 L, or bfloat16 MFMA on the bfloat16 L
    if (nsteps > 0) {
      float* hs = reinterpret_cast<float*>(static_cast<char*>(c->h_stage) + b * sizeof(double));
      std::memcpy(hs, c->h_coef32.data(), size_t(nsteps) * b2 * sizeof(float));
      CK(hipMemcpyAsync(c->coef32, hs, size_t(nsteps) * b2 * sizeof(float), hipMemcpyHostToDevice,
                        c->stream));
    }
    float* RX = c->f32_a;
    float* RY = c->f32_b;
    float* Yc = c->f32_c;
    float* Zt = static_cast<float*>(c->Zt);
    const bool bf = c->prm.filter_prec == CHFSI_PREC_BF16;
    CK(hipEventRecord(c->ev_stage, c->stream));
    CK(cplx_init<float>(resid, ldr, n, b, scale1, RY, RX, Yc, c->stream));
    for (int s = 0; s < nsteps; ++s) {
      const Step& sp = steps[s];
      CK(cplx_rhs<float>(RY, n, b, Zt, c->stream));
      GemmDesc<float> g;
      g.M = n;
      g.N = b2;
      g.K = 2 * n;
      g.A = bf ? nullptr : static_cast<const float*>(c->Lc);
      g.sak = 1;
      g.sam = 2 * n;
      g.B = Zt;
      g.sbk = 1;
      g.sbn = 2 * n;
      g.kscale = static_cast<const float*>(c->dinv2);
      g.C = RX;
      g.ldc = n;
      g.epi.alpha = float(sp.a);
      g.epi.beta = float(sp.bb);
      g.epi.C1 = RY;
      g.epi.ldc1 = n;
      g.epi.gamma = float(sp.cc);
      g.epi.C2 = RX;
      g.epi.ldc2 = n;
      g.epi.delta = float(sp.a);
      g.epi.colscale3 = c->coef32 + int64_t(s) * b2;
      g.epi.C3 = Yc;
      g.epi.ldc3 = n;
      CK(prof_pair(c, &g.ev_begin, &g.ev_end));
      if (bf) {
        uint16_t* Zt16 = reinterpret_cast<uint16_t*>(Zt + size_t(2) * n * b2);
        CK(gemm_bf16_filter(g, static_cast<const uint16_t*>(c->Lc), 2 * n, Zt16, c->stream, c->ws,
                            filter_gemm_splits()));
      } else {
        CK(gemm<float>(g, c->stream, c->ws, filter_gemm_splits(), filter_gemm_cfg()));
      }
      fl += 8.0 * double(n) * double(n) * double(b);
      std::swap(RX, RY);
    }
    CK(cplx_reconstruct<float>(RY, c->dinv, X, ldx, c->lamY, Yp, ldy, n, b, c->stream));
  }
  if (flops) *flops += fl;
  return CHFSI_OK;
}

// Algorithm 2 with H = D^{-1} A.
chfsi_status filter_chfsi(chfsi_ctx* c, const double* X, int64_t ldx, double* Yp, int64_t ldy,
                          double lmin, double lmax, double lT, int p, double* flops) {
  const int64_t n = c->n, b = c->b;
  const FilterScalars f = filter_scalars(lmin, lmax, lT);
  const double gamma = 2.0 / f.sigma1;
  const bool dense = c->A.kind == CHFSI_OP_DENSE;
  double fl = 0.0;
  if (c->prm.filter_prec == CHFSI_PREC_FP64) {
    // Y1 = (sigma1/e)(D^{-1} A X - c X)
    double* cur = c->f64_a;
    double* nxt = c->f64_b;
    const double* prev = X;
    int64_t ldprev = ldx;
    auto step = [&](const double* src, int64_t ldsrc, double* dst, double alpha, double beta,
                    const double* Cprev, int64_t ldp, double gam) -> chfsi_status {
      if (dense) {
        GemmDesc<double> g;
        g.M = n;
        g.N = b;
        g.K = n;
        // H = D^{-1} A (A symmetric, read k-contiguous, rows scaled by D^{-1}),
        // or the exact H = B^{-1} A read k-contiguous from its transpose A B^{-1}
        g.A = c->Ht ? c->Ht : c->A.dense;
        g.sak = 1;
        g.sam = c->Ht ? n : c->A.ld;
        g.B = src;
        g.sbk = 1;
        g.sbn = ldsrc;
        g.C = dst;
        g.ldc = n;
        g.epi.alpha = alpha;
        g.epi.rowscale = c->Ht ? nullptr : c->dinv;
        g.epi.beta = beta;
        g.epi.C1 = src;
        g.epi.ldc1 = ldsrc;
        if (Cprev) {
          g.epi.gamma = gam;
          g.epi.C2 = Cprev;
          g.epi.ldc2 = ldp;
        }
        CK(prof_pair(c, &g.ev_begin, &g.ev_end));
        CK(gemm<double>(g, c->stream, c->ws, filter_gemm_splits(), filter_gemm_cfg()));
        fl += 2.0 * double(n) * double(n) * double(b);
      } else {
        StencilStep ss{alpha, beta, gam, 0.0};
        {
          hipEvent_t e0, e1;
          CK(prof_pair(c, &e0, &e1));
          if (e0) CK(hipEventRecord(e0, c->stream));
          if (c->A.kind == CHFSI_OP_CSR)
            CK(csr_chfsi_step_f64(csr_of(c, c->A, false), c->dinv, src, ldsrc, Cprev, ldp, dst, ss,
                                  b, c->stream));
          else
            CK(stencil_chfsi_step_f64(c->A, c->dinv, src, ldsrc, Cprev, ldp, dst, ss, b,
                                      c->stream));
          if (e1) CK(hipEventRecord(e1, c->stream));
        }
        fl += op_flops(c->A) * double(n) * double(b);
      }
      return CHFSI_OK;
    };
    chfsi_status st = step(X, ldx, cur, f.sigma1 / f.e, -f.sigma1 * f.c / f.e, nullptr, 0, 0.0);
    if (st != CHFSI_OK) return st;
    double sigma = f.sigma1;
    for (int k = 2; k <= p; ++k) {
      const double sigma2 = 1.0 / (gamma - sigma);
      const double a = 2.0 * sigma2 / f.e;
      // new = a H cur - a c cur - sigma sigma2 prev; write into prev's storage
      // unless prev is the caller's X
      double* dst = (prev == X) ? nxt : const_cast<double*>(prev);
      st = step(cur, n, dst, a, -a * f.c, prev, ldprev, -sigma * sigma2);
      if (st != CHFSI_OK) return st;
      prev = cur;
      ldprev = n;
      cur = dst;
      sigma = sigma2;
    }
    CK(copy_block(cur, n, Yp, ldy, n, b, c->stream));
  } else if (c->prm.filter_prec == CHFSI_PREC_FP32 && dense) {
    float* Xc = c->f32_c;
    float* cur = c->f32_a;
    float* nxt = c->f32_b;
    CK(convert_f64_f32(X, ldx, Xc, n, n, b, c->stream));
    const float* prev = Xc;
    auto step = [&](const float* src, float* dst, double alpha, double beta, const float* Cprev,
                    double gam) -> chfsi_status {
      GemmDesc<float> g;
      g.M = n;
      g.N = b;
      g.K = n;
      g.A = c->A32;
      g.sak = 1;
      g.sam = n;
      g.B = src;
      g.sbk = 1;
      g.sbn = n;
      g.C = dst;
      g.ldc = n;
      g.epi.alpha = float(alpha);
      g.epi.rowscale = c->dinv32;
      g.epi.beta = float(beta);
      g.epi.C1 = src;
      g.epi.ldc1 = n;
      if (Cprev) {
        g.epi.gamma = float(gam);
        g.epi.C2 = Cprev;
        g.epi.ldc2 = n;
      }
      CK(prof_pair(c, &g.ev_begin, &g.ev_end));
      CK(gemm<float>(g, c->stream, c->ws, filter_gemm_splits(), filter_gemm_cfg()));
      fl += 2.0 * double(n) * double(n) * double(b);
      return CHFSI_OK;
    };
    chfsi_status st = step(Xc, cur, f.sigma1 / f.e, -f.sigma1 * f.c / f.e, nullptr, 0.0);
    if (st != CHFSI_OK) return st;
    double sigma = f.sigma1;
    for (int k = 2; k <= p; ++k) {
      const double sigma2 = 1.0 / (gamma - sigma);
      const double a = 2.0 * sigma2 / f.e;
      float* dst = (prev == Xc) ? nxt : const_cast<float*>(prev);
      st = step(cur, dst, a, -a * f.c, prev, -sigma * sigma2);
      if (st != CHFSI_OK) return st;
      prev = cur;
      cur = dst;
      sigma = sigma2;
    }
    CK(convert_f32_f64(cur, n, Yp, ldy, n, b, c->stream));
  } else {
    set_error("the plain Chebyshev filter supports FP64 (any operator) and FP32 (dense)");
    return CHFSI_ERR_ARG;
  }
  if (flops) *flops += fl;
  return CHFSI_OK;
}

chfsi_status rayleigh_ritz(chfsi_ctx* c, const double* Y, int64_t ldy, double* X, int64_t ldx,
                           double* R, int64_t ldr, double* ritz, double* resnorm,
                           bool allow_svqb);

// norms, finiteness check and read-back of Ritz values and residual norms
chfsi_status finish_rr(chfsi_ctx* c, double* R, int64_t ldr, double* ritz, double* resnorm) {
  const int64_t n = c->n, b = c->b;
  hipStream_t st = c->stream;
  CK(column_norms(R, ldr, n, b, c->norms, st));
  CK(check_finite(c->w, b, c->dflags + 2, st));
  CK(check_finite(c->norms, b, c->dflags + 2, st));
  CK(hipMemcpyAsync(c->h_w, c->w, b * sizeof(double), hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(c->h_norms, c->norms, b * sizeof(double), hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(c->h_flags, c->dflags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (c->h_flags[2] != 0) {
    set_error("non-finite Ritz value or residual norm");
    return CHFSI_ERR_NUMERIC;
  }
  std::memcpy(ritz, c->h_w, b * sizeof(double));
  std::memcpy(resnorm, c->h_norms, b * sizeof(double));
  return CHFSI_OK;
}

chfsi_status rotate_and_residual(chfsi_ctx* c, const double* Y, int64_t ldy, const double* BY,
                                 int64_t ldby, const double* Tm, int64_t k, double* X,
                                 int64_t ldx, double* R, int64_t ldr);

// the fused stencil residual applies (tensor-product stencils for A and B)
bool stencil_residual_ok(const chfsi_ctx* c) {
  return c->A.kind == CHFSI_OP_STENCIL27 && stencil_separable(c->A) &&
         (c->B_identity || (c->B.kind == CHFSI_OP_STENCIL27 && stencil_separable(c->B)));
}

// SVQB reading for a numerically singular scaled Gram matrix G = s Y^T B Y s
// (kept in c->Linv): G = U diag(g) U^T; keep the k directions with
// g > 1e-14 max g; W = diag(s) U_k diag(g_k^{-1/2}) is a B-orthonormal basis
// of the kept span; solve the k x k standard problem W^T (Y^T A Y) W; the
// b - k dropped columns are refilled with N(0,1) values and Rayleigh-Ritz is
// repeated once on the refilled block.
chfsi_status rayleigh_ritz_svqb(chfsi_ctx* c, const double* Y, int64_t ldy, const double* BY,
                                int64_t ldby, double* X, int64_t ldx, double* R, int64_t ldr,
                                double* ritz, double* resnorm) {
  const int64_t n = c->n, b = c->b;
  hipStream_t st = c->stream;
  chfsi_status s;
  int sweeps = 0;
  CK(syev_traced(c->Linv, b, b, c->w, c->E, b, st, c->ws_eig, &sweeps, &c->jacobi_unconv,
                 c->h_flags + 8, c->ev_jac));
  if (c->jacobi_unconv) c->flags |= 2;
  c->last_sweeps += sweeps;
  CK(hipMemcpyAsync(c->h_w, c->w, b * sizeof(double), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  const double gmax = c->h_w[b - 1];
  int64_t first = 0;
  while (first < b && !(c->h_w[first] > 1e-14 * gmax)) ++first;
  const int64_t k = b - first;
  if (k <= 0) {
    set_error("Gram matrix Y^T B Y is numerically zero");
    return CHFSI_ERR_NOT_SPD;
  }
  c->flags |= 1;
  c->svqb_events += 1;
  c->svqb_dropped += int(b - k);
  // W (b x k) in c->T: columns first.. of U, scaled by g^{-1/2}, rows by s
  std::vector<double> colv(k);
  for (int64_t j = 0; j < k; ++j) colv[j] = 1.0 / std::sqrt(c->h_w[first + j]);
  CK(hipEventSynchronize(c->ev_stage));
  std::memcpy(c->h_stage, colv.data(), k * sizeof(double));
  CK(hipMemcpyAsync(c->lamY, c->h_stage, k * sizeof(double), hipMemcpyHostToDevice, st));
  CK(hipEventRecord(c->ev_stage, st));
  CK(copy_block(c->E + first * b, b, c->T, b, b, k, st));
  CK(scale_columns(c->T, b, b, k, c->lamY, st));
  CK(scale_rows(c->T, b, b, k, c->svec, st));
  {
    GemmDesc<double> g;   // Tmp (b x k) = Ga W
    g.M = b;
    g.N = k;
    g.K = b;
    g.A = c->Ga;
    g.sam = 1;
    g.sak = b;
    g.B = c->T;
    g.sbk = 1;
    g.sbn = b;
    g.C = c->Tmp;
    g.ldc = b;
    CK(gemm<double>(g, st, c->ws));
    GemmDesc<double> h;   // Hp (k x k) = W^T Tmp
    h.M = k;
    h.N = k;
    h.K = b;
    h.A = c->T;           // A(m,kk) = W(kk,m)
    h.sak = 1;
    h.sam = b;
    h.B = c->Tmp;
    h.sbk = 1;
    h.sbn = b;
    h.C = c->Hp;
    h.ldc = b;
    CK(gemm<double>(h, st, c->ws));
  }
  CK(symmetrize(c->Hp, b, k, st));
  CK(syev_traced(c->Hp, b, k, c->w, c->E, b, st, c->ws_eig, &sweeps, &c->jacobi_unconv,
                 c->h_flags + 8, c->ev_jac));
  if (c->jacobi_unconv) c->flags |= 2;
  c->last_sweeps += sweeps;
  {
    GemmDesc<double> g;   // Tfin (b x k) = W E, stored in c->Linv
    g.M = b;
    g.N = k;
    g.K = k;
    g.A = c->T;
    g.sam = 1;
    g.sak = b;
    g.B = c->E;
    g.sbk = 1;
    g.sbn = b;
    g.C = c->Linv;
    g.ldc = b;
    CK(gemm<double>(g, st, c->ws));
  }
  if ((s = rotate_and_residual(c, Y, ldy, BY, ldby, c->Linv, k, X, ldx, R, ldr)) != CHFSI_OK)
    return s;
  if (k == b) return finish_rr(c, R, ldr, ritz, resnorm);
  // refill the dropped columns and repeat Rayleigh-Ritz on the refilled block
  c->refill_seed += 1;
  CK(fill_gaussian(X + k * ldx, ldx, n, b - k, c->prm.seed * 7919 + c->refill_seed, st));
  double* tmp = c->Yw;   // free scratch: the input block is no longer needed
  if (tmp == Y) tmp = const_cast<double*>(Y);
  s = rayleigh_ritz(c, X, ldx, tmp, n, R, ldr, ritz, resnorm, false);
  if (s != CHFSI_OK) return s;
  CK(copy_block(tmp, n, X, ldx, n, b, st));
  return CHFSI_OK;
}

// X = Y Tm and R = AY Tm - BY (Tm diag(w)) for the first k columns
chfsi_status rotate_and_residual(chfsi_ctx* c, const double* Y, int64_t ldy, const double* BY,
                                 int64_t ldby, const double* Tm, int64_t k, double* X,
                                 int64_t ldx, double* R, int64_t ldr) {
  TraceRange tr("chfsi rotation + residual");
  const int64_t n = c->n, b = c->b;
  hipStream_t st = c->stream;
  auto rotate = [&](const double* Src, int64_t lds, const double* Tmat, double* Dst, int64_t ldd,
                    double alpha, const double* accum) -> chfsi_status {
    GemmDesc<double> g;
    g.M = n;
    g.N = k;
    g.K = b;
    g.A = Src;
    g.sam = 1;
    g.sak = lds;
    g.B = Tmat;
    g.sbk = 1;
    g.sbn = b;
    g.C = Dst;
    g.ldc = ldd;
    g.epi.alpha = alpha;
    if (accum) {
      g.epi.beta = 1.0;
      g.epi.C1 = accum;
      g.epi.ldc1 = ldd;
    }
    CK(gemm<double>(g, st, c->ws));
    return CHFSI_OK;
  };
  chfsi_status s;
  if ((s = rotate(Y, ldy, Tm, X, ldx, 1.0, nullptr)) != CHFSI_OK) return s;
  if (stencil_residual_ok(c)) {
    // grid operators: R = A X - B X diag(w) in one stencil pass over X instead
    // of rotating A Y and B Y (two N x b x b products)
    CK(stencil_residual_f64(c->A, c->B_identity ? nullptr : &c->B, X, ldx, c->w, R, ldr, k, st));
    return CHFSI_OK;
  }
  if ((s = rotate(c->AY, n, Tm, R, ldr, 1.0, nullptr)) != CHFSI_OK) return s;
  CK(copy_block(Tm, b, c->TL, b, b, k, st));
  CK(scale_columns(c->TL, b, b, k, c->w, st));
  if ((s = rotate(BY, ldby, c->TL, R, ldr, -1.0, R)) != CHFSI_OK) return s;
  return CHFSI_OK;
}

// Rayleigh-Ritz + residuals (see chfsi_rayleigh_ritz).  allow_svqb: on a
// numerically singular Gram matrix fall back to SVQB (see below) once.
chfsi_status rayleigh_ritz(chfsi_ctx* c, const double* Y, int64_t ldy, double* X, int64_t ldx,
                           double* R, int64_t ldr, double* ritz, double* resnorm,
                           bool allow_svqb = true) {
  const int64_t n = c->n, b = c->b;
  hipStream_t st = c->stream;
  chfsi_status s;
  CK(fill_zero(c->dflags, 4 * sizeof(int), st));
  // AY = A Y, BY = B Y
  if ((s = apply_op64(c, &c->A, Y, ldy, c->AY, n, b)) != CHFSI_OK) return s;
  const double* BY = Y;
  int64_t ldby = ldy;
  if (!c->B_identity) {
    if ((s = apply_op64(c, &c->B, Y, ldy, c->BY, n, b)) != CHFSI_OK) return s;
    BY = c->BY;
    ldby = n;
  }
  // Gram matrices Ga = Y^T A Y, Gb = Y^T B Y (K = n).  Both are symmetric:
  // only the tiles on and below the diagonal are formed, then mirrored.
  auto gram = [&](const double* W, int64_t ldw, double* G) -> chfsi_status {
    GemmDesc<double> g;
    g.M = b;
    g.N = b;
    g.K = n;
    g.A = Y;
    g.sak = 1;
    g.sam = ldy;
    g.B = W;
    g.sbk = 1;
    g.sbn = ldw;
    g.C = G;
    g.ldc = b;
    g.lower_only = true;
    CK(gemm<double>(g, st, c->ws));
    CK(symmetrize_panels(G, b, b, 1, st));
    return CHFSI_OK;
  };
  if ((s = gram(c->AY, n, c->Ga)) != CHFSI_OK) return s;
  if ((s = gram(BY, ldby, c->Gb)) != CHFSI_OK) return s;
  // column scaling s = diag(Gb)^{-1/2}; Cholesky of the scaled Gram matrix
  CK(scale_gram(c->Gb, b, b, c->Gs, b, c->svec, c->dflags + 1, st));
  CK(copy_block(c->Gs, b, c->Linv, b, b, b, st));      // kept for the SVQB fallback
  CK(potrf_traced(c->Gs, b, b, c->dflags, st, c->ws, c->tri));
  CK(hipMemcpyAsync(c->h_flags, c->dflags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (c->h_flags[1] != 0) {
    set_error("Gram matrix Y^T B Y has a non-positive diagonal (a zero or non-finite column)");
    return CHFSI_ERR_NOT_SPD;
  }
  if (c->h_flags[0] != 0) {
    if (!allow_svqb) {
      set_error("Gram matrix Y^T B Y is not positive definite (pivot %d) after refill",
                c->h_flags[0]);
      return CHFSI_ERR_NOT_SPD;
    }
    return rayleigh_ritz_svqb(c, Y, ldy, BY, ldby, X, ldx, R, ldr, ritz, resnorm);
  }
  // Linv = L^{-1}
  CK(set_identity(c->Linv, b, b, st));
  CK(trsm_lower_left(c->Gs, b, c->Linv, b, b, b, st, c->ws, c->tri, true));
  // Hp = Linv (s Ga s) Linv^T
  CK(scale_sym(c->Ga, b, b, c->svec, c->Hp, b, st));
  {
    GemmDesc<double> g;   // Tmp = Linv * Hp(scaled Ga)
    g.M = b;
    g.N = b;
    g.K = b;
    g.A = c->Linv;
    g.sam = 1;
    g.sak = b;
    g.B = c->Hp;
    g.sbk = 1;
    g.sbn = b;
    g.C = c->Tmp;
    g.ldc = b;
    CK(gemm<double>(g, st, c->ws));
    GemmDesc<double> h;   // Hp = Tmp * Linv^T
    h.M = b;
    h.N = b;
    h.K = b;
    h.A = c->Tmp;
    h.sam = 1;
    h.sak = b;
    h.B = c->Linv;        // B(k,n) = Linv(n,k) = Linv[n + k*b]
    h.sbn = 1;
    h.sbk = b;
    h.C = c->Hp;
    h.ldc = b;
    CK(gemm<double>(h, st, c->ws));
  }
  CK(symmetrize(c->Hp, b, b, st));
  int sweeps = 0;
  CK(syev_traced(c->Hp, b, b, c->w, c->E, b, st, c->ws_eig, &sweeps, &c->jacobi_unconv,
                 c->h_flags + 8, c->ev_jac));
  if (c->jacobi_unconv) c->flags |= 2;
  c->last_sweeps += sweeps;
  {
    GemmDesc<double> g;   // T = diag(s) Linv^T E
    g.M = b;
    g.N = b;
    g.K = b;
    g.A = c->Linv;        // A(m,k) = Linv(k,m) = Linv[k + m*b]
    g.sak = 1;
    g.sam = b;
    g.B = c->E;
    g.sbk = 1;
    g.sbn = b;
    g.C = c->T;
    g.ldc = b;
    g.epi.rowscale = c->svec;
    CK(gemm<double>(g, st, c->ws));
  }
  if ((s = rotate_and_residual(c, Y, ldy, BY, ldby, c->T, b, X, ldx, R, ldr)) != CHFSI_OK)
    return s;
  return finish_rr(c, R, ldr, ritz, resnorm);
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz for a complex Hermitian pencil (Section 4.3), on interleaved
// complex blocks.  The projected pencil (Y^H A Y, Y^H B Y) is carried by its
// real embedding M(G) = [[G_r, -G_i], [G_i, G_r]] (2b x 2b, real symmetric):
// M(Ga) t = lambda M(Gb) t exactly when x = t(0:b) + i t(b:2b) solves
// Ga x = lambda Gb x, so every Ritz value appears twice and each pair's
// eigenspace is {x c : c complex}.  The real CholQR + Jacobi path runs on the
// embedding unchanged; the first vector of each (ascending) pair gives the
// complex Ritz vector.  Products use the planar real form: AY = L_A Y~,
// Grams P = [Y_r Y_i]^T [W_r W_i], rotation X = [Y_r Y_i] X~.
// ---------------------------------------------------------------------------
chfsi_status rayleigh_ritz_complex(chfsi_ctx* c, const double* Y, int64_t ldy, double* X,
                                   int64_t ldx, double* R, int64_t ldr, double* ritz,
                                   double* resnorm, bool allow_svqb = true);

// The real embedding M(H) of a Hermitian H (cd x cd) has each eigenvalue of H
// twice, with the eigenspace {[Re x; Im x], [-Im x; Re x]}, so the first vector
// of each ascending pair is a complex eigenvector.  When eigenvalues of H are
// equal (to 1e-8 relative), Jacobi returns an arbitrary real basis of their
// joint eigenspace and the first vectors of its pairs need not span it.  For
// each such cluster of the first 2 np eigenvalues (ascending, w on the host),
// the cluster's columns of E (2 cd rows, ld lde, device) are read as complex
// vectors and a pivoted complex Gram-Schmidt on the device (one workgroup,
// cluster_orthonormalize) keeps an orthonormal set of the cluster's size / 2;
// the pairs are rewritten as [Re x; Im x], [-Im x; Re x].  With Mg (device, the embedding M(G) of a
// Hermitian positive definite G, ld 2 cd) the set is orthonormal in x^H G y
// instead (columns of E in the coordinates where G is the metric).  Clusters
// are rare; nothing moves otherwise.
chfsi_status fix_pair_clusters(chfsi_ctx* c, double* E, int64_t lde, int64_t cd, int64_t np,
                               const double* w, const double* Mg = nullptr) {
  double scale = 0.0;
  for (int64_t j = 0; j < 2 * np; ++j) scale = std::max(scale, std::fabs(w[j]));
  const double tol = 1e-8 * std::max(scale, 1e-300);
  hipStream_t st = c->stream;
  // the cluster's Gram-Schmidt runs on the device in the context's scratch
  // for it (sized for a cluster of b pairs of length b)
  const size_t tmp_bytes = cluster_gs_work_bytes(c->b, c->b);
  int64_t j0 = 0;
  while (j0 < np) {
    int64_t j1 = j0 + 1;   // pairs [j0, j1) form one cluster
    while (j1 < np && std::fabs(w[2 * j1] - w[2 * j1 - 1]) <= tol) ++j1;
    if (j1 - j0 > 1) {
      const int64_t ncl = j1 - j0;
      if (cluster_gs_work_bytes(cd, ncl) > tmp_bytes) {
        set_error("a cluster of %lld equal complex eigenvalues is too large for the "
                  "orthonormalisation scratch", (long long)ncl);
        return CHFSI_ERR_NUMERIC;
      }
      CK(cluster_orthonormalize(E + 2 * j0 * lde, lde, cd, ncl, Mg, 2 * cd, c->gs_work,
                                c->dflags + 3, st));
      CK(hipMemcpyAsync(c->h_flags + 3, c->dflags + 3, sizeof(int), hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
      if (c->h_flags[3] != 0) {
        set_error("a cluster of %lld equal complex eigenvalues has no orthonormal basis in the "
                  "embedded eigenvectors", (long long)ncl);
        return CHFSI_ERR_NUMERIC;
      }
    }
    j0 = j1;
  }
  return CHFSI_OK;
}

// SVQB reading for a numerically singular complex Gram matrix, on the real
// embedding, where every complex direction is an eigenvalue pair: the scaled
// embedded Gram matrix (kept in c->Linv) is M(G) = U diag(g) U^T; the pairs
// with g > 1e-14 max g are kept whole, k of them; W = diag(s) U_k diag(g_k^{-1/2})
// (one complex vector per pair) is a B-orthonormal basis of the kept span;
// the k x k Hermitian problem W^H (Y^H A Y) W is solved as the 2k x 2k real
// problem M(W)^T M(Y^H A Y) M(W); `tail` forms X, R and the norms from its
// pairs; the b - k dropped columns are refilled with N(0,1) values (real and
// imaginary parts) and Rayleigh-Ritz is repeated once on the refilled block.
template <typename Tail>
chfsi_status rayleigh_ritz_complex_svqb(chfsi_ctx* c, const double* Y, int64_t ldy, double* X,
                                        int64_t ldx, double* R, int64_t ldr, double* ritz,
                                        double* resnorm, Tail& tail) {
  const int64_t n = c->n, b = c->b, m = 2 * b;
  hipStream_t st = c->stream;
  int sweeps = 0;
  CK(syev_traced(c->Linv, m, m, c->w, c->E, m, st, c->ws_eig, &sweeps, &c->jacobi_unconv,
                 c->h_flags + 8, c->ev_jac));
  if (c->jacobi_unconv) c->flags |= 2;
  c->last_sweeps += sweeps;
  CK(hipMemcpyAsync(c->h_w, c->w, m * sizeof(double), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  const double gmax = c->h_w[m - 1];
  int64_t first = 0;
  while (first < m && !(c->h_w[first] > 1e-14 * gmax)) ++first;
  first += first & 1;                                   // whole pairs only
  const int64_t k = (m - first) / 2;
  if (k <= 0) {
    set_error("Gram matrix Y^H B Y is numerically zero");
    return CHFSI_ERR_NOT_SPD;
  }
  c->flags |= 1;
  c->svqb_events += 1;
  c->svqb_dropped += int(b - k);
  {
    chfsi_status fs = fix_pair_clusters(c, c->E + first * m, m, b, k, c->h_w + first);
    if (fs != CHFSI_OK) return fs;
  }
  std::vector<double> gs(k);
  for (int64_t j = 0; j < k; ++j) gs[j] = 1.0 / std::sqrt(c->h_w[first + 2 * j]);
  CK(hipEventSynchronize(c->ev_stage));
  std::memcpy(c->h_stage, gs.data(), k * sizeof(double));
  CK(hipMemcpyAsync(c->lamY, c->h_stage, k * sizeof(double), hipMemcpyHostToDevice, st));
  CK(hipEventRecord(c->ev_stage, st));
  // W (planar b x 2k) in Zx, M(W) (2b x 2k) in TL
  CK(pairs_to_planar(c->E, m, b, first, k, c->lamY, c->svec, c->Zx, st));
  CK(embed_block(c->Zx, b, k, c->TL, m, st));
  {
    GemmDesc<double> g;   // Tmp (2b x 2k) = M(Ga) M(W)
    g.M = m;
    g.N = 2 * k;
    g.K = m;
    g.A = c->Ga;
    g.sam = 1;
    g.sak = m;
    g.B = c->TL;
    g.sbk = 1;
    g.sbn = m;
    g.C = c->Tmp;
    g.ldc = m;
    CK(gemm<double>(g, st, c->ws));
    GemmDesc<double> h;   // Hp (2k x 2k) = M(W)^T Tmp
    h.M = 2 * k;
    h.N = 2 * k;
    h.K = m;
    h.A = c->TL;
    h.sak = 1;
    h.sam = m;
    h.B = c->Tmp;
    h.sbk = 1;
    h.sbn = m;
    h.C = c->Hp;
    h.ldc = m;
    CK(gemm<double>(h, st, c->ws));
  }
  CK(symmetrize(c->Hp, m, 2 * k, st));
  CK(syev_traced(c->Hp, m, 2 * k, c->w, c->E, m, st, c->ws_eig, &sweeps, &c->jacobi_unconv,
                 c->h_flags + 8, c->ev_jac));
  if (c->jacobi_unconv) c->flags |= 2;
  c->last_sweeps += sweeps;
  {
    std::vector<double> hw(2 * k);
    CK(hipMemcpyAsync(hw.data(), c->w, 2 * k * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    chfsi_status fs = fix_pair_clusters(c, c->E, m, k, k, hw.data());
    if (fs != CHFSI_OK) return fs;
  }
  {
    GemmDesc<double> g;   // T (2b x 2k) = M(W) E: the embedded Ritz coefficient vectors
    g.M = m;
    g.N = 2 * k;
    g.K = 2 * k;
    g.A = c->TL;
    g.sam = 1;
    g.sak = m;
    g.B = c->E;
    g.sbk = 1;
    g.sbn = m;
    g.C = c->T;
    g.ldc = m;
    CK(gemm<double>(g, st, c->ws));
  }
  chfsi_status s = tail(k);
  if (s != CHFSI_OK || k == b) return s;
  // refill the dropped columns (interleaved: 2n doubles each) and repeat once
  c->refill_seed += 1;
  CK(fill_gaussian(X + 2 * k * ldx, 2 * ldx, 2 * n, b - k,
                   c->prm.seed * 7919 + c->refill_seed, st));
  double* tmp = c->Yw;   // free scratch: the input block is no longer needed
  if (tmp == Y) tmp = const_cast<double*>(Y);
  s = rayleigh_ritz_complex(c, X, ldx, tmp, n, R, ldr, ritz, resnorm, false);
  if (s != CHFSI_OK) return s;
  CK(copy_block(tmp, 2 * n, X, 2 * ldx, 2 * n, b, st));
  return CHFSI_OK;
}

chfsi_status rayleigh_ritz_complex(chfsi_ctx* c, const double* Y, int64_t ldy, double* X,
                                   int64_t ldx, double* R, int64_t ldr, double* ritz,
                                   double* resnorm, bool allow_svqb) {
  const int64_t n = c->n, b = c->b, m = 2 * b;
  hipStream_t st = c->stream;
  CK(fill_zero(c->dflags, 4 * sizeof(int), st));
  // a Bloch grid context works in the twisted frame (planar D Y)
  if (c->bloch) {
    CK(bloch_to_planar(Y, ldy, n, b, c->Ypl, twist_of(c), st));
    // row ends of Y for the wrap corrections of A Y and B Y
    CK(bloch_edges<double>(c->A, c->Ypl, n, c->redge, m, st));
  } else {
    CK(cplx_to_planar(Y, ldy, n, b, c->Ypl, st));
    CK(cplx_rhs<double>(c->Ypl, n, b, c->Yt, st));
  }
  auto product = [&](bool useB, double* out) -> chfsi_status {
    if (c->bloch) {
      // out = A_tw Y: the periodic stencil on 2b columns plus the wrap correction
      const chfsi_operator& op = useB ? c->B : c->A;
      CK(stencil_apply_f64(op, c->Ypl, n, out, n, m, st));
      CK(bloch_fix<double>(op, nullptr, 1.0, c->Ypl, n, out, n, b, st, nullptr, c->redge));
      return CHFSI_OK;
    }
    GemmDesc<double> g;   // out (n x 2b planar) = L (n x 2n) Y~ (2n x 2b)
    g.M = n;
    g.N = m;
    g.K = 2 * n;
    g.A = useB ? c->LB64 : c->LA64;
    g.sak = 1;
    g.sam = 2 * n;
    g.B = c->Yt;
    g.sbk = 1;
    g.sbn = 2 * n;
    g.C = out;
    g.ldc = n;
    CK(gemm<double>(g, st, c->ws));
    return CHFSI_OK;
  };
  chfsi_status s;
  if ((s = product(false, c->AYpl)) != CHFSI_OK) return s;
  const double* BYpl = c->Ypl;
  if (!c->B_identity) {
    if ((s = product(true, c->BYpl)) != CHFSI_OK) return s;
    BYpl = c->BYpl;
  }
  auto gram = [&](const double* W, double* G) -> chfsi_status {
    // the embedding of G = Y^H W needs only the lower triangles of the four
    // b x b blocks of [Y_r Y_i]^T [W_r W_i]: P11, P22 (one batched product)
    // and P12, P21 (a second, stepping back through W), into Tmp
    for (int h = 0; h < 2; ++h) {
      GemmDesc<double> g;
      g.M = b;
      g.N = b;
      g.K = n;
      g.A = c->Ypl;
      g.sak = 1;
      g.sam = n;
      g.B = h == 0 ? W : W + b * n;
      g.sbk = 1;
      g.sbn = n;
      g.C = c->Tmp + h * 2 * b * b;
      g.ldc = b;
      g.batch = 2;
      g.bsA = b * n;
      g.bsB = h == 0 ? b * n : -b * n;
      g.bsC = b * b;
      g.lower_only = true;
      CK(gemm<double>(g, st, c->ws));
    }
    CK(embed_gram_lower(c->Tmp, b, G, st));
    return CHFSI_OK;
  };
  if ((s = gram(c->AYpl, c->Ga)) != CHFSI_OK) return s;
  if ((s = gram(BYpl, c->Gb)) != CHFSI_OK) return s;
  // Ritz pairs from the first vector of each of the np eigenvalue pairs of the
  // embedded problem (columns 2j of T, eigenvalues in w), then X, R and norms
  auto tail = [&](int64_t np) -> chfsi_status {
    // the embedded eigenvalues come in equal pairs; Ritz value j is pair j
    CK(hipMemcpyAsync(c->h_w, c->w, m * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    double scale = 0.0, split = 0.0;
    for (int64_t j = 0; j < 2 * np; ++j) scale = std::max(scale, std::fabs(c->h_w[j]));
    for (int64_t j = 0; j < np; ++j)
      split = std::max(split, std::fabs(c->h_w[2 * j + 1] - c->h_w[2 * j]));
    if (!(split <= 1e-8 * std::max(scale, 1e-300))) {
      set_error("embedded Ritz values do not come in equal pairs (split %.3e of %.3e): the "
                "projected matrices are not Hermitian to working accuracy",
                split, scale);
      return CHFSI_ERR_NUMERIC;
    }
    std::vector<double> lam(b), dup(m);
    for (int64_t j = 0; j < b; ++j) {
      lam[j] = c->h_w[2 * std::min(j, np - 1)];   // columns past the kept pairs are zero
      dup[j] = dup[b + j] = lam[j];
    }
    CK(hipEventSynchronize(c->ev_stage));
    std::memcpy(c->h_stage, dup.data(), m * sizeof(double));
    CK(hipMemcpyAsync(c->wdup, c->h_stage, m * sizeof(double), hipMemcpyHostToDevice, st));
    CK(hipEventRecord(c->ev_stage, st));
    // X~ = [[x_r, x_i], [-x_i, x_r]] (2b x 2b) from the selected complex vectors
    CK(select_pairs_n(c->T, m, b, np, c->Zx, st));
    CK(cplx_rhs<double>(c->Zx, b, b, c->Xt, st));
    auto rotate = [&](const double* Src, const double* Tmat, double* Dst, double alpha,
                      const double* accum) -> chfsi_status {
      GemmDesc<double> g;   // Dst (n x 2b planar) = alpha Src (n x 2b planar) Tmat (2b x 2b)
      g.M = n;
      g.N = m;
      g.K = m;
      g.A = Src;
      g.sam = 1;
      g.sak = n;
      g.B = Tmat;
      g.sbk = 1;
      g.sbn = m;
      g.C = Dst;
      g.ldc = n;
      g.epi.alpha = alpha;
      if (accum) {
        g.epi.beta = 1.0;
        g.epi.C1 = accum;
        g.epi.ldc1 = n;
      }
      CK(gemm<double>(g, st, c->ws));
      return CHFSI_OK;
    };
    if ((s = rotate(c->Ypl, c->Xt, c->Xpl, 1.0, nullptr)) != CHFSI_OK) return s;
    if (c->bloch && stencil_separable(c->A) && (c->B_identity || stencil_separable(c->B))) {
      // grid operators: R = A_tw X - B_tw X Lambda as one periodic stencil pass
      // over X plus the wrap corrections (instead of rotating A Y and B Y)
      CK(stencil_residual_f64(c->A, c->B_identity ? nullptr : &c->B, c->Xpl, n, c->wdup, c->Rpl,
                              n, m, st));
      CK(bloch_edges<double>(c->A, c->Xpl, n, c->redge, m, st));
      CK(bloch_fix<double>(c->A, nullptr, 1.0, c->Xpl, n, c->Rpl, n, b, st, nullptr, c->redge));
      if (!c->B_identity)
        CK(bloch_fix<double>(c->B, nullptr, -1.0, c->Xpl, n, c->Rpl, n, b, st, c->wdup,
                             c->redge));
    } else {
      if ((s = rotate(c->AYpl, c->Xt, c->Rpl, 1.0, nullptr)) != CHFSI_OK) return s;
      CK(copy_block(c->Xt, m, c->TL, m, m, m, st));
      CK(scale_columns(c->TL, m, m, m, c->wdup, st));
      if ((s = rotate(BYpl, c->TL, c->Rpl, -1.0, c->Rpl)) != CHFSI_OK) return s;
    }
    // residual norms: r_j^2 = ||Re R_j||^2 + ||Im R_j||^2
    CK(column_norms(c->Rpl, n, n, m, c->norms, st));
    CK(check_finite(c->wdup, m, c->dflags + 2, st));
    CK(check_finite(c->norms, m, c->dflags + 2, st));
    if (c->bloch) {
      CK(bloch_from_planar(c->Xpl, n, b, X, ldx, twist_of(c), st));
      CK(bloch_from_planar(c->Rpl, n, b, R, ldr, twist_of(c), st));
    } else {
      CK(planar_to_cplx(c->Xpl, n, b, X, ldx, st));
      CK(planar_to_cplx(c->Rpl, n, b, R, ldr, st));
    }
    CK(hipMemcpyAsync(c->h_norms, c->norms, m * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(c->h_flags, c->dflags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (c->h_flags[2] != 0) {
      set_error("non-finite Ritz value or residual norm");
      return CHFSI_ERR_NUMERIC;
    }
    for (int64_t j = 0; j < b; ++j) {
      ritz[j] = lam[j];
      resnorm[j] = std::sqrt(c->h_norms[j] * c->h_norms[j] + c->h_norms[b + j] * c->h_norms[b + j]);
    }
    return CHFSI_OK;
  };
  // CholQR of the scaled embedded Gram matrix, projected matrix, Jacobi
  CK(scale_gram(c->Gb, m, m, c->Gs, m, c->svec, c->dflags + 1, st));
  CK(copy_block(c->Gs, m, c->Linv, m, m, m, st));      // kept for the SVQB fallback
  CK(potrf_traced(c->Gs, m, m, c->dflags, st, c->ws, c->tri));
  CK(hipMemcpyAsync(c->h_flags, c->dflags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (c->h_flags[1] != 0) {
    set_error("Gram matrix Y^H B Y has a non-positive diagonal (a zero or non-finite column)");
    return CHFSI_ERR_NOT_SPD;
  }
  if (c->h_flags[0] != 0) {
    if (!allow_svqb) {
      set_error("Gram matrix Y^H B Y is not positive definite (pivot %d) after refill",
                c->h_flags[0]);
      return CHFSI_ERR_NOT_SPD;
    }
    return rayleigh_ritz_complex_svqb(c, Y, ldy, X, ldx, R, ldr, ritz, resnorm, tail);
  }
  CK(set_identity(c->Linv, m, m, st));
  CK(trsm_lower_left(c->Gs, m, c->Linv, m, m, m, st, c->ws, c->tri, true));
  CK(scale_sym(c->Ga, m, m, c->svec, c->Hp, m, st));
  {
    GemmDesc<double> g;   // Tmp = Linv Hp
    g.M = m;
    g.N = m;
    g.K = m;
    g.A = c->Linv;
    g.sam = 1;
    g.sak = m;
    g.B = c->Hp;
    g.sbk = 1;
    g.sbn = m;
    g.C = c->Tmp;
    g.ldc = m;
    CK(gemm<double>(g, st, c->ws));
    GemmDesc<double> h;   // Hp = Tmp Linv^T
    h.M = m;
    h.N = m;
    h.K = m;
    h.A = c->Tmp;
    h.sam = 1;
    h.sak = m;
    h.B = c->Linv;
    h.sbn = 1;
    h.sbk = m;
    h.C = c->Hp;
    h.ldc = m;
    CK(gemm<double>(h, st, c->ws));
  }
  CK(symmetrize(c->Hp, m, m, st));
  int sweeps = 0;
  CK(syev_traced(c->Hp, m, m, c->w, c->E, m, st, c->ws_eig, &sweeps, &c->jacobi_unconv,
                 c->h_flags + 8, c->ev_jac));
  if (c->jacobi_unconv) c->flags |= 2;
  c->last_sweeps += sweeps;
  {
    GemmDesc<double> g;   // T = diag(s) Linv^T E
    g.M = m;
    g.N = m;
    g.K = m;
    g.A = c->Linv;
    g.sak = 1;
    g.sam = m;
    g.B = c->E;
    g.sbk = 1;
    g.sbn = m;
    g.C = c->T;
    g.ldc = m;
    g.epi.rowscale = c->svec;
    CK(gemm<double>(g, st, c->ws));
  }
  {
    // equal Ritz values: the coefficient vectors of their eigenspace (columns
    // of T, in the coordinates where Y^H B Y is the metric), made B-orthonormal
    CK(hipMemcpyAsync(c->h_w, c->w, m * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    chfsi_status fs = fix_pair_clusters(c, c->T, m, b, b, c->h_w, c->Gb);
    if (fs != CHFSI_OK) return fs;
  }
  return tail(b);
}

// ---------------------------------------------------------------------------
// Slab-wise Rayleigh-Ritz (memory_mode 1): the same algebra as rayleigh_ritz,
// with A Y and B Y materialised one z-slab at a time.  X is rotated in place.
// ---------------------------------------------------------------------------
chfsi_status slab_grams(chfsi_ctx* c, const double* X, int64_t ldx) {
  const int64_t b = c->b;
  const int nz = c->A.nz, nzs = c->slab_planes;
  const int64_t plane = int64_t(c->A.nx) * c->A.ny;
  hipStream_t st = c->stream;
  for (int z0 = 0; z0 < nz; z0 += nzs) {
    const int cnt = std::min(nzs, nz - z0);
    const int64_t rows = plane * cnt, r0 = plane * z0;
    CK(stencil_apply_slab_f64(c->A, X, ldx, c->S1, rows, b, z0, cnt, st));
    const double* BYs = X + r0;
    int64_t ldby = ldx;
    if (!c->B_identity) {
      CK(stencil_apply_slab_f64(c->B, X, ldx, c->S2, rows, b, z0, cnt, st));
      BYs = c->S2;
      ldby = rows;
    }
    // tiles on and below the diagonal only (the Gram matrices are symmetric)
    for (int which = 0; which < 2; ++which) {
      GemmDesc<double> g;
      g.M = b;
      g.N = b;
      g.K = rows;
      g.A = X + r0;
      g.sak = 1;
      g.sam = ldx;
      g.B = which == 0 ? c->S1 : BYs;
      g.sbk = 1;
      g.sbn = which == 0 ? rows : ldby;
      g.C = which == 0 ? c->Ga : c->Gb;
      g.ldc = b;
      g.lower_only = true;
      if (z0 > 0) {
        g.epi.beta = 1.0;
        g.epi.C1 = g.C;
        g.epi.ldc1 = b;
      }
      CK(gemm<double>(g, st, c->ws));
    }
  }
  CK(symmetrize_panels(c->Ga, b, b, 1, st));
  CK(symmetrize_panels(c->Gb, b, b, 1, st));
  return CHFSI_OK;
}

// X[:, :k] <- X Tm (b x k, ld b), slab by slab in place
chfsi_status slab_rotate(chfsi_ctx* c, double* X, int64_t ldx, const double* Tm, int64_t k) {
  const int64_t b = c->b;
  const int nz = c->A.nz, nzs = c->slab_planes;
  const int64_t plane = int64_t(c->A.nx) * c->A.ny;
  hipStream_t st = c->stream;
  for (int z0 = 0; z0 < nz; z0 += nzs) {
    const int cnt = std::min(nzs, nz - z0);
    const int64_t rows = plane * cnt, r0 = plane * z0;
    GemmDesc<double> g;
    g.M = rows;
    g.N = k;
    g.K = b;
    g.A = X + r0;
    g.sam = 1;
    g.sak = ldx;
    g.B = Tm;
    g.sbk = 1;
    g.sbn = b;
    g.C = c->S1;
    g.ldc = rows;
    CK(gemm<double>(g, st, c->ws));
    CK(copy_block(c->S1, rows, X + r0, ldx, rows, k, st));
  }
  return CHFSI_OK;
}

chfsi_status slab_residual(chfsi_ctx* c, const double* X, int64_t ldx, double* R, int64_t ldr) {
  CK(stencil_residual_f64(c->A, c->B_identity ? nullptr : &c->B, X, ldx, c->w, R, ldr, c->b,
                          c->stream));
  return CHFSI_OK;
}

chfsi_status rayleigh_ritz_slabs(chfsi_ctx* c, double* X, int64_t ldx, double* R, int64_t ldr,
                                 double* ritz, double* resnorm, bool allow_svqb) {
  const int64_t n = c->n, b = c->b;
  hipStream_t st = c->stream;
  chfsi_status s;
  CK(fill_zero(c->dflags, 4 * sizeof(int), st));
  if ((s = slab_grams(c, X, ldx)) != CHFSI_OK) return s;
  CK(scale_gram(c->Gb, b, b, c->Gs, b, c->svec, c->dflags + 1, st));
  CK(copy_block(c->Gs, b, c->Linv, b, b, b, st));
  CK(potrf_traced(c->Gs, b, b, c->dflags, st, c->ws, c->tri));
  CK(hipMemcpyAsync(c->h_flags, c->dflags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (c->h_flags[1] != 0) {
    set_error("Gram matrix Y^T B Y has a non-positive diagonal (a zero or non-finite column)");
    return CHFSI_ERR_NOT_SPD;
  }
  int sweeps = 0;
  if (c->h_flags[0] == 0) {
    CK(set_identity(c->Linv, b, b, st));
    CK(trsm_lower_left(c->Gs, b, c->Linv, b, b, b, st, c->ws, c->tri, true));
    CK(scale_sym(c->Ga, b, b, c->svec, c->Hp, b, st));
    GemmDesc<double> g;
    g.M = b;
    g.N = b;
    g.K = b;
    g.A = c->Linv;
    g.sam = 1;
    g.sak = b;
    g.B = c->Hp;
    g.sbk = 1;
    g.sbn = b;
    g.C = c->Tmp;
    g.ldc = b;
    CK(gemm<double>(g, st, c->ws));
    GemmDesc<double> h;
    h.M = b;
    h.N = b;
    h.K = b;
    h.A = c->Tmp;
    h.sam = 1;
    h.sak = b;
    h.B = c->Linv;
    h.sbn = 1;
    h.sbk = b;
    h.C = c->Hp;
    h.ldc = b;
    CK(gemm<double>(h, st, c->ws));
    CK(symmetrize(c->Hp, b, b, st));
    CK(syev_traced(c->Hp, b, b, c->w, c->E, b, st, c->ws_eig, &sweeps, &c->jacobi_unconv,
                 c->h_flags + 8, c->ev_jac));
  if (c->jacobi_unconv) c->flags |= 2;
    c->last_sweeps += sweeps;
    GemmDesc<double> t;
    t.M = b;
    t.N = b;
    t.K = b;
    t.A = c->Linv;
    t.sak = 1;
    t.sam = b;
    t.B = c->E;
    t.sbk = 1;
    t.sbn = b;
    t.C = c->T;
    t.ldc = b;
    t.epi.rowscale = c->svec;
    CK(gemm<double>(t, st, c->ws));
    if ((s = slab_rotate(c, X, ldx, c->T, b)) != CHFSI_OK) return s;
    if ((s = slab_residual(c, X, ldx, R, ldr)) != CHFSI_OK) return s;
    return finish_rr(c, R, ldr, ritz, resnorm);
  }
  if (!allow_svqb) {
    set_error("Gram matrix Y^T B Y is not positive definite (pivot %d) after refill",
              c->h_flags[0]);
    return CHFSI_ERR_NOT_SPD;
  }
  // SVQB on the scaled Gram matrix kept in c->Linv (same reading as rayleigh_ritz_svqb)
  CK(syev_traced(c->Linv, b, b, c->w, c->E, b, st, c->ws_eig, &sweeps, &c->jacobi_unconv,
                 c->h_flags + 8, c->ev_jac));
  if (c->jacobi_unconv) c->flags |= 2;
  c->last_sweeps += sweeps;
  CK(hipMemcpyAsync(c->h_w, c->w, b * sizeof(double), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  const double gmax = c->h_w[b - 1];
  int64_t first = 0;
  while (first < b && !(c->h_w[first] > 1e-14 * gmax)) ++first;
  const int64_t k = b - first;
  if (k <= 0) {
    set_error("Gram matrix Y^T B Y is numerically zero");
    return CHFSI_ERR_NOT_SPD;
  }
  c->flags |= 1;
  c->svqb_events += 1;
  c->svqb_dropped += int(b - k);
  std::vector<double> colv(k);
  for (int64_t j = 0; j < k; ++j) colv[j] = 1.0 / std::sqrt(c->h_w[first + j]);
  CK(hipEventSynchronize(c->ev_stage));
  std::memcpy(c->h_stage, colv.data(), k * sizeof(double));
  CK(hipMemcpyAsync(c->lamY, c->h_stage, k * sizeof(double), hipMemcpyHostToDevice, st));
  CK(hipEventRecord(c->ev_stage, st));
  CK(copy_block(c->E + first * b, b, c->T, b, b, k, st));
  CK(scale_columns(c->T, b, b, k, c->lamY, st));
  CK(scale_rows(c->T, b, b, k, c->svec, st));
  {
    GemmDesc<double> g;
    g.M = b;
    g.N = k;
    g.K = b;
    g.A = c->Ga;
    g.sam = 1;
    g.sak = b;
    g.B = c->T;
    g.sbk = 1;
    g.sbn = b;
    g.C = c->Tmp;
    g.ldc = b;
    CK(gemm<double>(g, st, c->ws));
    GemmDesc<double> h;
    h.M = k;
    h.N = k;
    h.K = b;
    h.A = c->T;
    h.sak = 1;
    h.sam = b;
    h.B = c->Tmp;
    h.sbk = 1;
    h.sbn = b;
    h.C = c->Hp;
    h.ldc = b;
    CK(gemm<double>(h, st, c->ws));
  }
  CK(symmetrize(c->Hp, b, k, st));
  CK(syev_traced(c->Hp, b, k, c->w, c->E, b, st, c->ws_eig, &sweeps, &c->jacobi_unconv,
                 c->h_flags + 8, c->ev_jac));
  if (c->jacobi_unconv) c->flags |= 2;
  c->last_sweeps += sweeps;
  {
    GemmDesc<double> g;
    g.M = b;
    g.N = k;
    g.K = k;
    g.A = c->T;
    g.sam = 1;
    g.sak = b;
    g.B = c->E;
    g.sbk = 1;
    g.sbn = b;
    g.C = c->Linv;
    g.ldc = b;
    CK(gemm<double>(g, st, c->ws));
  }
  if ((s = slab_rotate(c, X, ldx, c->Linv, k)) != CHFSI_OK) return s;
  c->refill_seed += 1;
  if (k < b)
    CK(fill_gaussian(X + k * ldx, ldx, n, b - k, c->prm.seed * 7919 + c->refill_seed, st));
  return rayleigh_ritz_slabs(c, X, ldx, R, ldr, ritz, resnorm, false);
}

// Lanczos estimate of the spectrum bounds of B^{-1} A (lanczos.hip) on the
// context's operators: real blocks of length n, or planar complex vectors of
// length 2 n ([re; im], the Bloch operators in the twisted frame)
// the estimate's vectors (allocated on first use)
chfsi_status ensure_lanczos_work(chfsi_ctx* c) {
  if (c->lz_work) return CHFSI_OK;
  chfsi_status ls = CHFSI_OK;
  c->lz_work = ctx_alloc<double>(c, lanczos_ctx_bytes(c->n, c->cplx), &ls);
  return ls;
}

// stream: where the estimate runs (null: the context's stream)
chfsi_status estimate_bounds(chfsi_ctx* c, const double* v0_user, int steps, LanczosResult* res,
                             hipStream_t stream = nullptr) {
  TraceRange tr("chfsi lanczos bound estimate");
  const int64_t n = c->n;
  const int64_t L = c->cplx ? 2 * n : n;
  hipStream_t st = stream ? stream : c->stream;
  {
    const chfsi_status ls = ensure_lanczos_work(c);
    if (ls != CHFSI_OK) return ls;
  }
  double* tmp = c->lz_work + (lanczos_workspace_bytes(L) + 255) / 256 * 256 / sizeof(double);
  double* v0 = tmp;            // L
  double* dl = tmp + L;        // L: D^{-1} on planar complex vectors
  double* Yt = tmp + 2 * L;    // 4 n: right operand of the dense Hermitian product
  if (v0_user) {
    if (c->bloch)
      CK(bloch_to_planar(v0_user, n, n, 1, v0, twist_of(c), st));
    else if (c->cplx)
      CK(cplx_to_planar(v0_user, n, n, 1, v0, st));
    else
      CK(copy_block(v0_user, n, v0, n, n, 1, st));
  } else {
    CK(fill_gaussian(v0, L, L, 1, c->prm.seed ^ 0x4c414e43u, st));
  }
  const double* dinv = c->dinv;
  if (c->cplx && c->dinv) {
    CK(dup_dinv<double>(c->dinv, n, dl, st));
    dinv = dl;
  }
  auto apply = [c, st, n, Yt](const chfsi_operator& op, bool useB, const double* x,
                              double* y) -> hipError_t {
    if (c->bloch) {
      hipError_t e = stencil_apply_f64(op, x, n, y, n, 2, st);
      if (e != hipSuccess) return e;
      return bloch_fix<double>(op, nullptr, 1.0, x, n, y, n, 1, st, nullptr, nullptr);
    }
    if (c->cplx) {
      hipError_t e = cplx_rhs<double>(x, n, 1, Yt, st);
      if (e != hipSuccess) return e;
      GemmDesc<double> g;   // y (n x 2 planar) = L (n x 2n) Yt (2n x 2)
      g.M = n;
      g.N = 2;
      g.K = 2 * n;
      g.A = useB ? c->LB64 : c->LA64;
      g.sak = 1;
      g.sam = 2 * n;
      g.B = Yt;
      g.sbk = 1;
      g.sbn = 2 * n;
      g.C = y;
      g.ldc = n;
      return gemm<double>(g, st, c->ws);
    }
    if (op.kind == CHFSI_OP_DENSE) return gemv_rows_f64(op.dense, op.ld, n, x, y, st);
    if (op.kind == CHFSI_OP_STENCIL27) return stencil_apply_f64(op, x, n, y, n, 1, st);
    if (op.kind == CHFSI_OP_CSR) return csr_apply_f64(csr_of(c, op, false), x, n, y, n, 1, st);
    return hipErrorInvalidValue;
  };
  LanczosOps ops;
  ops.apply_A = [&](const double* x, double* y) { return apply(c->A, false, x, y); };
  if (!c->B_identity)
    ops.apply_B = [&](const double* x, double* y) { return apply(c->B, true, x, y); };
  ops.dinv = dinv;
  ops.v0 = v0;
  ops.steps = steps > 0 ? steps : (c->prm.lanczos_steps > 0 ? c->prm.lanczos_steps : 12);
  const hipError_t e = lanczos_bounds(ops, L, c->lz_work, c->h_lz, st, res);
  if (e == hipErrorInvalidValue) {
    set_error("Lanczos bound estimate: B is not positive definite on the Krylov space "
              "(or the start vector is zero)");
    return CHFSI_ERR_NOT_SPD;
  }
  CK(e);
  if (!std::isfinite(res->upper) || !std::isfinite(res->lower)) {
    set_error("Lanczos bound estimate is not finite");
    return CHFSI_ERR_NUMERIC;
  }
  return CHFSI_OK;
}

// overlap the estimate with the first Rayleigh-Ritz pass: dense real operators
// whose memory the library allocates itself (knob CHFSI_LANCZOS_OVERLAP=0: off)
bool lanczos_overlap_ok(const chfsi_ctx* c) {
  const char* e = std::getenv("CHFSI_LANCZOS_OVERLAP");
  if (e && std::atoi(e) == 0) return false;
  return !c->cplx && !c->bloch && c->al == nullptr && c->A.kind == CHFSI_OP_DENSE &&
         (c->B_identity || c->B.kind == CHFSI_OP_DENSE);
}

void bounds_policy(const chfsi_params& p, double lmax_used, const double* ritz, int64_t b,
                   double* lmin, double* lmax, double* lT) {
  *lmax = lmax_used;
  const double e1 = ritz[0], eb = ritz[b - 1];
  *lmin = std::isnan(p.lambda_min) ? e1 - 0.05 * (eb - e1) : p.lambda_min;
  *lT = std::isnan(p.lambda_T) ? eb : p.lambda_T;
}

// Amplification of one pass (Section 3.1's condition): the filter maps
// [lT, lmax] onto [-1, 1] by L(x) = (x - c) / e, c = (lT + lmax) / 2,
// e = (lmax - lT) / 2, and scales the lowest part of the spectrum by up to
// T_p(|L(lmin)|) = cosh(p acosh |L(lmin)|) relative to it.  With amp_cap > 0
// the pass uses the largest p' <= p whose amplification stays within the cap
// (at least 1).  Returns the degree; *amp receives its amplification.
int pass_degree(const chfsi_params& prm, double lmin, double lmax, double lT, double* amp) {
  const double cc = 0.5 * (lT + lmax), e = 0.5 * (lmax - lT);
  const double ax = std::acosh(std::max(std::fabs((lmin - cc) / e), 1.0));
  int p = prm.degree;
  if (prm.amp_cap > 0.0 && ax > 0.0) {
    const double pmax = std::acosh(std::max(prm.amp_cap, 1.0)) / ax;
    if (pmax < double(p)) p = std::max(1, int(std::floor(pmax)));
  }
  *amp = std::cosh(double(p) * ax);
  return p;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// H^T = A B^{-1} for the exact-inverse plain filter (Algorithm 2 with
// H = B^{-1} A): B = L L^T (blocked Cholesky), L^{-1} by a triangular solve
// on the identity, B^{-1} = L^{-T} L^{-1} and A B^{-1} as FP64 products.  The
// n x n temporaries are the function's own and freed before it returns.
chfsi_status form_exact_operator(chfsi_ctx* c, const chfsi_operator* A, const chfsi_operator* B) {
  const int64_t n = c->n;
  hipStream_t st = c->stream;
  const size_t bytes = size_t(n) * n * sizeof(double);
  double *L = nullptr, *Li = nullptr, *tri = nullptr;
  int* info = nullptr;
  auto release = [&]() {
    if (L) (void)hipFree(L);
    if (Li) (void)hipFree(Li);
    if (tri) (void)hipFree(tri);
    if (info) (void)hipFree(info);
  };
  if (hipMalloc(&L, bytes) != hipSuccess || hipMalloc(&Li, bytes) != hipSuccess ||
      hipMalloc(&tri, tri_workspace_bytes(n, n)) != hipSuccess ||
      hipMalloc(&info, 64) != hipSuccess) {
    release();
    set_error("hipMalloc failed for the exact inverse (3 n^2 doubles)");
    return CHFSI_ERR_NOMEM;
  }
  chfsi_status s = CHFSI_OK;
  auto run = [&]() -> chfsi_status {
    CK(copy_block(B->dense, B->ld, L, n, n, n, st));
    CK(fill_zero(info, sizeof(int), st));
    CK(potrf_lower(L, n, n, info, st, c->ws, tri));
    int h_info = 0;
    CK(hipMemcpyAsync(&h_info, info, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (h_info != 0) {
      set_error("B is not positive definite (Cholesky pivot %d)", h_info);
      return CHFSI_ERR_NOT_SPD;
    }
    CK(set_identity(Li, n, n, st));
    CK(trsm_lower_left(L, n, Li, n, n, n, st, c->ws, tri, true));
    {
      GemmDesc<double> g;   // B^{-1} = L^{-T} L^{-1}, into L
      g.M = n;
      g.N = n;
      g.K = n;
      g.A = Li;             // A(m, k) = L^{-1}(k, m)
      g.sak = 1;
      g.sam = n;
      g.B = Li;
      g.sbk = 1;
      g.sbn = n;
      g.C = L;
      g.ldc = n;
      CK(gemm<double>(g, st, c->ws));
      GemmDesc<double> h;   // H^T = A B^{-1}
      h.M = n;
      h.N = n;
      h.K = n;
      h.A = A->dense;       // A symmetric: A(m, k) = dense[k + m ld]
      h.sak = 1;
      h.sam = A->ld;
      h.B = L;
      h.sbk = 1;
      h.sbn = n;
      h.C = c->Ht;
      h.ldc = n;
      CK(gemm<double>(h, st, c->ws));
    }
    CK(hipStreamSynchronize(st));
    return CHFSI_OK;
  };
  s = run();
  release();
  return s;
}

extern "C" {

const char* chfsi_last_error(void) { return g_last_error.c_str(); }

const char* chfsi_version(void) { return "libchfsi 0.1 (gfx950)"; }

size_t chfsi_workspace_bytes(const chfsi_operator* A, const chfsi_operator* B,
                             const chfsi_params* params) {
  if (check_params(A, B, params) != CHFSI_OK) return 0;
  return plan_sizes(A, B, params).total;
}

void chfsi_destroy(chfsi_ctx* c) {
  if (!c) return;
  if (c->stream) hipStreamSynchronize(c->stream);
  for (void* p : c->allocs) {
    if (c->al)
      c->al->dev_free(c->al->self, p);
    else
      hipFree(p);
  }
  for (void* h : {static_cast<void*>(c->h_w), static_cast<void*>(c->h_norms),
                  static_cast<void*>(c->h_flags), c->h_stage, static_cast<void*>(c->h_lz)}) {
    if (!h) continue;
    if (c->al)
      c->al->host_free(c->al->self, h);
    else
      hipHostFree(h);
  }
  for (auto& e : c->ev)
    if (e) hipEventDestroy(e);
  if (c->ev_stage) hipEventDestroy(c->ev_stage);
  if (c->ev_jac) hipEventDestroy(c->ev_jac);
  if (c->aux_stream) {
    hipStreamSynchronize(c->aux_stream);
    hipStreamDestroy(c->aux_stream);
  }
  if (c->ev_aux) hipEventDestroy(c->ev_aux);
  for (auto e : c->pev)
    if (e) hipEventDestroy(e);
  delete c;
}

chfsi_status chfsi_create(chfsi_ctx** out, const chfsi_operator* A, const chfsi_operator* B,
                          const double* d_inv, const chfsi_params* params, void* stream) {
  return chfsi::create_with_allocator(out, A, B, d_inv, params, stream, nullptr);
}

}  // extern "C"

chfsi_status chfsi::create_with_allocator(chfsi_ctx** out, const chfsi_operator* A,
                                          const chfsi_operator* B, const double* d_inv,
                                          const chfsi_params* params, void* stream,
                                          const Allocator* al) {
  if (!out) {
    set_error("out must be non-null");
    return CHFSI_ERR_ARG;
  }
  *out = nullptr;
  chfsi_status st = check_params(A, B, params);
  if (st != CHFSI_OK) return st;
  if (std::isinf(params->lambda_max) || std::isinf(params->lambda_min) ||
      std::isinf(params->lambda_T)) {
    set_error("filter bounds must be finite or NaN (NaN: estimated)");
    return CHFSI_ERR_ARG;
  }
  if (params->lanczos_steps < 0 || params->stall_iters < 0) {
    set_error("lanczos_steps and stall_iters must be >= 0");
    return CHFSI_ERR_ARG;
  }
  if (!(params->amp_cap >= 0.0)) {
    set_error("amp_cap must be >= 0 (0: no cap)");
    return CHFSI_ERR_ARG;
  }
  if (params->escalate != 0 &&
      (params->escalate != 1 || params->stall_iters <= 0 ||
       params->filter_prec != CHFSI_PREC_BF16 || params->method != CHFSI_METHOD_RCHFSI ||
       (A->kind != CHFSI_OP_DENSE && A->kind != CHFSI_OP_STENCIL27 && A->kind != CHFSI_OP_CSR))) {
    set_error("escalate needs stall_iters > 0 and a BF16 residual filter on a real operator");
    return CHFSI_ERR_ARG;
  }
  chfsi_ctx* c = new chfsi_ctx();
  c->al = al;
  c->stream = static_cast<hipStream_t>(stream);
  hipGetDevice(&c->device);
  c->A = *A;
  c->B_identity = is_identity(B);
  if (!c->B_identity) c->B = *B;
  c->B.kind = c->B_identity ? CHFSI_OP_IDENTITY : B->kind;
  c->dinv = d_inv;
  c->prm = *params;
  c->n = A->n;
  c->b = params->block;
  const int64_t n = c->n, b = c->b;
  const SizePlan sp = plan_sizes(A, B, params);
  st = CHFSI_OK;
  const bool dense = A->kind == CHFSI_OP_DENSE;
  c->bloch = A->kind == CHFSI_OP_STENCIL27_BLOCH;
  c->cplx = A->kind == CHFSI_OP_DENSE_HERMITIAN || c->bloch;
  if (c->cplx) {
    // dense: planar operator copy, [d; d], Z~ (and its bfloat16 copy); grid:
    // FP32 copies of D^{-1} and V for FP32/BF16 filters.  Three planar filter
    // blocks and the coefficient tables for 2b columns.
    const bool f64 = params->filter_prec == CHFSI_PREC_FP64;
    const size_t el = f64 ? sizeof(double) : sizeof(float);
    const size_t lel = params->filter_prec == CHFSI_PREC_BF16 ? sizeof(uint16_t) : el;
    if (c->bloch) {
      if (!f64 && d_inv) c->dinv32 = ctx_alloc<float>(c, size_t(n) * sizeof(float), &st);
      if (!f64 && A->field_mode != 0) c->Vf = ctx_alloc<float>(c, size_t(n) * sizeof(float), &st);
      // leading dimension of the correction: the boundary point count rounded
      // up to a multiple of 4 (aligned vector loads in the z-march)
      c->nbnd = (bloch_boundary_points(A->nx, A->ny, A->nz) + 3) / 4 * 4;
      c->bcorr = ctx_alloc<char>(c, size_t(c->nbnd) * 2 * b * el, &st);
      const size_t sel = params->filter_prec == CHFSI_PREC_BF16 ? sizeof(uint16_t) : el;
      for (auto& e : c->bedge)
        e = ctx_alloc<char>(c, size_t(2) * A->ny * A->nz * 2 * b * sel, &st);
      c->redge = ctx_alloc<double>(c, size_t(2) * A->ny * A->nz * 2 * b * sizeof(double), &st);
    } else {
      c->Lc = ctx_alloc<char>(c, size_t(n) * 2 * n * lel, &st);
      c->dinv2 = ctx_alloc<char>(c, size_t(2) * n * el, &st);
      size_t zt = size_t(2) * n * 2 * b * el;
      if (params->filter_prec == CHFSI_PREC_BF16) zt += size_t(2) * n * 2 * b * sizeof(uint16_t);
      c->Zt = ctx_alloc<char>(c, zt, &st);
    }
    if (f64) {
      c->f64_a = ctx_alloc<double>(c, sp.f32blk, &st);
      c->f64_b = ctx_alloc<double>(c, sp.f32blk, &st);
      c->f64_c = ctx_alloc<double>(c, sp.f32blk, &st);
    } else if (c->bloch && params->filter_prec == CHFSI_PREC_BF16) {
      c->bf_a = ctx_alloc<char>(c, sp.f32blk, &st);
      c->bf_b = ctx_alloc<char>(c, sp.f32blk, &st);
      c->bf_c = ctx_alloc<char>(c, sp.f32blk, &st);
    } else {
      c->f32_a = ctx_alloc<float>(c, sp.f32blk, &st);
      c->f32_b = ctx_alloc<float>(c, sp.f32blk, &st);
      c->f32_c = ctx_alloc<float>(c, sp.f32blk, &st);
    }
    c->coef_cap = params->degree;
    c->coef32 = ctx_alloc<float>(c, size_t(params->degree) * 2 * b * sizeof(float), &st);
    c->coef64 = ctx_alloc<double>(c, size_t(params->degree) * 2 * b * sizeof(double), &st);
    c->lamY = ctx_alloc<double>(c, b * sizeof(double), &st);
    c->h_coef32.assign(size_t(params->degree) * 2 * b, 0.0f);
    c->h_coef64.assign(size_t(params->degree) * 2 * b, 0.0);
    c->ws.bytes = sp.ws;
    c->ws.ptr = ctx_alloc<char>(c, sp.ws, &st);
    // Rayleigh-Ritz (FP64) on the real embedding of the 2b x 2b projected pencil
    const int64_t m = 2 * b;
    if (!c->bloch) {
      c->LA64 = f64 ? static_cast<double*>(c->Lc)
                    : ctx_alloc<double>(c, size_t(n) * 2 * n * sizeof(double), &st);
      if (!c->B_identity)
        c->LB64 = ctx_alloc<double>(c, size_t(n) * 2 * n * sizeof(double), &st);
    }
    c->Ypl = ctx_alloc<double>(c, sp.blk, &st);
    c->AYpl = ctx_alloc<double>(c, sp.blk, &st);
    c->BYpl = c->B_identity ? nullptr : ctx_alloc<double>(c, sp.blk, &st);
    c->Xpl = ctx_alloc<double>(c, sp.blk, &st);
    c->Rpl = ctx_alloc<double>(c, sp.blk, &st);
    if (!c->bloch) c->Yt = ctx_alloc<double>(c, size_t(2) * n * m * sizeof(double), &st);
    c->Xw = ctx_alloc<double>(c, sp.blk, &st);
    c->Yw = ctx_alloc<double>(c, sp.blk, &st);
    c->R = ctx_alloc<double>(c, sp.blk, &st);
    c->Ga = ctx_alloc<double>(c, sp.bb, &st);
    c->Gb = ctx_alloc<double>(c, sp.bb, &st);
    c->Gs = ctx_alloc<double>(c, sp.bb, &st);
    c->Linv = ctx_alloc<double>(c, sp.bb, &st);
    c->Tmp = ctx_alloc<double>(c, sp.bb, &st);
    c->Hp = ctx_alloc<double>(c, sp.bb, &st);
    c->E = ctx_alloc<double>(c, sp.bb, &st);
    c->T = ctx_alloc<double>(c, sp.bb, &st);
    c->TL = ctx_alloc<double>(c, sp.bb, &st);
    c->Xt = ctx_alloc<double>(c, sp.bb, &st);
    c->Zx = ctx_alloc<double>(c, sp.bb, &st);
    c->gs_work = ctx_alloc<double>(c, cluster_gs_work_bytes(b, b), &st);
    c->svec = ctx_alloc<double>(c, m * sizeof(double), &st);
    c->w = ctx_alloc<double>(c, m * sizeof(double), &st);
    c->norms = ctx_alloc<double>(c, m * sizeof(double), &st);
    c->wdup = ctx_alloc<double>(c, m * sizeof(double), &st);
    c->dflags = ctx_alloc<int>(c, 64, &st);
    c->tri = ctx_alloc<double>(c, sp.tri, &st);
    c->ws_eig.bytes = sp.ws_eig;
    c->ws_eig.ptr = ctx_alloc<char>(c, sp.ws_eig, &st);
  } else if (params->filter_prec == CHFSI_PREC_FP32) {
    if (dense) c->A32 = ctx_alloc<float>(c, size_t(n) * n * sizeof(float), &st);
    if (dense || d_inv) c->dinv32 = ctx_alloc<float>(c, size_t(n) * sizeof(float), &st);
    c->f32_a = ctx_alloc<float>(c, sp.f32blk, &st);
    c->f32_b = ctx_alloc<float>(c, sp.f32blk, &st);
    c->f32_c = ctx_alloc<float>(c, sp.f32blk, &st);
  } else if (params->filter_prec == CHFSI_PREC_FP64) {
    c->f64_a = ctx_alloc<double>(c, sp.f64blk, &st);
    c->f64_b = ctx_alloc<double>(c, sp.f64blk, &st);
  } else if (dense) {
    c->A16 = ctx_alloc<uint16_t>(c, size_t(n) * n * sizeof(uint16_t), &st);
    if (params->escalate) c->A32 = ctx_alloc<float>(c, size_t(n) * n * sizeof(float), &st);
    c->bf_a = ctx_alloc<char>(c, size_t(n) * b * sizeof(uint16_t), &st);   // bf16(D^-1 R_Y)
    c->dinv32 = ctx_alloc<float>(c, size_t(n) * sizeof(float), &st);
    c->f32_a = ctx_alloc<float>(c, sp.f32blk, &st);
    c->f32_b = ctx_alloc<float>(c, sp.f32blk, &st);
    c->f32_c = ctx_alloc<float>(c, sp.f32blk, &st);
  } else if (params->escalate) {
    // FP32 blocks for the escalated passes; the BF16 blocks live in their first halves
    if (d_inv) c->dinv32 = ctx_alloc<float>(c, size_t(n) * sizeof(float), &st);
    c->f32_a = ctx_alloc<float>(c, sp.f32blk, &st);
    c->f32_b = ctx_alloc<float>(c, sp.f32blk, &st);
    c->f32_c = ctx_alloc<float>(c, sp.f32blk, &st);
    c->bf_a = c->f32_a;
    c->bf_b = c->f32_b;
    c->bf_c = c->f32_c;
  } else {
    if (d_inv) c->dinv32 = ctx_alloc<float>(c, size_t(n) * sizeof(float), &st);
    c->bf_a = ctx_alloc<char>(c, sp.bfblk, &st);
    c->bf_b = ctx_alloc<char>(c, sp.bfblk, &st);
    c->bf_c = ctx_alloc<char>(c, sp.bfblk, &st);
  }
  if (!c->cplx) {
  if (A->kind == CHFSI_OP_STENCIL27 && params->filter_prec != CHFSI_PREC_FP64 &&
      A->field_mode != 0)
    c->Vf = ctx_alloc<float>(c, size_t(n) * sizeof(float), &st);
  if (A->kind == CHFSI_OP_CSR && params->filter_prec != CHFSI_PREC_FP64)
    c->val32 = ctx_alloc<float>(c, size_t(std::max<int64_t>(A->nnz, 1)) * sizeof(float), &st);
  if (params->binv_exact) c->Ht = ctx_alloc<double>(c, size_t(n) * n * sizeof(double), &st);
  c->coef_cap = params->degree;
  c->coef32 = ctx_alloc<float>(c, size_t(params->degree) * b * sizeof(float), &st);
  c->coef64 = ctx_alloc<double>(c, size_t(params->degree) * b * sizeof(double), &st);
  c->lamY = ctx_alloc<double>(c, b * sizeof(double), &st);
  c->ritz_d = ctx_alloc<double>(c, b * sizeof(double), &st);
  c->tri = ctx_alloc<double>(c, sp.tri, &st);
  if (params->memory_mode == 1) {
    c->slab_planes = sp.slab_planes;
    c->R = ctx_alloc<double>(c, sp.blk, &st);
    c->S1 = ctx_alloc<double>(c, sp.slab, &st);
    c->S2 = ctx_alloc<double>(c, sp.slab, &st);
  } else {
    c->Yw = ctx_alloc<double>(c, sp.blk, &st);
    c->Xw = ctx_alloc<double>(c, sp.blk, &st);
    c->AY = ctx_alloc<double>(c, sp.blk, &st);
    c->R = ctx_alloc<double>(c, sp.blk, &st);
    if (!c->B_identity) c->BY = ctx_alloc<double>(c, sp.blk, &st);
  }
  c->Ga = ctx_alloc<double>(c, sp.bb, &st);
  c->Gb = ctx_alloc<double>(c, sp.bb, &st);
  c->Gs = ctx_alloc<double>(c, sp.bb, &st);
  c->Linv = ctx_alloc<double>(c, sp.bb, &st);
  c->Tmp = ctx_alloc<double>(c, sp.bb, &st);
  c->Hp = ctx_alloc<double>(c, sp.bb, &st);
  c->E = ctx_alloc<double>(c, sp.bb, &st);
  c->T = ctx_alloc<double>(c, sp.bb, &st);
  c->TL = ctx_alloc<double>(c, sp.bb, &st);
  c->svec = ctx_alloc<double>(c, b * sizeof(double), &st);
  c->w = ctx_alloc<double>(c, b * sizeof(double), &st);
  c->norms = ctx_alloc<double>(c, b * sizeof(double), &st);
  c->dflags = ctx_alloc<int>(c, 64, &st);
  c->ws.bytes = sp.ws;
  c->ws.ptr = ctx_alloc<char>(c, sp.ws, &st);
  c->ws_eig.bytes = sp.ws_eig;
  c->ws_eig.ptr = ctx_alloc<char>(c, sp.ws_eig, &st);
  }
  if (st != CHFSI_OK) {
    chfsi_destroy(c);
    return st;
  }
  c->h_stage_bytes = b * sizeof(double) + size_t(params->degree) * (c->cplx ? 2 : 1) * b *
                                                sizeof(double) + 64;
  const int64_t hb = c->cplx ? 2 * b : b;
  auto pinned = [c](void** p, size_t bytes) -> bool {
    if (c->al) {
      *p = c->al->host_alloc(c->al->self, bytes);
      return *p != nullptr;
    }
    return hipHostMalloc(p, bytes) == hipSuccess;
  };
  if (!pinned(reinterpret_cast<void**>(&c->h_w), hb * sizeof(double)) ||
      !pinned(reinterpret_cast<void**>(&c->h_norms), hb * sizeof(double)) ||
      !pinned(reinterpret_cast<void**>(&c->h_flags), 64) ||
      !pinned(&c->h_stage, c->h_stage_bytes) ||
      !pinned(reinterpret_cast<void**>(&c->h_lz), 64)) {
    set_error("pinned host allocation failed");
    chfsi_destroy(c);
    return CHFSI_ERR_NOMEM;
  }
  if (hipEventCreateWithFlags(&c->ev_stage, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_jac, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(c->ev_stage, c->stream) != hipSuccess) {
    set_error("hipEventCreate failed");
    chfsi_destroy(c);
    return CHFSI_ERR_DEVICE;
  }
  for (auto& e : c->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      set_error("hipEventCreate failed");
      chfsi_destroy(c);
      return CHFSI_ERR_DEVICE;
    }
  }
  if (params->profile) {
    c->pev.assign(size_t(8) * (params->degree + 1), nullptr);
    for (auto& e : c->pev)
      if (hipEventCreate(&e) != hipSuccess) {
        set_error("hipEventCreate failed");
        chfsi_destroy(c);
        return CHFSI_ERR_DEVICE;
      }
  }
  // precision-converted operator copies (owned)
  hipError_t e = hipSuccess;
  if (c->cplx && !c->bloch) {
    // FP64 planar A (Rayleigh-Ritz; also the FP64 filter's operand) and B
    e = herm_to_planar<double>(A->dense, A->ld, n, c->LA64, c->stream);
    if (e == hipSuccess && c->LB64) e = herm_to_planar<double>(B->dense, B->ld, n, c->LB64, c->stream);
    // the filter's operand in its precision, and [d; d]
    if (e == hipSuccess && params->filter_prec == CHFSI_PREC_FP64)
      e = dup_dinv<double>(d_inv, n, static_cast<double*>(c->dinv2), c->stream);
    if (e == hipSuccess && params->filter_prec == CHFSI_PREC_FP32)
      e = herm_to_planar<float>(A->dense, A->ld, n, static_cast<float*>(c->Lc), c->stream);
    if (e == hipSuccess && params->filter_prec == CHFSI_PREC_BF16)
      e = herm_to_planar<uint16_t>(A->dense, A->ld, n, static_cast<uint16_t*>(c->Lc), c->stream);
    if (e == hipSuccess && params->filter_prec != CHFSI_PREC_FP64)
      e = dup_dinv<float>(d_inv, n, static_cast<float*>(c->dinv2), c->stream);
  }
  if (c->A32) e = convert_f64_f32(A->dense, A->ld, c->A32, n, n, n, c->stream);
  if (e == hipSuccess && c->A16) e = convert_f64_bf16(A->dense, A->ld, c->A16, n, n, n, c->stream);
  if (e == hipSuccess && c->dinv32) {
    if (d_inv)
      e = convert_f64_f32(d_inv, n, c->dinv32, n, n, 1, c->stream);
    else
      e = fill_ones_f32(c->dinv32, n, c->stream);
  }
  if (e == hipSuccess && c->Vf) e = convert_f64_f32(A->field, n, c->Vf, n, n, 1, c->stream);
  // CSR operators: structure check, longest rows, FP32 values
  for (int which = 0; which < 2 && e == hipSuccess; ++which) {
    const chfsi_operator& op = which == 0 ? c->A : c->B;
    if (op.kind != CHFSI_OP_CSR) continue;
    int kmax = 0;
    const hipError_t ce = csr_check(op, c->dflags, c->h_flags, &kmax, c->stream);
    if (ce == hipErrorInvalidValue) {
      set_error("CSR %s: invalid structure (rowptr must start at 0, not decrease and end at nnz; "
                "column indices must lie in [0, n))", which == 0 ? "A" : "B");
      chfsi_destroy(c);
      return CHFSI_ERR_ARG;
    }
    e = ce;
    (which == 0 ? c->csrA_kmax : c->csrB_kmax) = kmax;
  }
  if (e == hipSuccess && c->val32 && A->nnz > 0)
    e = convert_f64_f32(A->val, A->nnz, c->val32, A->nnz, A->nnz, 1, c->stream);
  if (e == hipSuccess && (A->kind == CHFSI_OP_STENCIL27 || c->bloch)) e = stencil_check(*A);
  if (e == hipSuccess && c->Ht) {
    const chfsi_status fs = form_exact_operator(c, A, B);
    if (fs != CHFSI_OK) {
      chfsi_destroy(c);
      return fs;
    }
  }
  if (e == hipSuccess && params->keep_best) {
    chfsi_status ks = CHFSI_OK;
    c->Xbest = ctx_alloc<double>(c, size_t(n) * (c->cplx ? 2 : 1) * b * sizeof(double), &ks);
    if (ks != CHFSI_OK) {
      chfsi_destroy(c);
      return ks;
    }
  }
  if (e == hipSuccess && std::isnan(params->lambda_max)) {
    chfsi_status ls = CHFSI_OK;
    c->lz_work = ctx_alloc<double>(c, lanczos_ctx_bytes(n, c->cplx), &ls);
    if (ls != CHFSI_OK) {
      chfsi_destroy(c);
      return ls;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    set_error("context setup failed: %s", hipGetErrorString(e));
    chfsi_destroy(c);
    return CHFSI_ERR_DEVICE;
  }
  *out = c;
  return CHFSI_OK;
}

extern "C" {

chfsi_status chfsi_filter(chfsi_ctx* c, const double* X, int64_t ldx, const double* ritz,
                          const double* resid, int64_t ldr, double* Yp, int64_t ldy, double lmin,
                          double lmax, double lT, int32_t degree) {
  TraceRange tr("chfsi_filter");
  if (!c || !X || !Yp) {
    set_error("ctx, X and Yp must be non-null");
    return CHFSI_ERR_ARG;
  }
  const int p = degree > 0 ? degree : c->prm.degree;
  if (ldx < c->n || ldy < c->n) {
    set_error("leading dimensions must be >= n");
    return CHFSI_ERR_ARG;
  }
  if (!(lmin < lT && lT < lmax) || !std::isfinite(lmin) || !std::isfinite(lmax)) {
    set_error("filter bounds must satisfy lmin < lT < lmax");
    return CHFSI_ERR_ARG;
  }
  if (c->prm.method == CHFSI_METHOD_RCHFSI) {
    if (!ritz || !resid || ldr < c->n) {
      set_error("the residual filter needs ritz (host), resid (device) and ldr >= n");
      return CHFSI_ERR_ARG;
    }
    if (p > c->coef_cap) {
      set_error("degree %d exceeds the context's degree %d", p, c->coef_cap);
      return CHFSI_ERR_ARG;
    }
    if (c->cplx)
      return filter_rchfsi_complex(c, X, ldx, ritz, resid, ldr, Yp, ldy, lmin, lmax, lT, p,
                                   nullptr);
    return filter_rchfsi(c, X, ldx, ritz, resid, ldr, Yp, ldy, lmin, lmax, lT, p, nullptr);
  }
  return filter_chfsi(c, X, ldx, Yp, ldy, lmin, lmax, lT, p, nullptr);
}

chfsi_status chfsi_filter_kernel_time(chfsi_ctx* c, double* total_ms, int32_t* launches) {
  if (!c || !total_ms || !launches) {
    set_error("null argument");
    return CHFSI_ERR_ARG;
  }
  if (!c->prm.profile) {
    set_error("profiling is off (params.profile = 0)");
    return CHFSI_ERR_ARG;
  }
  CK(prof_flush(c));
  *total_ms = c->pacc_ms;
  *launches = c->pacc_n;
  c->pacc_ms = 0.0;
  c->pacc_n = 0;
  return CHFSI_OK;
}

chfsi_status chfsi_rayleigh_ritz(chfsi_ctx* c, const double* Y, int64_t ldy, double* X,
                                 int64_t ldx, double* R, int64_t ldr, double* ritz,
                                 double* resnorm) {
  TraceRange tr("chfsi_rayleigh_ritz");
  if (!c || !Y || !X || !R || !ritz || !resnorm) {
    set_error("null argument");
    return CHFSI_ERR_ARG;
  }
  if (ldy < c->n || ldx < c->n || ldr < c->n) {
    set_error("leading dimensions must be >= n");
    return CHFSI_ERR_ARG;
  }
  if (c->cplx) {
    if (X == Y) {
      set_error("X must not alias Y");
      return CHFSI_ERR_ARG;
    }
    c->last_sweeps = 0;
    return rayleigh_ritz_complex(c, Y, ldy, X, ldx, R, ldr, ritz, resnorm);
  }
  if (X == Y && c->prm.memory_mode != 1) {
    set_error("X must not alias Y");
    return CHFSI_ERR_ARG;
  }
  c->last_sweeps = 0;
  if (c->prm.memory_mode == 1) {
    // slab-wise: rotate in the output buffer
    CK(copy_block(Y, ldy, X, ldx, c->n, c->b, c->stream));
    return rayleigh_ritz_slabs(c, X, ldx, R, ldr, ritz, resnorm, true);
  }
  return rayleigh_ritz(c, Y, ldy, X, ldx, R, ldr, ritz, resnorm, true);
}

chfsi_status chfsi_estimate_bounds(chfsi_ctx* c, const double* v0, int32_t steps, double* lower,
                                   double* upper, double* theta) {
  if (!c || !lower || !upper) {
    set_error("null argument");
    return CHFSI_ERR_ARG;
  }
  if (steps < 0) {
    set_error("steps must be >= 0");
    return CHFSI_ERR_ARG;
  }
  LanczosResult lr;
  const chfsi_status st = estimate_bounds(c, v0, steps, &lr);
  if (st != CHFSI_OK) return st;
  *lower = lr.lower;
  *upper = lr.upper;
  if (theta) {
    theta[0] = lr.theta_min;
    theta[1] = lr.theta_max;
  }
  return CHFSI_OK;
}

chfsi_status chfsi_solve(chfsi_ctx* c, double* X, int64_t ldx, double* evals, double* resnorms,
                         chfsi_report* rep) {
  TraceRange tr("chfsi_solve");
  if (!c || !X || !evals || !resnorms) {
    set_error("null argument");
    return CHFSI_ERR_ARG;
  }
  if (ldx < c->n) {
    set_error("ldx must be >= n");
    return CHFSI_ERR_ARG;
  }
  const int64_t n = c->n, b = c->b, nw = c->prm.n_wanted;
  const double t0 = now_ms();
  chfsi_report local{};
  chfsi_report& r = rep ? *rep : local;
  std::memset(&r, 0, sizeof(r));
  // complex contexts: interleaved blocks are 2n x b real arrays for fills and copies
  const int64_t rows = c->cplx ? 2 * n : n, lds = c->cplx ? 2 * ldx : ldx,
                ldn = c->cplx ? 2 * n : n;
  if (c->prm.init_random) CK(fill_gaussian(X, lds, rows, b, c->prm.seed, c->stream));
  std::vector<double> ritz(b), norms(b);
  float ms = 0.0f;
  double lmax_used = c->prm.lambda_max;
  // The Lanczos estimate of lambda_max (when needed) does not depend on the
  // first Rayleigh-Ritz pass.  For dense real operators it runs on a second
  // stream from a helper thread while this thread runs that pass: its
  // matrix-vector products stream the operator from HBM, the eigensolver of
  // the pass keeps a few CUs busy.  Joined before the first filter.
  // (the thread's results are declared before the thread and its joiner, so
  // that on every return the joiner runs while they still exist)
  chfsi_status lz_status = CHFSI_OK;
  std::string lz_error;
  LanczosResult lz_res;
  double lz_ms = 0.0;
  std::thread lz_thread;
  struct Joiner {
    std::thread& t;
    ~Joiner() {
      if (t.joinable()) t.join();
    }
  } lz_join{lz_thread};
  if (std::isnan(lmax_used) && !c->have_lmax) {
    if (lanczos_overlap_ok(c)) {
      if (!c->aux_stream) CK(hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking));
      if (!c->ev_aux) CK(hipEventCreateWithFlags(&c->ev_aux, hipEventDisableTiming));
      const chfsi_status ls = ensure_lanczos_work(c);
      if (ls != CHFSI_OK) return ls;
      // after everything the caller queued on the context's stream
      CK(hipEventRecord(c->ev_aux, c->stream));
      CK(hipStreamWaitEvent(c->aux_stream, c->ev_aux, 0));
      lz_thread = std::thread([c, &lz_status, &lz_error, &lz_res, &lz_ms]() {
        const double tb = now_ms();
        if (hipSetDevice(c->device) != hipSuccess) {
          lz_status = CHFSI_ERR_DEVICE;
          lz_error = "hipSetDevice failed in the bound-estimate thread";
          return;
        }
        lz_status = estimate_bounds(c, nullptr, 0, &lz_res, c->aux_stream);
        if (lz_status != CHFSI_OK) lz_error = chfsi_last_error();
        lz_ms = now_ms() - tb;
      });
    } else {
      const double tb = now_ms();
      LanczosResult lr;
      const chfsi_status bs = estimate_bounds(c, nullptr, 0, &lr);
      if (bs != CHFSI_OK) return bs;
      c->lmax_est = lr.upper;
      c->have_lmax = true;
      r.time_bounds_ms = now_ms() - tb;
    }
  }
  CK(hipEventRecord(c->ev[2], c->stream));
  c->last_sweeps = 0;
  c->svqb_events = 0;
  c->svqb_dropped = 0;
  c->flags = 0;
  const bool slabs = c->prm.memory_mode == 1;
  double* Xw = slabs ? X : c->Xw;            // working Ritz block
  const int64_t ldw = slabs ? ldx : n;
  chfsi_status st =
      c->cplx ? rayleigh_ritz_complex(c, X, ldx, c->Xw, n, c->R, n, ritz.data(), norms.data())
      : slabs ? rayleigh_ritz_slabs(c, X, ldx, c->R, n, ritz.data(), norms.data(), true)
              : rayleigh_ritz(c, X, ldx, c->Xw, n, c->R, n, ritz.data(), norms.data(), true);
  if (st != CHFSI_OK) return st;
  CK(hipEventRecord(c->ev[3], c->stream));
  CK(hipEventSynchronize(c->ev[3]));
  CK(hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
  r.time_rr_ms += ms;
  r.jacobi_sweeps += c->last_sweeps;
  if (lz_thread.joinable()) {
    lz_thread.join();
    if (lz_status != CHFSI_OK) {
      set_error_message(lz_error.c_str());
      return lz_status;
    }
    c->lmax_est = lz_res.upper;
    c->have_lmax = true;
    r.time_bounds_ms = lz_ms;
  }
  if (std::isnan(lmax_used)) lmax_used = c->lmax_est;
  r.lambda_max_used = lmax_used;
  auto maxres = [&]() {
    double m = 0.0;
    for (int64_t j = 0; j < nw; ++j) m = std::max(m, norms[j]);
    return m;
  };
  double mr = maxres();
  r.history[0] = mr;
  // lowest max residual so far (and, with keep_best, its pairs); the stall
  // test counts the passes since the lowest value last fell below half of the
  // value at the previous such point
  double best = mr;
  int best_it = 0;
  double mark = mr;
  int mark_it = 0;
  std::vector<double> best_ritz, best_norms;
  auto keep = [&]() -> chfsi_status {
    if (!c->Xbest) return CHFSI_OK;
    CK(copy_block(Xw, c->cplx ? 2 * ldw : ldw, c->Xbest, ldn, rows, b, c->stream));
    best_ritz = ritz;
    best_norms = norms;
    return CHFSI_OK;
  };
  if ((st = keep()) != CHFSI_OK) return st;
  int it = 0;
  for (; it < c->prm.max_iter && !(mr < c->prm.tol); ++it) {
    if (c->cancel && c->cancel->load()) {
      set_error("cancelled");
      st = CHFSI_ERR_CANCELLED;
      break;
    }
    double lmin, lmax, lT;
    bounds_policy(c->prm, lmax_used, ritz.data(), b, &lmin, &lmax, &lT);
    if (!(lmin < lT && lT < lmax)) {
      set_error("filter bounds collapsed (lmin %.6g, lT %.6g, lmax %.6g): lambda_max too small?",
                lmin, lT, lmax);
      st = CHFSI_ERR_ARG;
      break;
    }
    double amp = 0.0;
    const int deg = pass_degree(c->prm, lmin, lmax, lT, &amp);
    r.max_amplification = std::max(r.max_amplification, amp);
    r.min_degree_used = r.min_degree_used == 0 ? deg : std::min(r.min_degree_used, deg);
    if (amp > 1e12) c->flags |= 16;
    if (deg < c->prm.degree) c->flags |= 32;
    CK(hipEventRecord(c->ev[0], c->stream));
    {
      TraceRange tr("chfsi filter");
      if (c->cplx)
        st = filter_rchfsi_complex(c, c->Xw, n, ritz.data(), c->R, n, c->Yw, n, lmin, lmax, lT,
                                   deg, &r.filter_flops);
      else if (c->prm.method == CHFSI_METHOD_RCHFSI)
        st = filter_rchfsi(c, Xw, ldw, ritz.data(), c->R, n, slabs ? Xw : c->Yw,
                           slabs ? ldw : n, lmin, lmax, lT, deg, &r.filter_flops);
      else
        st = filter_chfsi(c, c->Xw, n, c->Yw, n, lmin, lmax, lT, deg, &r.filter_flops);
    }
    if (st != CHFSI_OK) break;
    CK(hipEventRecord(c->ev[1], c->stream));
    c->last_sweeps = 0;
    {
      TraceRange tr("chfsi rayleigh-ritz");
      st = c->cplx ? rayleigh_ritz_complex(c, c->Yw, n, c->Xw, n, c->R, n, ritz.data(),
                                           norms.data())
           : slabs ? rayleigh_ritz_slabs(c, Xw, ldw, c->R, n, ritz.data(), norms.data(), true)
                   : rayleigh_ritz(c, c->Yw, n, c->Xw, n, c->R, n, ritz.data(), norms.data(),
                                   true);
    }
    if (st != CHFSI_OK) break;
    CK(hipEventRecord(c->ev[3], c->stream));
    CK(hipEventSynchronize(c->ev[3]));
    CK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    r.time_filter_ms += ms;
    CK(hipEventElapsedTime(&ms, c->ev[1], c->ev[3]));
    r.time_rr_ms += ms;
    r.jacobi_sweeps += c->last_sweeps;
    if (c->prm.profile) {
      CK(prof_flush(c));
      r.kernel_ms += c->pacc_ms;
      r.kernel_launches += c->pacc_n;
      c->pacc_ms = 0.0;
      c->pacc_n = 0;
    }
    mr = maxres();
    if (it + 1 < CHFSI_MAX_HISTORY) r.history[it + 1] = mr;
    if (mr < best) {
      best = mr;
      best_it = it + 1;
      if ((st = keep()) != CHFSI_OK) break;
    }
    if (best < 0.5 * mark) {
      mark = best;
      mark_it = it + 1;
    }
    if (mr < c->prm.tol) {
      // converged
    } else if (c->prm.stall_iters > 0 && it + 1 - mark_it >= c->prm.stall_iters &&
               c->prm.escalate && c->prm.filter_prec == CHFSI_PREC_BF16) {
      // stagnation of the BF16 filter: the remaining passes filter in FP32
      c->prm.filter_prec = CHFSI_PREC_FP32;
      c->flags |= 8;
      r.escalation_iteration = it + 1;
      mark = best;
      mark_it = it + 1;
      if (progress_log())
        std::fprintf(stderr, "chfsi_solve: BF16 filter stagnated at %.3e; FP32 from iteration %d\n",
                     mr, it + 2);
    } else if (c->prm.stall_iters > 0 && it + 1 - mark_it >= c->prm.stall_iters) {
      // stagnation: no new lowest max residual for stall_iters passes
      c->flags |= 4;
      ++it;
      if (progress_log())
        std::fprintf(stderr, "chfsi_solve: stagnation after %d iterations (best %.3e at %d)\n",
                     it, best, best_it);
      break;
    }
    if (progress_log())
      std::fprintf(stderr,
                   "chfsi_solve: iteration %d, max residual %.3e (filter %.1f ms, RR %.1f ms, "
                   "SVQB fallbacks %d, dropped directions %d)\n",
                   it + 1, mr, r.time_filter_ms, r.time_rr_ms, c->svqb_events, c->svqb_dropped);
  }
  if (c->prm.escalate) c->prm.filter_prec = CHFSI_PREC_BF16;   // the context's own precision
  r.iterations = it;
  r.max_residual = mr;
  r.converged = mr < c->prm.tol;
  r.best_iteration = best_it;
  r.best_residual = best;
  r.flags = c->flags;
  if (st == CHFSI_OK && !r.converged && c->Xbest && best_it != it) {
    // CHFSI_ERR_NOCONV with keep_best: return the pairs of the lowest max residual
    CK(copy_block(c->Xbest, ldn, Xw, c->cplx ? 2 * ldw : ldw, rows, b, c->stream));
    ritz = best_ritz;
    norms = best_norms;
    r.max_residual = best;
  }
  r.svqb_events = c->svqb_events;
  r.svqb_dropped = c->svqb_dropped;
  if (st != CHFSI_OK && st != CHFSI_ERR_NOCONV) return st;
  if (!slabs) CK(copy_block(c->Xw, ldn, X, lds, rows, b, c->stream));
  CK(hipStreamSynchronize(c->stream));
  std::memcpy(evals, ritz.data(), b * sizeof(double));
  std::memcpy(resnorms, norms.data(), b * sizeof(double));
  r.time_total_ms = now_ms() - t0;
  if (!r.converged) {
    set_error("no convergence after %d iterations (max residual %.3e)", it, mr);
    return CHFSI_ERR_NOCONV;
  }
  return CHFSI_OK;
}

}  // extern "C"
