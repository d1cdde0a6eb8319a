// Residual filter (Algorithm 3) in FP64 without any device allocation:
// chfsi_filter_static (include/chfsi.h).  Every intermediate -- the per-step
// Lambda_Y table of the eigenvalue recurrence, the final Lambda_Y, the two
// recurrence blocks R_X and R_Y and the split-K partial sums of the dense
// product -- lives in one file-scope device array.  The host obtains that
// array's device address with hipGetSymbolAddress once per device and passes
// the address (never the array's name) to the kernels, which are the same
// ones the context-based filter launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "internal.h"
#include "stencil_api.h"

// One copy per device, held from the code object's load to the end of the
// process.  Host code must not take this name's address for device use: in
// host code it denotes a host-side shadow.
static __device__ __align__(256) unsigned char scratch[CHFSI_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on each device, with that device current).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

namespace {

chfsi_status fail(chfsi_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  chfsi::set_error_message(buf);
  return st;
}

#define CKS(x)                                                                     \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess)                                                          \
      return fail(CHFSI_ERR_DEVICE, "%s: %s", #x, hipGetErrorString(e_));          \
  } while (0)

}  // namespace

extern "C" {

size_t chfsi_filter_static_bytes(int64_t n, int64_t b, int32_t degree) {
  if (n <= 0 || b <= 0 || degree < 1) return 0;
  const size_t nb = size_t(n) * size_t(b) * sizeof(double);
  return round_up(size_t(degree) * size_t(b) * sizeof(double), 256) + 2 * round_up(nb, 256);
}

chfsi_status chfsi_filter_static(const chfsi_operator* A, const double* d_inv, int64_t b,
                                 const double* X, int64_t ldx, const double* ritz,
                                 const double* resid, int64_t ldr, double* Yp, int64_t ldy,
                                 double lmin, double lmax, double lT, int32_t degree,
                                 void* stream) {
  using namespace chfsi;
  if (!A) return fail(CHFSI_ERR_ARG, "null operator");
  if (A->kind != CHFSI_OP_DENSE && A->kind != CHFSI_OP_STENCIL27)
    return fail(CHFSI_ERR_ARG, "chfsi_filter_static takes a dense or 27-point grid operator");
  const int64_t n = A->n;
  if (n <= 0) return fail(CHFSI_ERR_ARG, "operator size must be positive");
  if (A->kind == CHFSI_OP_DENSE && (!A->dense || A->ld < n))
    return fail(CHFSI_ERR_ARG, "dense operator needs a matrix with ld >= n");
  if (A->kind == CHFSI_OP_STENCIL27 && stencil_check(*A) != hipSuccess)
    return fail(CHFSI_ERR_ARG, "invalid grid operator");
  if (b < 0) return fail(CHFSI_ERR_ARG, "b must be >= 0");
  if (degree < 1) return fail(CHFSI_ERR_ARG, "degree must be >= 1");
  // set-up: the scratch array's address on this device (a call with b = 0
  // does only this, so that callers can bind it before a stream capture)
  void* base = nullptr;
  CKS(scratch_address(&base));
  if (b == 0) return CHFSI_OK;
  if (!X || !ritz || !resid || !Yp) return fail(CHFSI_ERR_ARG, "null block argument");
  if (ldx < n || ldr < n || ldy < n) return fail(CHFSI_ERR_ARG, "leading dimensions must be >= n");
  if (!(lmin < lT && lT < lmax) || !std::isfinite(lmin) || !std::isfinite(lmax))
    return fail(CHFSI_ERR_ARG, "filter bounds must satisfy lmin < lT < lmax (finite)");
  const size_t need = chfsi_filter_static_bytes(n, b, degree);
  if (need == 0 || need > size_t(CHFSI_STATIC_SCRATCH_BYTES))
    return fail(CHFSI_ERR_ARG,
                "n = %lld, b = %lld, degree %d need %zu bytes of static scratch; the maximum is "
                "%zu (CHFSI_STATIC_SCRATCH_BYTES)",
                (long long)n, (long long)b, degree, need, size_t(CHFSI_STATIC_SCRATCH_BYTES));
  hipStream_t st = static_cast<hipStream_t>(stream);

  // scratch layout: [Lambda_Y table (p - 1) x b | final Lambda_Y (b)] [R_X] [R_Y] [partials]
  char* s = static_cast<char*>(base);
  double* coef = reinterpret_cast<double*>(s);
  double* lamY = coef + int64_t(degree - 1) * b;
  s += round_up(size_t(degree) * size_t(b) * sizeof(double), 256);
  const size_t blk = round_up(size_t(n) * size_t(b) * sizeof(double), 256);
  double* RX = reinterpret_cast<double*>(s);
  double* RY = reinterpret_cast<double*>(s + blk);
  Workspace ws;
  ws.ptr = s + 2 * blk;
  ws.bytes = size_t(CHFSI_STATIC_SCRATCH_BYTES) - need;

  // Algorithm 3: e, c, sigma_1 from the bounds; the Lambda recurrence on the
  // device; R_Y = (sigma_1 / e) Y, R_X = 0; p - 1 fused recurrence steps
  const double e = (lmax - lT) / 2.0, c = (lmax + lT) / 2.0;
  const double sigma1 = e / (lmin - c);
  const double gamma = 2.0 / sigma1;
  CKS(rchfsi_coef(ritz, b, e, c, sigma1, degree, coef, nullptr, lamY, st));
  CKS(rchfsi_init_f64(resid, ldr, n, b, sigma1 / e, RY, RX, n, st));
  double sigma = sigma1;
  for (int k = 2; k <= degree; ++k) {
    const double sigma2 = 1.0 / (gamma - sigma);
    const double a = 2.0 * sigma2 / e;
    const double* colcoef = coef + int64_t(k - 2) * b;
    if (A->kind == CHFSI_OP_DENSE) {
      // R_X <- a A (D^{-1} R_Y) - a c R_Y - sigma sigma2 R_X + a Y diag(Lambda_Y)
      GemmDesc<double> g;
      g.M = n;
      g.N = b;
      g.K = n;
      g.A = A->dense;
      g.sak = 1;
      g.sam = A->ld;
      g.B = RY;
      g.sbk = 1;
      g.sbn = n;
      g.kscale = d_inv;
      g.C = RX;
      g.ldc = n;
      g.epi.alpha = a;
      g.epi.beta = -a * c;
      g.epi.C1 = RY;
      g.epi.ldc1 = n;
      g.epi.gamma = -sigma * sigma2;
      g.epi.C2 = RX;
      g.epi.ldc2 = n;
      g.epi.delta = a;
      g.epi.colscale3 = colcoef;
      g.epi.C3 = resid;
      g.epi.ldc3 = ldr;
      CKS(gemm<double>(g, st, ws, 0, -1));
    } else {
      const StencilStep ss{a, -a * c, -sigma * sigma2, a};
      CKS(stencil_rchfsi_step_f64(*A, d_inv, RY, RX, resid, ldr, colcoef, ss, b, st));
    }
    std::swap(RX, RY);
    sigma = sigma2;
  }
  // Y_p = D^{-1} R_Y + X diag(Lambda_Y)
  CKS(rchfsi_reconstruct_f64(RY, n, d_inv, X, ldx, lamY, Yp, ldy, n, b, st));
  return CHFSI_OK;
}

}  // extern "C"
