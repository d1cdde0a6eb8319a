// Internal interface of the operator kernels other than the dense GEMM: the
// periodic 27-point grid operators and the sparse (CSR) operators.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/chfsi.h"

namespace chfsi {

// Coefficients of one filter step: out = alpha * (op applied) + beta * src
// + gamma * prev + delta * colcoef[j] * forcing.
struct StencilStep {
  double alpha, beta, gamma, delta;
};

hipError_t stencil_check(const chfsi_operator& op);

// Bloch-phase operators in the twisted frame (bloch.hip).  Planar blocks of
// `pairs` complex columns (real parts, then imaginary parts; 2 x pairs
// columns).  The correction (A_tw - A_per) psi (p) = sum over the offsets o
// wrapped at p of w(p, o) (phi(o) - 1) psi(p + o), phi the wrap phase, is
// nonzero at the n - (nx-2)(ny-2)(nz-2) boundary points only.
// dst += alpha * colscale[j] * correction of (dinv .* src) for column pair j,
// in place (dinv NULL: identity; colscale NULL: ones; both device arrays)
// edge (may be null): src's row ends as for bloch_corr below.
template <typename F>
hipError_t bloch_fix(const chfsi_operator& op, const double* dinv, double alpha, const F* src,
                     int64_t lds, F* dst, int64_t ldd, int64_t pairs, hipStream_t st,
                     const double* colscale = nullptr, const F* edge = nullptr);
// edge (2 ny nz per column, ld 2 ny nz) = the x = 0 and x = nx-1 values of
// every grid row of the planar block src (cols columns, ld lds)
template <typename T>
hipError_t bloch_edges(const chfsi_operator& op, const T* src, int64_t lds, T* edge, int64_t cols,
                       hipStream_t st);
// corr (boundary points x 2 pairs, ld ldc >= boundary points) = alpha *
// correction of (dinv .* src), in the boundary-point enumeration of bloch.hip.
// edge (may be null): src's x = 0 and x = nx-1 values, ((z ny + y) 2 +
// (x == nx-1)) per column, ld 2 ny nz; the x-face points then read their
// wrapped neighbours there instead of gathering them from src.
template <typename T, typename C>
hipError_t bloch_corr(const chfsi_operator& op, const double* dinv, double alpha, const T* src,
                      int64_t lds, const T* edge, C* corr, int64_t ldc, int64_t pairs,
                      hipStream_t st);
// A residual-filter step on a Bloch operator's planar block adds the
// correction: through `corr` in the z-marching kernel's epilogue, else by
// bloch_fix after the step.
struct BlochStep {
  void* corr;          // boundary points x b buffer in the step's arithmetic type
  int64_t ld_corr;     // >= boundary points, a multiple of 4 (16-byte aligned column starts)
  const double* dinv;  // FP64 D^{-1} of the correction (NULL: identity)
  const void* edge_in; // row-end values of RY (storage type; may be null)
  void* edge_out;      // receives the row-end values of the step's output (may be null)
};
// nominal flops per element and step (for reporting)
double stencil_flops(const chfsi_operator& op);

// Y = op X (FP64), X/Y column-major n x b
hipError_t stencil_apply_f64(const chfsi_operator& op, const double* X, int64_t ldx, double* Y,
                             int64_t ldy, int64_t b, hipStream_t st);

// Residual filter step (Algorithm 3 loop body), RX updated in place, ld = n:
// RX <- a op(dinv .* RY) + b RY + c RX + delta colcoef[j] Yf
hipError_t stencil_rchfsi_step_f64(const chfsi_operator& op, const double* dinv, const double* RY,
                                   double* RX, const double* Yf, int64_t ldf,
                                   const double* colcoef, StencilStep s, int64_t b,
                                   hipStream_t st,
                                   const BlochStep* bloch = nullptr);
// Vf: the potential in FP32 (length n; may be NULL when the operator has no
// field); dinv: NULL for D^{-1} = I.
hipError_t stencil_rchfsi_step_f32(const chfsi_operator& op, const float* Vf, const float* dinv,
                                   const float* RY, float* RX, const float* Yf,
                                   const float* colcoef, StencilStep s, int64_t b, hipStream_t st,
                                   const BlochStep* bloch = nullptr);
// BF16-stored blocks (uint16 bit patterns), FP32 arithmetic
hipError_t stencil_rchfsi_step_bf16(const chfsi_operator& op, const float* Vf, const float* dinv,
                                    const void* RY, void* RX, const void* Yf,
                                    const float* colcoef, StencilStep s, int64_t b,
                                    hipStream_t st,
                                   const BlochStep* bloch = nullptr);
// Plain filter step (Algorithm 2): dst <- alpha dinv .* op(src) + beta src + gamma prev
hipError_t stencil_chfsi_step_f64(const chfsi_operator& op, const double* dinv, const double* src,
                                  int64_t lds, const double* prev, int64_t ldp, double* dst,
                                  StencilStep s, int64_t b, hipStream_t st);

// Slab-wise application: Yslab = rows of (op X) in planes [z0, z0 + nzs)
hipError_t stencil_apply_slab_f64(const chfsi_operator& op, const double* X, int64_t ldx,
                                  double* Yslab, int64_t ldy, int64_t b, int z0, int nzs,
                                  hipStream_t st);
// Fused residual R = A X - B X diag(lam) (B NULL: identity)
hipError_t stencil_residual_f64(const chfsi_operator& A, const chfsi_operator* B, const double* X,
                                int64_t ldx, const double* lam, double* R, int64_t ldr, int64_t b,
                                hipStream_t st);
// true when the z-marching class-sum kernels apply (tensor-product coefficients)
bool stencil_separable(const chfsi_operator& op);

// ---------------------------------------------------------------------------
// Sparse symmetric operators in CSR form (csr.hip).  val is double for the
// FP64 kernels and float (the context's copy) for the FP32 / BF16 ones; kmax
// is the longest row.
// ---------------------------------------------------------------------------
struct CsrMat {
  int64_t n = 0;
  const int64_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const void* val = nullptr;
  int kmax = 0;
};
// Validates the structure of op (rowptr[0] = 0, non-decreasing, rowptr[n] =
// nnz, column indices in [0, n)) and returns its longest row in *kmax;
// flags_dev: 2 device ints of scratch, flags_host: 2 pinned host ints.
// Synchronises the stream.  hipErrorInvalidValue: invalid structure.
hipError_t csr_check(const chfsi_operator& op, int* flags_dev, int* flags_host, int* kmax,
                     hipStream_t st);
// Y = A X (FP64), column-major n x b blocks
hipError_t csr_apply_f64(const CsrMat& A, const double* X, int64_t ldx, double* Y, int64_t ldy,
                         int64_t b, hipStream_t st);
// residual-filter step (ld n): RX <- alpha A (dinv .* RY) + beta RY + gamma RX
//                                    + delta colcoef[j] Yf
hipError_t csr_rchfsi_step_f64(const CsrMat& A, const double* dinv, const double* RY, double* RX,
                               const double* Yf, int64_t ldf, const double* colcoef,
                               StencilStep s, int64_t b, hipStream_t st);
hipError_t csr_rchfsi_step_f32(const CsrMat& A32, const float* dinv, const float* RY, float* RX,
                               const float* Yf, const float* colcoef, StencilStep s, int64_t b,
                               hipStream_t st);
// bfloat16-stored blocks, FP32 arithmetic
hipError_t csr_rchfsi_step_bf16(const CsrMat& A32, const float* dinv, const void* RY, void* RX,
                                const void* Yf, const float* colcoef, StencilStep s, int64_t b,
                                hipStream_t st);
// plain-filter step: dst <- alpha dinv .* (A src) + beta src + gamma prev (prev may be null)
hipError_t csr_chfsi_step_f64(const CsrMat& A, const double* dinv, const double* src,
                              int64_t lds, const double* prev, int64_t ldp, double* dst,
                              StencilStep s, int64_t b, hipStream_t st);

// BF16 block helpers
hipError_t rchfsi_init_bf16(const double* R, int64_t ldr, int64_t n, int64_t b, double scale,
                            void* RY, void* RX, void* Yc, hipStream_t st);
hipError_t rchfsi_reconstruct_bf16(const void* RY, const double* dinv, const double* X,
                                   int64_t ldx, const double* lamY, double* Yp, int64_t ldy,
                                   int64_t n, int64_t b, hipStream_t st);

// FP32 helpers used by the driver
hipError_t convert_f32_f64(const float* in, int64_t ldi, double* out, int64_t ldo, int64_t n,
                           int64_t m, hipStream_t st);
hipError_t fill_ones_f32(float* p, int64_t n, hipStream_t st);

}  // namespace chfsi
