// Sparse symmetric operators in compressed sparse row form: the operator
// products of the filter (Algorithms 2 and 3) and of Rayleigh-Ritz for the
// finite-element-type matrices of Section 4.2.
//
// Blocks are column-major n x b.  One workgroup owns a tile of 64 consecutive
// rows: it stages the tile's column indices and values in LDS as a padded
// [k][row] array (ELL layout within the tile; padding entries carry weight 0
// and a valid index), then its four waves sweep the block's columns, one
// column per wave at a time, one row per lane.  The matrix is read from HBM
// once per launch, whatever b is; the gathered source entries of neighbouring
// rows fall in the same cache lines for banded / grid-ordered matrices; the
// epilogue (the filter's three-term update, or the row scaling of the plain
// filter) reads and writes each output element once, coalesced across lanes.
// For the residual filter's A (D^{-1} R_Y), D^{-1} is folded into the staged
// values (column side).  Rows longer than kLdsKmax use a plain kernel with one
// thread per (row, column).
#include "internal.h"
#include "stencil_api.h"

#include <algorithm>

namespace chfsi {

namespace {

constexpr int kRows = 64;
constexpr int kThreads = 256;
constexpr int kLdsKmax = 80;   // staged row length: 64 x 80 x 12 B = 60 KB of LDS at most

enum { MODE_APPLY = 0, MODE_RSTEP = 1, MODE_CSTEP = 2 };

__device__ __forceinline__ double load_as(const double* p, int64_t i, double) { return p[i]; }
__device__ __forceinline__ float load_as(const float* p, int64_t i, float) { return p[i]; }
__device__ __forceinline__ float load_as(const uint16_t* p, int64_t i, float) {
  return __uint_as_float(uint32_t(p[i]) << 16);
}
__device__ __forceinline__ void store_to(double* p, int64_t i, double v) { p[i] = v; }
__device__ __forceinline__ void store_to(float* p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void store_to(uint16_t* p, int64_t i, float v) {
  // round to nearest even (v_cvt_pk_bf16_f32)
  p[i] = __builtin_bit_cast(uint16_t, static_cast<__bf16>(v));
}

template <typename S, typename AT, typename VT>
struct CsrArgs {
  int64_t n, b;
  const int64_t* rowptr;
  const int32_t* col;
  const VT* val;
  int kmax;
  const AT* cdinv;     // column-side scaling of the values (residual filter), or null
  const AT* rdinv;     // row-side scaling of the product (plain filter), or null
  const S* src;
  int64_t lds;
  S* dst;
  int64_t ldd;
  const S* prev;       // may alias dst
  int64_t ldp;
  const S* forc;
  int64_t ldf;
  const AT* colcoef;
  AT alpha, beta, gamma, delta;
};

template <typename S, typename AT, typename VT, int MODE>
__device__ __forceinline__ void epilogue(const CsrArgs<S, AT, VT>& a, int64_t row, int64_t j,
                                         AT acc) {
  AT out;
  if (MODE == MODE_APPLY) {
    out = acc;
  } else if (MODE == MODE_RSTEP) {
    out = a.alpha * acc + a.beta * load_as(a.src, row + j * a.lds, AT()) +
          a.gamma * load_as(a.prev, row + j * a.ldp, AT()) +
          a.delta * a.colcoef[j] * load_as(a.forc, row + j * a.ldf, AT());
  } else {
    const AT d = a.rdinv ? a.rdinv[row] : AT(1);
    out = a.alpha * d * acc + a.beta * load_as(a.src, row + j * a.lds, AT());
    if (a.prev) out += a.gamma * load_as(a.prev, row + j * a.ldp, AT());
  }
  store_to(a.dst, row + j * a.ldd, out);
}

template <typename S, typename AT, typename VT, int MODE>
__global__ __launch_bounds__(kThreads) void k_csr_tile(CsrArgs<S, AT, VT> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int kmax = a.kmax;
  int32_t* lc = reinterpret_cast<int32_t*>(smem);
  VT* lv = reinterpret_cast<VT*>(smem + ((size_t(kmax) * kRows * sizeof(int32_t) + 15) & ~size_t(15)));
  const int64_t row0 = int64_t(blockIdx.x) * kRows;
  for (int idx = threadIdx.x; idx < kmax * kRows; idx += kThreads) {
    const int r = idx & (kRows - 1), k = idx / kRows;
    const int64_t row = row0 + r;
    int32_t c = 0;
    VT v = VT(0);
    if (row < a.n) {
      c = int32_t(row);   // padding: this row's own index with weight 0
      const int64_t s = a.rowptr[row], e = a.rowptr[row + 1];
      if (k < e - s) {
        c = a.col[s + k];
        v = a.val[s + k];
        if (a.cdinv) v = VT(AT(v) * a.cdinv[c]);
      }
    }
    lc[idx] = c;
    lv[idx] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kRows - 1), wave = threadIdx.x / kRows;
  const int64_t row = row0 + lane;
  if (row >= a.n) return;   // no barrier follows
  for (int64_t j = wave; j < a.b; j += kThreads / kRows) {
    const S* sj = a.src + j * a.lds;
    AT acc = AT(0);
    for (int k = 0; k < kmax; ++k)
      acc += AT(lv[k * kRows + lane]) * load_as(sj, lc[k * kRows + lane], AT());
    epilogue<S, AT, VT, MODE>(a, row, j, acc);
  }
}

// rows longer than kLdsKmax: one thread per (row, column), entries from global memory
template <typename S, typename AT, typename VT, int MODE>
__global__ __launch_bounds__(kThreads) void k_csr_plain(CsrArgs<S, AT, VT> a) {
  const int64_t total = a.n * a.b;
  for (int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / a.n, row = idx - j * a.n;
    const S* sj = a.src + j * a.lds;
    AT acc = AT(0);
    for (int64_t p = a.rowptr[row]; p < a.rowptr[row + 1]; ++p) {
      const int32_t c = a.col[p];
      AT v = AT(a.val[p]);
      if (a.cdinv) v *= a.cdinv[c];
      acc += v * load_as(sj, c, AT());
    }
    epilogue<S, AT, VT, MODE>(a, row, j, acc);
  }
}

// structure checks and the longest row: flags[0] |= 1 bad rowptr, 2 bad
// column index; flags[1] = max row length
__global__ __launch_bounds__(kThreads) void k_csr_check(int64_t n, const int64_t* rowptr,
                                                        const int32_t* col, int64_t nnz,
                                                        int* flags) {
  for (int64_t row = int64_t(blockIdx.x) * kThreads + threadIdx.x; row < n;
       row += int64_t(gridDim.x) * kThreads) {
    const int64_t s = rowptr[row], e = rowptr[row + 1];
    if (row == 0 && s != 0) atomicOr(flags, 1);
    if (row == n - 1 && e != nnz) atomicOr(flags, 1);
    if (e < s || s < 0 || e > nnz) {
      atomicOr(flags, 1);
      continue;
    }
    const int64_t len = e - s;
    atomicMax(flags + 1, int(std::min<int64_t>(len, 0x7fffffff)));
    for (int64_t p = s; p < e; ++p)
      if (col[p] < 0 || int64_t(col[p]) >= n) atomicOr(flags, 2);
  }
}

template <typename S, typename AT, typename VT, int MODE>
hipError_t launch(const CsrArgs<S, AT, VT>& a, hipStream_t st) {
  if (a.n <= 0 || a.b <= 0) return hipSuccess;
  if (a.kmax <= kLdsKmax) {
    const int k = std::max(a.kmax, 1);
    CsrArgs<S, AT, VT> a2 = a;
    a2.kmax = k;
    const size_t lds = ((size_t(k) * kRows * sizeof(int32_t) + 15) & ~size_t(15)) +
                       size_t(k) * kRows * sizeof(VT);
    const int64_t tiles = (a.n + kRows - 1) / kRows;
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    k_csr_tile<S, AT, VT, MODE><<<dim3(unsigned(tiles)), kThreads, lds, st>>>(a2);
  } else {
    const int64_t g = std::min<int64_t>((a.n * a.b + kThreads - 1) / kThreads, 65536);
    k_csr_plain<S, AT, VT, MODE><<<dim3(unsigned(g)), kThreads, 0, st>>>(a);
  }
  return hipGetLastError();
}

template <typename S, typename AT, typename VT>
CsrArgs<S, AT, VT> base_args(const CsrMat& A, int64_t b) {
  CsrArgs<S, AT, VT> a{};
  a.n = A.n;
  a.b = b;
  a.rowptr = A.rowptr;
  a.col = A.col;
  a.val = static_cast<const VT*>(A.val);
  a.kmax = A.kmax;
  return a;
}

}  // namespace

hipError_t csr_check(const chfsi_operator& op, int* flags_dev, int* flags_host, int* kmax,
                     hipStream_t st) {
  hipError_t e = fill_zero(flags_dev, 2 * sizeof(int), st);
  if (e != hipSuccess) return e;
  const int64_t g = std::max<int64_t>(1, std::min<int64_t>((op.n + kThreads - 1) / kThreads, 4096));
  k_csr_check<<<dim3(unsigned(g)), kThreads, 0, st>>>(op.n, op.rowptr, op.colind, op.nnz, flags_dev);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(flags_host, flags_dev, 2 * sizeof(int), hipMemcpyDeviceToHost, st)) !=
      hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  *kmax = flags_host[1];
  return flags_host[0] == 0 ? hipSuccess : hipErrorInvalidValue;
}

hipError_t csr_apply_f64(const CsrMat& A, const double* X, int64_t ldx, double* Y, int64_t ldy,
                         int64_t b, hipStream_t st) {
  auto a = base_args<double, double, double>(A, b);
  a.src = X;
  a.lds = ldx;
  a.dst = Y;
  a.ldd = ldy;
  return launch<double, double, double, MODE_APPLY>(a, st);
}

hipError_t csr_rchfsi_step_f64(const CsrMat& A, const double* dinv, const double* RY, double* RX,
                               const double* Yf, int64_t ldf, const double* colcoef,
                               StencilStep s, int64_t b, hipStream_t st) {
  auto a = base_args<double, double, double>(A, b);
  a.cdinv = dinv;
  a.src = RY;
  a.lds = A.n;
  a.dst = RX;
  a.ldd = A.n;
  a.prev = RX;
  a.ldp = A.n;
  a.forc = Yf;
  a.ldf = ldf;
  a.colcoef = colcoef;
  a.alpha = s.alpha;
  a.beta = s.beta;
  a.gamma = s.gamma;
  a.delta = s.delta;
  return launch<double, double, double, MODE_RSTEP>(a, st);
}

template <typename S>
static hipError_t rstep_lowp(const CsrMat& A32, const float* dinv, const S* RY, S* RX, const S* Yf,
                             const float* colcoef, StencilStep s, int64_t b, hipStream_t st) {
  auto a = base_args<S, float, float>(A32, b);
  a.cdinv = dinv;
  a.src = RY;
  a.lds = A32.n;
  a.dst = RX;
  a.ldd = A32.n;
  a.prev = RX;
  a.ldp = A32.n;
  a.forc = Yf;
  a.ldf = A32.n;
  a.colcoef = colcoef;
  a.alpha = float(s.alpha);
  a.beta = float(s.beta);
  a.gamma = float(s.gamma);
  a.delta = float(s.delta);
  return launch<S, float, float, MODE_RSTEP>(a, st);
}

hipError_t csr_rchfsi_step_f32(const CsrMat& A32, const float* dinv, const float* RY, float* RX,
                               const float* Yf, const float* colcoef, StencilStep s, int64_t b,
                               hipStream_t st) {
  return rstep_lowp<float>(A32, dinv, RY, RX, Yf, colcoef, s, b, st);
}

hipError_t csr_rchfsi_step_bf16(const CsrMat& A32, const float* dinv, const void* RY, void* RX,
                                const void* Yf, const float* colcoef, StencilStep s, int64_t b,
                                hipStream_t st) {
  return rstep_lowp<uint16_t>(A32, dinv, static_cast<const uint16_t*>(RY),
                              static_cast<uint16_t*>(RX), static_cast<const uint16_t*>(Yf),
                              colcoef, s, b, st);
}

hipError_t csr_chfsi_step_f64(const CsrMat& A, const double* dinv, const double* src,
                              int64_t lds, const double* prev, int64_t ldp, double* dst,
                              StencilStep s, int64_t b, hipStream_t st) {
  auto a = base_args<double, double, double>(A, b);
  a.rdinv = dinv;
  a.src = src;
  a.lds = lds;
  a.dst = dst;
  a.ldd = A.n;
  a.prev = prev;
  a.ldp = ldp;
  a.alpha = s.alpha;
  a.beta = s.beta;
  a.gamma = s.gamma;
  return launch<double, double, double, MODE_CSTEP>(a, st);
}

}  // namespace chfsi
