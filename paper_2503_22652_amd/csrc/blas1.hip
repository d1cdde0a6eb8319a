// Bandwidth-bound helper kernels of the eigensolver: the initialisation and
// reconstruction steps of the residual filter (Algorithm 3, first and last
// lines), residual column norms (Algorithm 1 stopping test), Gram scaling for
// the Cholesky-based Rayleigh-Ritz step, conversions and fills.
//
// All are grid-stride kernels over column-major blocks with 64-bit indexing.
// Reductions use a fixed thread->element assignment and a fixed LDS tree, so
// results are bitwise reproducible run to run.
#include "internal.h"
#include "stencil_api.h"

#include <cmath>

namespace chfsi {

namespace {

constexpr int kThreads = 256;

inline int64_t grid_for(int64_t total, int64_t cap = 65536) {
  int64_t g = (total + kThreads - 1) / kThreads;
  if (g < 1) g = 1;
  return g > cap ? cap : g;
}

__global__ __launch_bounds__(kThreads) void k_rchfsi_init_f32(const double* __restrict__ R,
                                                               int64_t ldr, int64_t n, int64_t b,
                                                               double scale, float* RY, float* RX,
                                                               float* Yc, int64_t ld32) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    const double r = R[i + j * ldr];
    RY[i + j * ld32] = float(scale * r);
    RX[i + j * ld32] = 0.0f;
    Yc[i + j * ld32] = float(r);
  }
}

// Lambda recurrence of the residual filter (Algorithm 3; eq. ChFSIrecurrenceEigval),
// one thread per column: Lambda_X = 1, Lambda_Y = (sigma1 / e)(lambda_j - c), then
// for k = 2..p Lambda_X <- a Lambda_Y lambda_j - a c Lambda_Y - sigma sigma' Lambda_X
// with sigma' = 1 / (2 / sigma1 - sigma), a = 2 sigma' / e, and the pair swaps.  The
// step-k forcing coefficient of the block recurrence is Lambda_Y before that
// step's update: it goes to row k - 2 of the table (FP64 and/or FP32), and the
// final Lambda_Y to lamY for the reconstruction.
__global__ __launch_bounds__(kThreads) void k_rchfsi_coef(const double* __restrict__ ritz,
                                                           int64_t b, double e, double c,
                                                           double sigma1, int p, double* coef64,
                                                           float* coef32, double* lamY) {
  const int64_t j = blockIdx.x * int64_t(kThreads) + threadIdx.x;
  if (j >= b) return;
  const double lam = ritz[j];
  const double gamma = 2.0 / sigma1;
  double lx = 1.0, ly = (sigma1 / e) * (lam - c), sigma = sigma1;
  for (int k = 2; k <= p; ++k) {
    const double sigma2 = 1.0 / (gamma - sigma);
    const double a = 2.0 * sigma2 / e;
    if (coef64) coef64[int64_t(k - 2) * b + j] = ly;
    if (coef32) coef32[int64_t(k - 2) * b + j] = float(ly);
    const double ln = a * ly * lam - a * c * ly - sigma * sigma2 * lx;
    lx = ly;
    ly = ln;
    sigma = sigma2;
  }
  lamY[j] = ly;
}

__global__ __launch_bounds__(kThreads) void k_rchfsi_init_f64(const double* __restrict__ R,
                                                               int64_t ldr, int64_t n, int64_t b,
                                                               double scale, double* RY,
                                                               double* RX, int64_t ld) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    RY[i + j * ld] = scale * R[i + j * ldr];
    RX[i + j * ld] = 0.0;
  }
}

template <typename TR>
__global__ __launch_bounds__(kThreads) void k_reconstruct(const TR* __restrict__ RY, int64_t ldry,
                                                           const double* __restrict__ dinv,
                                                           const double* __restrict__ X,
                                                           int64_t ldx,
                                                           const double* __restrict__ lamY,
                                                           double* Yp, int64_t ldy, int64_t n,
                                                           int64_t b) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    double r = double(RY[i + j * ldry]);
    if (dinv) r *= dinv[i];
    Yp[i + j * ldy] = r + X[i + j * ldx] * lamY[j];
  }
}

// one workgroup per column: 16-byte loads (two doubles per lane) when the
// column is 16-byte aligned, per-lane partial sums, a butterfly across each
// wave's 64 lanes, then the wave sums in a fixed order (deterministic)
__global__ __launch_bounds__(kThreads) void k_column_norms(const double* __restrict__ R,
                                                            int64_t ldr, int64_t n,
                                                            double* out) {
  __shared__ double wsum[kThreads / 64];
  const int64_t j = blockIdx.x;
  const double* col = R + j * ldr;
  double s0 = 0.0, s1 = 0.0;
  int64_t tail = 0;
  if ((reinterpret_cast<uintptr_t>(col) & 15) == 0) {
    const int64_t nv = n / 2;
    const double2* cv = reinterpret_cast<const double2*>(col);
#pragma unroll 4
    for (int64_t v = threadIdx.x; v < nv; v += kThreads) {
      const double2 x = cv[v];
      s0 += x.x * x.x;
      s1 += x.y * x.y;
    }
    tail = 2 * nv;
  }
  for (int64_t i = tail + threadIdx.x; i < n; i += kThreads) {
    const double v = col[i];
    s0 += v * v;
  }
  double s = s0 + s1;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += wsum[w];
    out[j] = sqrt(t);
  }
}

__global__ __launch_bounds__(kThreads) void k_convert(const double* __restrict__ in, int64_t ldi,
                                                       float* out, int64_t ldo, int64_t n,
                                                       int64_t m) {
  const int64_t total = n * m;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    out[i + j * ldo] = float(in[i + j * ldi]);
  }
}

// FP64 -> bfloat16 (rounded to FP32, then to bfloat16 nearest-even)
__global__ __launch_bounds__(kThreads) void k_convert_bf16(const double* __restrict__ in,
                                                            int64_t ldi, uint16_t* out,
                                                            int64_t ldo, int64_t n, int64_t m) {
  const int64_t total = n * m;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    uint32_t u = __float_as_uint(float(in[i + j * ldi]));
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      out[i + j * ldo] = uint16_t((u >> 16) | 0x40u);
    } else {
      u += 0x7fffu + ((u >> 16) & 1u);
      out[i + j * ldo] = uint16_t(u >> 16);
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_copy(const double* __restrict__ in, int64_t ldi,
                                                    double* out, int64_t ldo, int64_t n,
                                                    int64_t b) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    out[i + j * ldo] = in[i + j * ldi];
  }
}

__global__ __launch_bounds__(kThreads) void k_gram_scale_vec(const double* __restrict__ G,
                                                              int64_t ldg, int64_t b, double* s,
                                                              int* bad) {
  const int64_t j = blockIdx.x * int64_t(kThreads) + threadIdx.x;
  if (j >= b) return;
  const double d = G[j + j * ldg];
  if (!(d > 0.0) || !isfinite(d)) {
    atomicExch(bad, 1);
    s[j] = 1.0;
  } else {
    s[j] = 1.0 / sqrt(d);
  }
}

__global__ __launch_bounds__(kThreads) void k_scale_sym(const double* __restrict__ G, int64_t ldg,
                                                         int64_t b, const double* __restrict__ s,
                                                         double* out, int64_t ldo) {
  const int64_t total = b * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / b, i = idx - j * b;
    out[i + j * ldo] = s[i] * G[i + j * ldg] * s[j];
  }
}

__global__ __launch_bounds__(kThreads) void k_symmetrize(double* A, int64_t lda, int64_t b) {
  const int64_t total = b * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / b, i = idx - j * b;
    if (i < j) {
      const double v = 0.5 * (A[i + j * lda] + A[j + i * lda]);
      A[i + j * lda] = v;
      A[j + i * lda] = v;
    }
  }
}

// Symmetric matrix of which only the block panels on and below the diagonal
// were formed (panel width w: column block p holds rows >= p*w): the upper
// part outside the diagonal blocks is copied from the lower part, entries of
// the diagonal blocks (both triangles formed) are averaged.
__global__ __launch_bounds__(kThreads) void k_symmetrize_panels(double* A, int64_t lda, int64_t b,
                                                                 int64_t w) {
  const int64_t total = b * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / b, i = idx - j * b;
    if (i < j) {
      if (i >= (j / w) * w) {
        const double v = 0.5 * (A[i + j * lda] + A[j + i * lda]);
        A[i + j * lda] = v;
        A[j + i * lda] = v;
      } else {
        A[i + j * lda] = A[j + i * lda];
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_scale_columns(double* M, int64_t ldm, int64_t n,
                                                             int64_t b,
                                                             const double* __restrict__ v) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    M[i + j * ldm] *= v[j];
  }
}

__global__ __launch_bounds__(kThreads) void k_set_identity(double* M, int64_t ldm, int64_t n) {
  const int64_t total = n * n;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    M[i + j * ldm] = (i == j) ? 1.0 : 0.0;
  }
}

__global__ __launch_bounds__(kThreads) void k_zero(uint32_t* p, int64_t words) {
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < words;
       idx += int64_t(gridDim.x) * kThreads)
    p[idx] = 0u;
}

__global__ __launch_bounds__(kThreads) void k_zero_bytes(unsigned char* p, int64_t nbytes) {
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < nbytes;
       idx += int64_t(gridDim.x) * kThreads)
    p[idx] = 0;
}

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): a counter-based
// generator; each element draws from its own counter so the fill is
// independent of the launch shape.
__device__ inline void philox_round(uint32_t c[4], uint32_t k[2]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint64_t p0 = uint64_t(M0) * c[0];
  const uint64_t p1 = uint64_t(M1) * c[2];
  const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
  const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
  const uint32_t n0 = hi1 ^ c[1] ^ k[0];
  const uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

__device__ inline void philox10(uint32_t c[4], uint32_t k[2]) {
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k);
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
  }
}

__global__ __launch_bounds__(kThreads) void k_gaussian(double* X, int64_t ldx, int64_t n,
                                                        int64_t b, uint64_t seed) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    uint32_t c[4] = {uint32_t(idx), uint32_t(uint64_t(idx) >> 32), 0u, 0u};
    uint32_t k[2] = {uint32_t(seed), uint32_t(seed >> 32)};
    philox10(c, k);
    // two 53-bit uniforms in (0,1], Box-Muller (cosine branch)
    const uint64_t a = (uint64_t(c[0]) << 21) ^ (uint64_t(c[1]) >> 11);
    const uint64_t bb = (uint64_t(c[2]) << 21) ^ (uint64_t(c[3]) >> 11);
    const double u1 = (double(a & ((uint64_t(1) << 53) - 1)) + 1.0) * (1.0 / 9007199254740992.0);
    const double u2 = double(bb & ((uint64_t(1) << 53) - 1)) * (1.0 / 9007199254740992.0);
    X[i + j * ldx] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

__global__ __launch_bounds__(kThreads) void k_check_finite(const double* __restrict__ v, int64_t n,
                                                            int* flag) {
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < n;
       idx += int64_t(gridDim.x) * kThreads)
    if (!isfinite(v[idx])) atomicExch(flag, 1);
}

}  // namespace

hipError_t rchfsi_init_f32(const double* R, int64_t ldr, int64_t n, int64_t b, double scale,
                           float* RY, float* RX, float* Ycopy, int64_t ld32, hipStream_t st) {
  k_rchfsi_init_f32<<<grid_for(n * b), kThreads, 0, st>>>(R, ldr, n, b, scale, RY, RX, Ycopy,
                                                          ld32);
  return hipGetLastError();
}

hipError_t rchfsi_coef(const double* ritz, int64_t b, double e, double c, double sigma1, int p,
                       double* coef64, float* coef32, double* lamY, hipStream_t st) {
  if (b <= 0) return hipSuccess;
  k_rchfsi_coef<<<grid_for(b), kThreads, 0, st>>>(ritz, b, e, c, sigma1, p, coef64, coef32, lamY);
  return hipGetLastError();
}

hipError_t rchfsi_init_f64(const double* R, int64_t ldr, int64_t n, int64_t b, double scale,
                           double* RY, double* RX, int64_t ld, hipStream_t st) {
  k_rchfsi_init_f64<<<grid_for(n * b), kThreads, 0, st>>>(R, ldr, n, b, scale, RY, RX, ld);
  return hipGetLastError();
}

hipError_t rchfsi_reconstruct_f32(const float* RY, int64_t ldry, const double* dinv,
                                  const double* X, int64_t ldx, const double* lamY, double* Yp,
                                  int64_t ldy, int64_t n, int64_t b, hipStream_t st) {
  k_reconstruct<float><<<grid_for(n * b), kThreads, 0, st>>>(RY, ldry, dinv, X, ldx, lamY, Yp,
                                                             ldy, n, b);
  return hipGetLastError();
}

hipError_t rchfsi_reconstruct_f64(const double* RY, int64_t ldry, const double* dinv,
                                  const double* X, int64_t ldx, const double* lamY, double* Yp,
                                  int64_t ldy, int64_t n, int64_t b, hipStream_t st) {
  k_reconstruct<double><<<grid_for(n * b), kThreads, 0, st>>>(RY, ldry, dinv, X, ldx, lamY, Yp,
                                                              ldy, n, b);
  return hipGetLastError();
}

hipError_t column_norms(const double* R, int64_t ldr, int64_t n, int64_t b, double* out,
                        hipStream_t st) {
  if (b <= 0) return hipSuccess;
  k_column_norms<<<dim3(unsigned(b)), kThreads, 0, st>>>(R, ldr, n, out);
  return hipGetLastError();
}

hipError_t convert_f64_f32(const double* in, int64_t ldi, float* out, int64_t ldo, int64_t n,
                           int64_t m, hipStream_t st) {
  k_convert<<<grid_for(n * m), kThreads, 0, st>>>(in, ldi, out, ldo, n, m);
  return hipGetLastError();
}

hipError_t convert_f64_bf16(const double* in, int64_t ldi, uint16_t* out, int64_t ldo, int64_t n,
                            int64_t m, hipStream_t st) {
  k_convert_bf16<<<grid_for(n * m), kThreads, 0, st>>>(in, ldi, out, ldo, n, m);
  return hipGetLastError();
}

hipError_t copy_block(const double* in, int64_t ldi, double* out, int64_t ldo, int64_t n,
                      int64_t b, hipStream_t st) {
  k_copy<<<grid_for(n * b), kThreads, 0, st>>>(in, ldi, out, ldo, n, b);
  return hipGetLastError();
}

hipError_t scale_gram(const double* G, int64_t ldg, int64_t b, double* Gs, int64_t lds,
                      double* s, int* bad_flag, hipStream_t st) {
  k_gram_scale_vec<<<grid_for(b), kThreads, 0, st>>>(G, ldg, b, s, bad_flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scale_sym<<<grid_for(b * b), kThreads, 0, st>>>(G, ldg, b, s, Gs, lds);
  return hipGetLastError();
}

hipError_t scale_sym(const double* G, int64_t ldg, int64_t b, const double* s, double* out,
                     int64_t ldo, hipStream_t st) {
  k_scale_sym<<<grid_for(b * b), kThreads, 0, st>>>(G, ldg, b, s, out, ldo);
  return hipGetLastError();
}

hipError_t symmetrize(double* A, int64_t lda, int64_t b, hipStream_t st) {
  k_symmetrize<<<grid_for(b * b), kThreads, 0, st>>>(A, lda, b);
  return hipGetLastError();
}

hipError_t symmetrize_panels(double* A, int64_t lda, int64_t b, int64_t w, hipStream_t st) {
  if (w < 1) return hipErrorInvalidValue;
  k_symmetrize_panels<<<grid_for(b * b), kThreads, 0, st>>>(A, lda, b, w);
  return hipGetLastError();
}

hipError_t scale_columns(double* M, int64_t ldm, int64_t n, int64_t b, const double* v,
                         hipStream_t st) {
  k_scale_columns<<<grid_for(n * b), kThreads, 0, st>>>(M, ldm, n, b, v);
  return hipGetLastError();
}

hipError_t set_identity(double* M, int64_t ldm, int64_t n, hipStream_t st) {
  k_set_identity<<<grid_for(n * n), kThreads, 0, st>>>(M, ldm, n);
  return hipGetLastError();
}

hipError_t fill_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if (reinterpret_cast<uintptr_t>(p) % 4 == 0 && bytes % 4 == 0) {
    k_zero<<<grid_for(int64_t(bytes / 4)), kThreads, 0, st>>>(static_cast<uint32_t*>(p),
                                                               int64_t(bytes / 4));
  } else {
    k_zero_bytes<<<grid_for(int64_t(bytes)), kThreads, 0, st>>>(static_cast<unsigned char*>(p),
                                                                int64_t(bytes));
  }
  return hipGetLastError();
}

hipError_t fill_gaussian(double* X, int64_t ldx, int64_t n, int64_t b, uint64_t seed,
                         hipStream_t st) {
  k_gaussian<<<grid_for(n * b), kThreads, 0, st>>>(X, ldx, n, b, seed);
  return hipGetLastError();
}

hipError_t check_finite(const double* v, int64_t n, int* flag, hipStream_t st) {
  k_check_finite<<<grid_for(n), kThreads, 0, st>>>(v, n, flag);
  return hipGetLastError();
}

}  // namespace chfsi

namespace chfsi {
namespace {
__global__ __launch_bounds__(256) void k_convert_up(const float* __restrict__ in, int64_t ldi,
                                                     double* out, int64_t ldo, int64_t n,
                                                     int64_t m) {
  const int64_t total = n * m;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t j = idx / n, i = idx - j * n;
    out[i + j * ldo] = double(in[i + j * ldi]);
  }
}
__global__ __launch_bounds__(256) void k_ones(float* p, int64_t n) {
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < n;
       idx += int64_t(gridDim.x) * 256)
    p[idx] = 1.0f;
}
}  // namespace

hipError_t convert_f32_f64(const float* in, int64_t ldi, double* out, int64_t ldo, int64_t n,
                           int64_t m, hipStream_t st) {
  k_convert_up<<<grid_for(n * m), 256, 0, st>>>(in, ldi, out, ldo, n, m);
  return hipGetLastError();
}

hipError_t fill_ones_f32(float* p, int64_t n, hipStream_t st) {
  k_ones<<<grid_for(n), 256, 0, st>>>(p, n);
  return hipGetLastError();
}
}  // namespace chfsi

namespace chfsi {
namespace {
__global__ __launch_bounds__(256) void k_scale_rows(double* M, int64_t ldm, int64_t n, int64_t b,
                                                     const double* __restrict__ v) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t j = idx / n, i = idx - j * n;
    M[i + j * ldm] *= v[i];
  }
}
}  // namespace

hipError_t scale_rows(double* M, int64_t ldm, int64_t n, int64_t b, const double* v,
                      hipStream_t st) {
  k_scale_rows<<<grid_for(n * b), 256, 0, st>>>(M, ldm, n, b, v);
  return hipGetLastError();
}
}  // namespace chfsi
