// Complex Hermitian problems (Section 4.3): layout kernels that let the real
// MFMA GEMM carry the complex residual filter.
//
// A complex product A Z (A Hermitian n x n, Z n x b) is one real product on
// planar data:
//   [Re(AZ) | Im(AZ)] = L Z~,   L = [A_r | A_i]  (n x 2n),
//   Z~ = [[Z_r, Z_i], [-Z_i, Z_r]]               (2n x 2b),
// where A_r(m,k) = Re A(m,k), A_i(m,k) = Im A(m,k).  The library keeps L
// k-contiguous (row m of L at L + m * 2n): since A(m,k) = conj(A(k,m)), row m
// of L is [Re A(:,m), -Im A(:,m)], read down column m of the column-major
// input.  Blocks are kept planar (n x 2b: real parts in columns 0..b-1,
// imaginary parts in b..2b-1); the recurrence's coefficients are real, so the
// fused three-term update of the real path applies to both halves unchanged.
// Interleaved complex data (the ABI's layout) is (re, im) pairs of doubles.
//
// All are grid-stride kernels with 64-bit indexing.
#include "internal.h"

#include <cstdint>

namespace chfsi {

namespace {

constexpr int kThreads = 256;

inline int64_t grid_for(int64_t total, int64_t cap = 65536) {
  int64_t g = (total + kThreads - 1) / kThreads;
  if (g < 1) g = 1;
  return g > cap ? cap : g;
}

template <typename F>
__device__ __forceinline__ F to_elem(double v) {
  return F(v);
}
template <>
__device__ __forceinline__ uint16_t to_elem<uint16_t>(double v) {
  // bfloat16, round to nearest even (hardware conversion)
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(float(v)));
}

// L (n x 2n, k-contiguous rows) from the interleaved column-major Hermitian A
template <typename F>
__global__ __launch_bounds__(kThreads) void k_herm_planar(const double* __restrict__ A, int64_t lda,
                                                          int64_t n, F* __restrict__ L) {
  const int64_t total = n * n;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t m = idx / n, k = idx - m * n;
    const double re = A[2 * (k + m * lda)], im = A[2 * (k + m * lda) + 1];
    L[m * 2 * n + k] = to_elem<F>(re);
    L[m * 2 * n + n + k] = to_elem<F>(-im);
  }
}

// [d; d] (length 2n) in the filter precision; d = 1 when dinv is null
template <typename F>
__global__ __launch_bounds__(kThreads) void k_dup_dinv(const double* __restrict__ dinv, int64_t n,
                                                       F* __restrict__ out) {
  for (int64_t i = blockIdx.x * int64_t(kThreads) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kThreads) {
    const F v = F(dinv ? dinv[i] : 1.0);
    out[i] = v;
    out[n + i] = v;
  }
}

// R_Y = scale * R, R_X = 0, Yc = R (planar, ld n) from the interleaved residual
template <typename F>
__global__ __launch_bounds__(kThreads) void k_cinit(const double* __restrict__ R, int64_t ldr,
                                                    int64_t n, int64_t b, double scale,
                                                    F* __restrict__ RY, F* __restrict__ RX,
                                                    F* __restrict__ Yc) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    const double re = R[2 * (i + j * ldr)], im = R[2 * (i + j * ldr) + 1];
    const int64_t pr = i + j * n, pi = i + (b + j) * n;
    RY[pr] = F(scale * re);
    RY[pi] = F(scale * im);
    RX[pr] = F(0);
    RX[pi] = F(0);
    Yc[pr] = F(re);
    Yc[pi] = F(im);
  }
}

// Z~ (2n x 2b, ld 2n) from the planar block Z (n x 2b, ld n)
template <typename F>
__global__ __launch_bounds__(kThreads) void k_crhs(const F* __restrict__ Z, int64_t n, int64_t b,
                                                   F* __restrict__ Zt) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, k = idx - j * n;
    const F re = Z[k + j * n], im = Z[k + (b + j) * n];
    F* c0 = Zt + j * 2 * n;          // column j: [Z_r; -Z_i]
    F* c1 = Zt + (b + j) * 2 * n;    // column b + j: [Z_i; Z_r]
    c0[k] = re;
    c0[n + k] = -im;
    c1[k] = im;
    c1[n + k] = re;
  }
}

// Yp = D^{-1} R_Y + X Lambda_Y (interleaved complex, FP64)
template <typename F>
__global__ __launch_bounds__(kThreads) void k_crecon(const F* __restrict__ RY,
                                                     const double* __restrict__ dinv,
                                                     const double* __restrict__ X, int64_t ldx,
                                                     const double* __restrict__ lam, double* Yp,
                                                     int64_t ldy, int64_t n, int64_t b) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    const double d = dinv ? dinv[i] : 1.0, l = lam[j];
    const double xr = X[2 * (i + j * ldx)], xi = X[2 * (i + j * ldx) + 1];
    const double re = d * double(RY[i + j * n]) + xr * l;
    const double im = d * double(RY[i + (b + j) * n]) + xi * l;
    Yp[2 * (i + j * ldy)] = re;
    Yp[2 * (i + j * ldy) + 1] = im;
  }
}

// planar P (n x 2b, ld n) from interleaved Z (ld ldz), and back
__global__ __launch_bounds__(kThreads) void k_to_planar(const double* __restrict__ Z, int64_t ldz,
                                                        int64_t n, int64_t b,
                                                        double* __restrict__ P) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    P[i + j * n] = Z[2 * (i + j * ldz)];
    P[i + (b + j) * n] = Z[2 * (i + j * ldz) + 1];
  }
}

__global__ __launch_bounds__(kThreads) void k_from_planar(const double* __restrict__ P, int64_t n,
                                                          int64_t b, double* __restrict__ Z,
                                                          int64_t ldz) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    Z[2 * (i + j * ldz)] = P[i + j * n];
    Z[2 * (i + j * ldz) + 1] = P[i + (b + j) * n];
  }
}

// The real embedding M(G) = [[G_r, -G_i], [G_i, G_r]] (2b x 2b, ld 2b) of
// G = Y^H W, G_r = P11 + P22 and G_i = P12 - P21 with P11 = Y_r^T W_r,
// P22 = Y_i^T W_i, P12 = Y_r^T W_i, P21 = Y_i^T W_r.  For a Hermitian
// operator G_r is symmetric and G_i antisymmetric, so the lower triangles
// (i >= j) of the four b x b blocks (consecutive in P4, ld b) determine M,
// which comes out exactly symmetric.
__global__ __launch_bounds__(kThreads) void k_embed_gram_lower(const double* __restrict__ P4,
                                                               int64_t b,
                                                               double* __restrict__ M) {
  const int64_t m = 2 * b, total = m * m, bb = b * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t c = idx / m, r = idx - c * m;
    const int64_t i = r % b, j = c % b;
    const int64_t lo = i >= j ? i + j * b : j + i * b;     // lower-triangle entry
    const double gr = P4[lo] + P4[bb + lo];
    double gi = P4[2 * bb + lo] - P4[3 * bb + lo];
    if (i == j) gi = 0.0;
    if (i < j) gi = -gi;
    const bool top = r < b, left = c < b;
    M[r + c * m] = top == left ? gr : (top ? -gi : gi);
  }
}

// SVQB for the embedded problem: planar W (b x 2k, ld b; real parts then
// imaginary parts) from the first vector of the eigenvalue pairs first,
// first + 2, ... of the m x m eigenvector matrix E (ld lde), scaled per pair
// by gs[j] and per row by s[i]
__global__ __launch_bounds__(kThreads) void k_pairs_to_planar(const double* __restrict__ E,
                                                              int64_t lde, int64_t b,
                                                              int64_t first, int64_t k,
                                                              const double* __restrict__ gs,
                                                              const double* __restrict__ s,
                                                              double* __restrict__ W) {
  const int64_t total = b * k;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / b, i = idx - j * b;
    const double f = gs[j] * s[i];
    const double* e = E + (first + 2 * j) * lde;
    W[i + j * b] = e[i] * f;
    W[i + (k + j) * b] = e[b + i] * f;
  }
}

// M(W) = [[W_r, -W_i], [W_i, W_r]] (2b x 2k, ld ldm) from planar W (b x 2k, ld b)
__global__ __launch_bounds__(kThreads) void k_embed_block(const double* __restrict__ W, int64_t b,
                                                          int64_t k, double* __restrict__ M,
                                                          int64_t ldm) {
  const int64_t total = b * k;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / b, i = idx - j * b;
    const double wr = W[i + j * b], wi = W[i + (k + j) * b];
    M[i + j * ldm] = wr;
    M[(b + i) + j * ldm] = wi;
    M[i + (k + j) * ldm] = -wi;
    M[(b + i) + (k + j) * ldm] = wr;
  }
}

// Zx (b x 2b planar, ld b) from the first vector of each of the first k
// eigenvalue pairs of an embedded problem's eigenvector matrix T (2b rows,
// ld ldt): x_j = T(0:b, 2j) + i T(b:2b, 2j); columns k..b-1 of both halves
// are zero
__global__ __launch_bounds__(kThreads) void k_select_pairs_n(const double* __restrict__ T,
                                                             int64_t ldt, int64_t b, int64_t k,
                                                             double* __restrict__ Zx) {
  const int64_t total = b * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / b, i = idx - j * b;
    const bool keep = j < k;
    Zx[i + j * b] = keep ? T[i + (2 * j) * ldt] : 0.0;
    Zx[i + (b + j) * b] = keep ? T[(b + i) + (2 * j) * ldt] : 0.0;
  }
}

}  // namespace

hipError_t pairs_to_planar(const double* E, int64_t lde, int64_t b, int64_t first, int64_t k,
                           const double* gs, const double* s, double* W, hipStream_t st) {
  k_pairs_to_planar<<<grid_for(b * k), kThreads, 0, st>>>(E, lde, b, first, k, gs, s, W);
  return hipGetLastError();
}

hipError_t embed_block(const double* W, int64_t b, int64_t k, double* M, int64_t ldm,
                       hipStream_t st) {
  k_embed_block<<<grid_for(b * k), kThreads, 0, st>>>(W, b, k, M, ldm);
  return hipGetLastError();
}

hipError_t select_pairs_n(const double* T, int64_t ldt, int64_t b, int64_t k, double* Zx,
                          hipStream_t st) {
  k_select_pairs_n<<<grid_for(b * b), kThreads, 0, st>>>(T, ldt, b, k, Zx);
  return hipGetLastError();
}

hipError_t cplx_to_planar(const double* Z, int64_t ldz, int64_t n, int64_t b, double* P,
                          hipStream_t st) {
  k_to_planar<<<grid_for(n * b), kThreads, 0, st>>>(Z, ldz, n, b, P);
  return hipGetLastError();
}

hipError_t planar_to_cplx(const double* P, int64_t n, int64_t b, double* Z, int64_t ldz,
                          hipStream_t st) {
  k_from_planar<<<grid_for(n * b), kThreads, 0, st>>>(P, n, b, Z, ldz);
  return hipGetLastError();
}

hipError_t embed_gram_lower(const double* P4, int64_t b, double* M, hipStream_t st) {
  k_embed_gram_lower<<<grid_for(4 * b * b), kThreads, 0, st>>>(P4, b, M);
  return hipGetLastError();
}

template <typename F>
hipError_t herm_to_planar(const double* A, int64_t lda, int64_t n, F* L, hipStream_t st) {
  k_herm_planar<F><<<grid_for(n * n), kThreads, 0, st>>>(A, lda, n, L);
  return hipGetLastError();
}

template <typename F>
hipError_t dup_dinv(const double* dinv, int64_t n, F* out, hipStream_t st) {
  k_dup_dinv<F><<<grid_for(n), kThreads, 0, st>>>(dinv, n, out);
  return hipGetLastError();
}

template <typename F>
hipError_t cplx_init(const double* R, int64_t ldr, int64_t n, int64_t b, double scale, F* RY,
                     F* RX, F* Yc, hipStream_t st) {
  k_cinit<F><<<grid_for(n * b), kThreads, 0, st>>>(R, ldr, n, b, scale, RY, RX, Yc);
  return hipGetLastError();
}

template <typename F>
hipError_t cplx_rhs(const F* Z, int64_t n, int64_t b, F* Zt, hipStream_t st) {
  k_crhs<F><<<grid_for(n * b), kThreads, 0, st>>>(Z, n, b, Zt);
  return hipGetLastError();
}

template <typename F>
hipError_t cplx_reconstruct(const F* RY, const double* dinv, const double* X, int64_t ldx,
                            const double* lamY, double* Yp, int64_t ldy, int64_t n, int64_t b,
                            hipStream_t st) {
  k_crecon<F><<<grid_for(n * b), kThreads, 0, st>>>(RY, dinv, X, ldx, lamY, Yp, ldy, n, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Equal complex Ritz values: a G-orthonormal basis of a cluster's eigenspace
// from the embedded eigenvectors, by pivoted Gram-Schmidt in one workgroup.
//
// The 2 ncl columns of E (each [Re u; Im u], 2 cd rows, ld lde) are read as
// complex candidate vectors u_v of length cd.  G is the identity (Mg null) or
// the Hermitian metric with G(i, j) = Mg(i, j) + i Mg(cd + i, j) (the real
// embedding M(G), ld ldm).  Each step keeps the candidate that retains the
// largest part of its G-norm outside the vectors kept so far (with the kept
// q_a G-orthonormal the coefficients are (G q_a)^H u and the remainder is
// |u|_G^2 - sum |coefficient|^2), projects it twice, and normalises it.  The
// kept vectors overwrite E as the pairs [Re q; Im q], [-Im q; Re q].  status:
// 0, or 1 when fewer than ncl independent directions are found (E untouched).
// work: (2 ncl + 2 ncl + 2) cd complex + 2 ncl doubles.
// ---------------------------------------------------------------------------
namespace {

constexpr int kGsThreads = 256;

// block sum of (re, im) pairs; every thread gets the result
__device__ double2 block_sum2(double2 v, double2* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kGsThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[threadIdx.x].x += red[threadIdx.x + w].x;
      red[threadIdx.x].y += red[threadIdx.x + w].y;
    }
    __syncthreads();
  }
  const double2 r = red[0];
  __syncthreads();
  return r;
}

// conj(a) . b over cd complex entries
__device__ double2 cdot(const double2* a, const double2* b, int64_t cd, double2* red) {
  double2 s = make_double2(0.0, 0.0);
  for (int64_t i = threadIdx.x; i < cd; i += kGsThreads) {
    s.x += a[i].x * b[i].x + a[i].y * b[i].y;
    s.y += a[i].x * b[i].y - a[i].y * b[i].x;
  }
  return block_sum2(s, red);
}

// out = G u
__device__ void apply_metric(const double* Mg, int64_t ldm, const double2* u, int64_t cd,
                             double2* out) {
  __syncthreads();
  for (int64_t i = threadIdx.x; i < cd; i += kGsThreads) {
    if (!Mg) {
      out[i] = u[i];
      continue;
    }
    double re = 0.0, im = 0.0;
    for (int64_t j = 0; j < cd; ++j) {
      const double gr = Mg[i + j * ldm], gi = Mg[cd + i + j * ldm];
      re += gr * u[j].x - gi * u[j].y;
      im += gr * u[j].y + gi * u[j].x;
    }
    out[i] = make_double2(re, im);
  }
  __syncthreads();
}

__global__ __launch_bounds__(kGsThreads) void k_cluster_gs(double* E, int64_t lde, int64_t cd,
                                                           int ncl, const double* Mg, int64_t ldm,
                                                           double* work, int* status) {
  __shared__ double2 red[kGsThreads];
  __shared__ int best_s;
  const int cols = 2 * ncl;
  double2* cand = reinterpret_cast<double2*>(work);
  double2* q = cand + int64_t(cols) * cd;
  double2* Gq = q + int64_t(ncl) * cd;
  double2* u = Gq + int64_t(ncl) * cd;
  double2* Gu = u + cd;
  double* n0 = reinterpret_cast<double*>(Gu + cd);
  double* used = n0 + cols;
  for (int v = 0; v < cols; ++v) {
    for (int64_t i = threadIdx.x; i < cd; i += kGsThreads)
      cand[int64_t(v) * cd + i] = make_double2(E[v * lde + i], E[v * lde + cd + i]);
    apply_metric(Mg, ldm, cand + int64_t(v) * cd, cd, Gu);
    const double2 r = cdot(cand + int64_t(v) * cd, Gu, cd, red);
    if (threadIdx.x == 0) {
      n0[v] = sqrt(fmax(r.x, 0.0));
      used[v] = 0.0;
    }
  }
  __syncthreads();
  int kept = 0;
  for (int t = 0; t < ncl; ++t) {
    // the candidate keeping the largest fraction of its norm
    double best_ratio = 0.0;
    int best = -1;
    for (int v = 0; v < cols; ++v) {
      if (used[v] != 0.0 || !(n0[v] > 0.0)) continue;
      double rem = n0[v] * n0[v];
      for (int a = 0; a < kept; ++a) {
        const double2 d = cdot(Gq + int64_t(a) * cd, cand + int64_t(v) * cd, cd, red);
        rem -= d.x * d.x + d.y * d.y;
      }
      const double ratio = sqrt(fmax(rem, 0.0)) / n0[v];
      if (ratio > best_ratio) {
        best_ratio = ratio;
        best = v;
      }
    }
    if (threadIdx.x == 0) best_s = (best >= 0 && best_ratio > 1e-6) ? best : -1;
    __syncthreads();
    const int bsel = best_s;
    __syncthreads();
    if (bsel < 0) break;
    if (threadIdx.x == 0) used[bsel] = 1.0;
    for (int64_t i = threadIdx.x; i < cd; i += kGsThreads) u[i] = cand[int64_t(bsel) * cd + i];
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass)     // projection, repeated once for accuracy
      for (int a = 0; a < kept; ++a) {
        const double2 d = cdot(Gq + int64_t(a) * cd, u, cd, red);
        for (int64_t i = threadIdx.x; i < cd; i += kGsThreads) {
          const double2 qa = q[int64_t(a) * cd + i];
          u[i].x -= d.x * qa.x - d.y * qa.y;
          u[i].y -= d.x * qa.y + d.y * qa.x;
        }
        __syncthreads();
      }
    apply_metric(Mg, ldm, u, cd, Gu);
    const double2 r = cdot(u, Gu, cd, red);
    const double nrm = sqrt(fmax(r.x, 0.0));
    if (!(nrm > 0.0)) break;
    for (int64_t i = threadIdx.x; i < cd; i += kGsThreads) {
      q[int64_t(kept) * cd + i] = make_double2(u[i].x / nrm, u[i].y / nrm);
      Gq[int64_t(kept) * cd + i] = make_double2(Gu[i].x / nrm, Gu[i].y / nrm);
    }
    __syncthreads();
    ++kept;
  }
  if (kept != ncl) {
    if (threadIdx.x == 0) *status = 1;
    return;
  }
  for (int t = 0; t < ncl; ++t)
    for (int64_t i = threadIdx.x; i < cd; i += kGsThreads) {
      const double2 x = q[int64_t(t) * cd + i];
      E[(2 * t) * lde + i] = x.x;
      E[(2 * t) * lde + cd + i] = x.y;
      E[(2 * t + 1) * lde + i] = -x.y;
      E[(2 * t + 1) * lde + cd + i] = x.x;
    }
  if (threadIdx.x == 0) *status = 0;
}

}  // namespace

size_t cluster_gs_work_bytes(int64_t cd, int64_t ncl) {
  return size_t(4 * ncl + 2) * size_t(cd) * 2 * sizeof(double) + size_t(2 * ncl) * sizeof(double);
}

hipError_t cluster_orthonormalize(double* E, int64_t lde, int64_t cd, int64_t ncl,
                                  const double* Mg, int64_t ldm, double* work, int* status,
                                  hipStream_t st) {
  if (ncl <= 0 || cd <= 0) return hipSuccess;
  if (ncl > 0x3fffffff) return hipErrorInvalidValue;
  k_cluster_gs<<<1, kGsThreads, 0, st>>>(E, lde, cd, int(ncl), Mg, ldm, work, status);
  return hipGetLastError();
}

template hipError_t herm_to_planar<float>(const double*, int64_t, int64_t, float*, hipStream_t);
template hipError_t herm_to_planar<double>(const double*, int64_t, int64_t, double*, hipStream_t);
template hipError_t herm_to_planar<uint16_t>(const double*, int64_t, int64_t, uint16_t*,
                                             hipStream_t);
template hipError_t dup_dinv<float>(const double*, int64_t, float*, hipStream_t);
template hipError_t dup_dinv<double>(const double*, int64_t, double*, hipStream_t);
template hipError_t cplx_init<float>(const double*, int64_t, int64_t, int64_t, double, float*,
                                     float*, float*, hipStream_t);
template hipError_t cplx_init<double>(const double*, int64_t, int64_t, int64_t, double, double*,
                                      double*, double*, hipStream_t);
template hipError_t cplx_rhs<float>(const float*, int64_t, int64_t, float*, hipStream_t);
template hipError_t cplx_rhs<double>(const double*, int64_t, int64_t, double*, hipStream_t);
template hipError_t cplx_reconstruct<float>(const float*, const double*, const double*, int64_t,
                                            const double*, double*, int64_t, int64_t, int64_t,
                                            hipStream_t);
template hipError_t cplx_reconstruct<double>(const double*, const double*, const double*, int64_t,
                                             const double*, double*, int64_t, int64_t, int64_t,
                                             hipStream_t);

}  // namespace chfsi
