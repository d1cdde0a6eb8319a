// Spectrum-bound estimates of the pencil (A, B) by a k-step Lanczos process
// on B^{-1} A in the B-inner product (the filter needs lambda_max above the
// whole spectrum of B^{-1} A; Section 2.1 takes the bounds as estimates).
//
//   v_1 = v_0 / ||v_0||_B
//   for j = 1..k:  w = A v_j;  u = B^{-1} w  (preconditioned CG, D^{-1});
//                  alpha_j = v_j^T w;  u -= alpha_j v_j + beta_{j-1} v_{j-1};
//                  beta_j = ||u||_B;  v_{j+1} = u / beta_j
//
// The B-products of the v_j are carried along (B u = w - alpha_j B v_j -
// beta_{j-1} B v_{j-1}), so each step costs one A product and the CG
// iterations.  The extreme eigenvalues theta_1 <= ... <= theta_k of the
// tridiagonal T_k = tridiag(beta, alpha, beta) with the safeguard |beta_k|
// (the "Ritz value + |beta_k|" rule of Zhou, Saad, Tiago and Chelikowsky,
// 2006) give lower = theta_1 - |beta_k| and upper = theta_k + |beta_k|.
//
// Vectors are FP64 of length L (n for real pencils; 2n planar for complex
// Hermitian pencils, whose real embedding has the same eigenvalues).  Dot
// products are two-stage reductions in a fixed order (bitwise reproducible).
#include "internal.h"

#include <cstdlib>

#include <algorithm>
#include <cmath>
#include <vector>

namespace chfsi {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 512;

inline int blocks_for(int64_t L) {
  int64_t g = (L + 4 * kThreads - 1) / (4 * kThreads);
  return int(std::max<int64_t>(1, std::min<int64_t>(g, kMaxBlocks)));
}

// sum of a wave's 64 values into lane 0 (fixed butterfly order)
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// block-level sum of one value per thread into out (fixed order)
__device__ inline double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kThreads / 64; ++w) s += lds[w];
  __syncthreads();
  return s;
}

// partial[blk * 2 + t] = sum over the block's share of x_t . y_t (t = 0, 1)
__global__ __launch_bounds__(kThreads) void k_dot2_partial(const double* __restrict__ x0,
                                                            const double* __restrict__ y0,
                                                            const double* __restrict__ x1,
                                                            const double* __restrict__ y1,
                                                            int64_t L, double* partial) {
  __shared__ double lds[kThreads / 64];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = blockIdx.x * int64_t(kThreads) + threadIdx.x; i < L;
       i += int64_t(gridDim.x) * kThreads) {
    s0 += x0[i] * y0[i];
    if (x1) s1 += x1[i] * y1[i];
  }
  s0 = block_sum(s0, lds);
  s1 = block_sum(s1, lds);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s0;
    partial[2 * blockIdx.x + 1] = s1;
  }
}

// *out0 (and *out1) = sum_b partial[2 b + t] over nb blocks, one wave, fixed order
__global__ __launch_bounds__(64) void k_dot2_final(const double* __restrict__ partial, int nb,
                                                   double* out0, double* out1) {
  double s0 = 0.0, s1 = 0.0;
  for (int b = threadIdx.x; b < nb; b += 64) {
    s0 += partial[2 * b];
    s1 += partial[2 * b + 1];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (threadIdx.x == 0) {
    *out0 = s0;
    if (out1) *out1 = s1;
  }
}

// out = a x + b y + c z (null terms skipped); out may alias any input
__global__ __launch_bounds__(kThreads) void k_lincomb3(double a, const double* x, double b,
                                                       const double* y, double c, const double* z,
                                                       int64_t L, double* out) {
  for (int64_t i = blockIdx.x * int64_t(kThreads) + threadIdx.x; i < L;
       i += int64_t(gridDim.x) * kThreads) {
    double v = a * x[i];
    if (y) v += b * y[i];
    if (z) v += c * z[i];
    out[i] = v;
  }
}

// out = a x - (*bp) y + c z (null z skipped): a coefficient that stays on the device
__global__ __launch_bounds__(kThreads) void k_lincomb3_dev(double a, const double* x,
                                                           const double* __restrict__ bp,
                                                           const double* y, double c,
                                                           const double* z, int64_t L,
                                                           double* out) {
  const double b = -*bp;
  for (int64_t i = blockIdx.x * int64_t(kThreads) + threadIdx.x; i < L;
       i += int64_t(gridDim.x) * kThreads) {
    double v = a * x[i];
    v += b * y[i];
    if (z) v += c * z[i];
    out[i] = v;
  }
}

// CG direction p = z + (*rz_new / *rz_old) p
__global__ __launch_bounds__(kThreads) void k_cg_dir(const double* __restrict__ rz_new,
                                                     const double* __restrict__ rz_old,
                                                     const double* z, int64_t L, double* p) {
  // (a zero residual, which a batch of iterations can run into, keeps p)
  const double beta = *rz_old != 0.0 ? *rz_new / *rz_old : 0.0;
  for (int64_t i = blockIdx.x * int64_t(kThreads) + threadIdx.x; i < L;
       i += int64_t(gridDim.x) * kThreads)
    p[i] = z[i] + beta * p[i];
}

// one CG update with alpha = *rz / *pq: x += alpha p; r -= alpha q;
// z = dinv .* r; partial sums of r . r and r . z.  A non-positive p . B p with
// a nonzero residual (B not positive definite on the Krylov space) sets the
// sticky flag *bad; a zero residual gives alpha = 0.
__global__ __launch_bounds__(kThreads) void k_cg_update(const double* __restrict__ rz,
                                                        const double* __restrict__ pq,
                                                        const double* __restrict__ p,
                                                        const double* __restrict__ q, double* x,
                                                        double* r, double* z,
                                                        const double* __restrict__ dinv,
                                                        int64_t L, double* partial, double* bad) {
  __shared__ double lds[kThreads / 64];
  const double d = *pq, rzv = *rz;
  if (!(d > 0.0) && rzv != 0.0 && blockIdx.x == 0 && threadIdx.x == 0) *bad = 1.0;
  const double alpha = d > 0.0 ? rzv / d : 0.0;
  double srr = 0.0, srz = 0.0;
  for (int64_t i = blockIdx.x * int64_t(kThreads) + threadIdx.x; i < L;
       i += int64_t(gridDim.x) * kThreads) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    const double zi = dinv ? dinv[i] * ri : ri;
    z[i] = zi;
    srr += ri * ri;
    srz += ri * zi;
  }
  srr = block_sum(srr, lds);
  srz = block_sum(srz, lds);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = srr;
    partial[2 * blockIdx.x + 1] = srz;
  }
}

// z = dinv .* r (or r)
__global__ __launch_bounds__(kThreads) void k_precond(const double* __restrict__ dinv,
                                                      const double* __restrict__ r, int64_t L,
                                                      double* z) {
  for (int64_t i = blockIdx.x * int64_t(kThreads) + threadIdx.x; i < L;
       i += int64_t(gridDim.x) * kThreads)
    z[i] = dinv ? dinv[i] * r[i] : r[i];
}

// Sturm count: eigenvalues of the symmetric tridiagonal (a, b) below x
int sturm_below(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int count = 0;
  double d = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    d = (a[i] - x) - (i > 0 ? off / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++count;
  }
  return count;
}

// i-th smallest eigenvalue (0-based) of the tridiagonal by bisection
double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, int i) {
  double lo = a[0], hi = a[0];
  for (size_t j = 0; j < a.size(); ++j) {
    const double r = (j > 0 ? std::fabs(b[j - 1]) : 0.0) + (j + 1 < a.size() ? std::fabs(b[j]) : 0.0);
    lo = std::min(lo, a[j] - r);
    hi = std::max(hi, a[j] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(a, b, mid) > i)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

// y = A x for a dense symmetric A read by rows (A(m, k) = A[k + m ld]): one
// wave per row, lanes over k, a fixed-order wave reduction
__global__ __launch_bounds__(kThreads) void k_gemv_rows(const double* __restrict__ A, int64_t ld,
                                                        int64_t n, const double* __restrict__ x,
                                                        double* __restrict__ y) {
  const int64_t m = int64_t(blockIdx.x) * (kThreads / 64) + (threadIdx.x >> 6);
  if (m >= n) return;
  const int lane = threadIdx.x & 63;
  const double* row = A + m * ld;
  double s = 0.0;
  for (int64_t k = lane; k < n; k += 64) s += row[k] * x[k];
  s = wave_sum(s);
  if (lane == 0) y[m] = s;
}

// The same product with 16-byte loads (A, x and ld allow them, n % 128 == 0):
// lane l takes the pairs at k = 2 l + 128 i; four partial sums over i mod 4,
// added in a fixed order, then the wave reduction
__global__ __launch_bounds__(kThreads) void k_gemv_rows_vec(const double* __restrict__ A,
                                                            int64_t ld, int64_t n,
                                                            const double* __restrict__ x,
                                                            double* __restrict__ y) {
  const int64_t m = int64_t(blockIdx.x) * (kThreads / 64) + (threadIdx.x >> 6);
  if (m >= n) return;
  const int lane = threadIdx.x & 63;
  const double2* row = reinterpret_cast<const double2*>(A + m * ld) + lane;
  const double2* xv = reinterpret_cast<const double2*>(x) + lane;
  const int64_t steps = n / 128;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t i = 0;
  for (; i + 4 <= steps; i += 4) {
    double2 a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = row[(i + u) * 64];
      b[u] = xv[(i + u) * 64];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = fma(a[u].y, b[u].y, fma(a[u].x, b[u].x, acc[u]));
  }
  for (; i < steps; ++i) {
    const double2 a = row[i * 64], b = xv[i * 64];
    acc[i & 3] = fma(a.y, b.y, fma(a.x, b.x, acc[i & 3]));
  }
  double s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  s = wave_sum(s);
  if (lane == 0) y[m] = s;
}

// The same product with x staged in LDS: 16 waves (rows) per workgroup share
// one copy of x per 4096-element chunk, so the x reads come from LDS instead
// of competing with the A stream for the caches; four partial sums per lane
// over the pairs k = 2 l + 128 i (i mod 4), added in a fixed order
constexpr int kLdsWaves = 16;
constexpr int kXChunk = 4096;
__global__ __launch_bounds__(64 * kLdsWaves) void k_gemv_rows_lds(const double* __restrict__ A,
                                                                  int64_t ld, int64_t n,
                                                                  const double* __restrict__ x,
                                                                  double* __restrict__ y) {
  __shared__ double2 xs[kXChunk / 2];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t m = int64_t(blockIdx.x) * kLdsWaves + wave;
  const double2* row = reinterpret_cast<const double2*>(A + (m < n ? m : 0) * ld) + lane;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t i = 0;   // global pair-step index (k = 2 lane + 128 i)
  for (int64_t c0 = 0; c0 < n; c0 += kXChunk) {
    const int cn = int(n - c0 < kXChunk ? n - c0 : kXChunk);   // a multiple of 128
    __syncthreads();
    for (int t = threadIdx.x; t < cn / 2; t += 64 * kLdsWaves)
      xs[t] = reinterpret_cast<const double2*>(x + c0)[t];
    __syncthreads();
    if (m < n) {
      const int steps = cn / 128;
      int s = 0;
      for (; s + 4 <= steps; s += 4) {
        double2 a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = row[(i + s + u) * 64];
          b[u] = xs[lane + (s + u) * 64];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = int((i + s + u) & 3);
          acc[q] = fma(a[u].y, b[u].y, fma(a[u].x, b[u].x, acc[q]));
        }
      }
      for (; s < steps; ++s) {
        const double2 a = row[(i + s) * 64], b = xs[lane + s * 64];
        const int q = int((i + s) & 3);
        acc[q] = fma(a.y, b.y, fma(a.x, b.x, acc[q]));
      }
    }
    i += cn / 128;
  }
  double sres = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  sres = wave_sum(sres);
  if (m < n && lane == 0) y[m] = sres;
}

}  // namespace

// 16-byte-load GEMV where the layout allows it (knob CHFSI_GEMV_VEC=0: off)
static bool gemv_vec_on() {
  static const bool on = [] {
    const char* e = std::getenv("CHFSI_GEMV_VEC");
    return !(e && std::atoi(e) == 0);
  }();
  return on;
}

hipError_t gemv_rows_f64(const double* A, int64_t ld, int64_t n, const double* x, double* y,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + kThreads / 64 - 1) / (kThreads / 64);
  const bool vec = gemv_vec_on() && n % 128 == 0 && ld % 2 == 0 &&
                   reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(x) % 16 == 0;
  const char* ev = std::getenv("CHFSI_GEMV_LDS");
  const bool lds = vec && !(ev && std::atoi(ev) == 0);
  if (lds)
    k_gemv_rows_lds<<<dim3(unsigned((n + kLdsWaves - 1) / kLdsWaves)), 64 * kLdsWaves, 0, st>>>(
        A, ld, n, x, y);
  else if (vec)
    k_gemv_rows_vec<<<dim3(unsigned(blocks)), kThreads, 0, st>>>(A, ld, n, x, y);
  else
    k_gemv_rows<<<dim3(unsigned(blocks)), kThreads, 0, st>>>(A, ld, n, x, y);
  return hipGetLastError();
}

size_t lanczos_workspace_bytes(int64_t L) {
  return size_t(10) * size_t(L) * sizeof(double) + size_t(2 * kMaxBlocks + 8) * sizeof(double);
}

hipError_t lanczos_bounds(const LanczosOps& ops, int64_t L, double* work, double* host_scalars,
                          hipStream_t st, LanczosResult* res) {
  double* v_prev = work;
  double* v = v_prev + L;
  double* Bv_prev = v + L;
  double* Bv = Bv_prev + L;
  double* w = Bv + L;
  double* u = w + L;
  double* r = u + L;
  double* z = r + L;
  double* p = z + L;
  double* q = p + L;
  double* partial = q + L;
  double* dres = partial + 2 * kMaxBlocks;
  const int nb = blocks_for(L);
  const int lb = int(std::min<int64_t>((L + kThreads - 1) / kThreads, 65536));
  hipError_t e;
#define LZ_CK(x)                          \
  do {                                    \
    if ((e = (x)) != hipSuccess) return e; \
  } while (0)
  // device scalars: dres[0] r.r, dres[1..2] r.z (alternating), dres[3] p.B p,
  // dres[4] alpha_j, dres[5] ||u||_B^2
  // two dot products on the device, read back (synchronises the stream)
  auto dot2 = [&](const double* a0, const double* b0, const double* a1, const double* b1,
                  double* o0, double* o1) -> hipError_t {
    k_dot2_partial<<<nb, kThreads, 0, st>>>(a0, b0, a1, b1, L, partial);
    k_dot2_final<<<1, 64, 0, st>>>(partial, nb, dres, dres + 1);
    hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) return e2;
    e2 = hipMemcpyAsync(host_scalars, dres, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e2 != hipSuccess) return e2;
    e2 = hipStreamSynchronize(st);
    if (e2 != hipSuccess) return e2;
    *o0 = host_scalars[0];
    if (o1) *o1 = host_scalars[1];
    return hipSuccess;
  };
  // solve B x = y by preconditioned CG from x = 0 (relative tolerance cg_tol).
  // alpha and the direction update take their scalars on the device, and the
  // iterations run in batches: as many as the previous solve needed, then one
  // read-back (r.r, r0.r0 and the sticky not-positive-definite flag); the
  // first solve, and iterations past a batch, read back after each.  Extra
  // iterations of a batch that overshoots only refine x.
  int cg_batch = 1;
  auto bsolve = [&](const double* y, double* x) -> hipError_t {
    LZ_CK(fill_zero(x, size_t(L) * sizeof(double), st));
    LZ_CK(hipMemcpyAsync(r, y, size_t(L) * sizeof(double), hipMemcpyDeviceToDevice, st));
    k_precond<<<lb, kThreads, 0, st>>>(ops.dinv, r, L, z);
    LZ_CK(hipGetLastError());
    LZ_CK(hipMemcpyAsync(p, z, size_t(L) * sizeof(double), hipMemcpyDeviceToDevice, st));
    // dres[7] = r0 . r0, dres[1] = r0 . z0, dres[6] = 0 (flag)
    k_dot2_partial<<<nb, kThreads, 0, st>>>(r, r, r, z, L, partial);
    k_dot2_final<<<1, 64, 0, st>>>(partial, nb, dres + 7, dres + 1);
    LZ_CK(hipGetLastError());
    LZ_CK(fill_zero(dres + 6, sizeof(double), st));
    double* rz_cur = dres + 1;
    double* rz_nxt = dres + 2;
    int it = 0;
    int batch = cg_batch;
    while (it < ops.cg_max_iter) {
      const int m = std::min(batch, ops.cg_max_iter - it);
      for (int j = 0; j < m; ++j) {
        if (it + j > 0) {
          k_cg_dir<<<lb, kThreads, 0, st>>>(rz_nxt, rz_cur, z, L, p);
          std::swap(rz_cur, rz_nxt);
        }
        LZ_CK(ops.apply_B(p, q));
        k_dot2_partial<<<nb, kThreads, 0, st>>>(p, q, nullptr, nullptr, L, partial);
        k_dot2_final<<<1, 64, 0, st>>>(partial, nb, dres + 3, nullptr);
        k_cg_update<<<nb, kThreads, 0, st>>>(rz_cur, dres + 3, p, q, x, r, z, ops.dinv, L,
                                             partial, dres + 6);
        k_dot2_final<<<1, 64, 0, st>>>(partial, nb, dres, rz_nxt);
        LZ_CK(hipGetLastError());
      }
      it += m;
      res->cg_iterations += m;
      LZ_CK(hipMemcpyAsync(host_scalars, dres, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
      LZ_CK(hipStreamSynchronize(st));
      if (host_scalars[6] != 0.0) return hipErrorInvalidValue;   // B not positive definite
      const double rr0 = host_scalars[7];
      if (!(rr0 > 0.0)) break;                                     // zero right-hand side
      if (host_scalars[0] <= ops.cg_tol * ops.cg_tol * rr0) break;
      batch = 1;
    }
    cg_batch = std::max(1, it);
    return hipSuccess;
  };
  // v_1 = v_0 / ||v_0||_B
  LZ_CK(hipMemcpyAsync(v, ops.v0, size_t(L) * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (ops.apply_B)
    LZ_CK(ops.apply_B(v, Bv));
  else
    LZ_CK(hipMemcpyAsync(Bv, v, size_t(L) * sizeof(double), hipMemcpyDeviceToDevice, st));
  double nrm2 = 0.0;
  LZ_CK(dot2(v, Bv, nullptr, nullptr, &nrm2, nullptr));
  if (!(nrm2 > 0.0)) return hipErrorInvalidValue;
  {
    const double s = 1.0 / std::sqrt(nrm2);
    k_lincomb3<<<lb, kThreads, 0, st>>>(s, v, 0.0, nullptr, 0.0, nullptr, L, v);
    k_lincomb3<<<lb, kThreads, 0, st>>>(s, Bv, 0.0, nullptr, 0.0, nullptr, L, Bv);
    LZ_CK(hipGetLastError());
  }
  std::vector<double> alpha, beta;
  double beta_prev = 0.0;
  res->cg_iterations = 0;
  for (int j = 0; j < ops.steps; ++j) {
    LZ_CK(ops.apply_A(v, w));                         // w = A v_j
    if (ops.apply_B)
      LZ_CK(bsolve(w, u));                            // u = B^{-1} A v_j
    else
      LZ_CK(hipMemcpyAsync(u, w, size_t(L) * sizeof(double), hipMemcpyDeviceToDevice, st));
    // alpha_j = v_j . w stays on the device until ||u||_B is read back with it
    k_dot2_partial<<<nb, kThreads, 0, st>>>(v, w, nullptr, nullptr, L, partial);
    k_dot2_final<<<1, 64, 0, st>>>(partial, nb, dres + 4, nullptr);
    // u -= a v_j + beta_{j-1} v_{j-1};  B u = w - a B v_j - beta_{j-1} B v_{j-1} (into w)
    k_lincomb3_dev<<<lb, kThreads, 0, st>>>(1.0, u, dres + 4, v, -beta_prev,
                                            j > 0 ? v_prev : nullptr, L, u);
    k_lincomb3_dev<<<lb, kThreads, 0, st>>>(1.0, w, dres + 4, Bv, -beta_prev,
                                            j > 0 ? Bv_prev : nullptr, L, w);
    k_dot2_partial<<<nb, kThreads, 0, st>>>(u, w, nullptr, nullptr, L, partial);
    k_dot2_final<<<1, 64, 0, st>>>(partial, nb, dres + 5, nullptr);
    LZ_CK(hipGetLastError());
    LZ_CK(hipMemcpyAsync(host_scalars, dres + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    LZ_CK(hipStreamSynchronize(st));
    const double a = host_scalars[0], bb = host_scalars[1];
    alpha.push_back(a);
    const double bj = std::sqrt(std::max(bb, 0.0));
    beta.push_back(bj);
    if (j + 1 == ops.steps || !(bj > 1e-14 * std::fabs(a) + 1e-300)) break;
    // shift: v_{j-1} <- v_j, v_j <- u / beta_j (and the B-products)
    std::swap(v_prev, v);
    std::swap(Bv_prev, Bv);
    k_lincomb3<<<lb, kThreads, 0, st>>>(1.0 / bj, u, 0.0, nullptr, 0.0, nullptr, L, v);
    k_lincomb3<<<lb, kThreads, 0, st>>>(1.0 / bj, w, 0.0, nullptr, 0.0, nullptr, L, Bv);
    LZ_CK(hipGetLastError());
    beta_prev = bj;
  }
#undef LZ_CK
  const int k = int(alpha.size());
  std::vector<double> off(beta.begin(), beta.begin() + (k - 1));
  res->steps = k;
  res->theta_min = tridiag_eig(alpha, off, 0);
  res->theta_max = tridiag_eig(alpha, off, k - 1);
  res->beta_last = std::fabs(beta[k - 1]);
  res->lower = res->theta_min - res->beta_last;
  res->upper = res->theta_max + res->beta_last;
  return hipSuccess;
}

}  // namespace chfsi
