// Small dense FP64 linear algebra of the Rayleigh-Ritz step (b x b, b up to a
// few thousand): blocked Cholesky, blocked triangular solve and a
// block-parallel Jacobi symmetric eigensolver.
//
// Rayleigh-Ritz (Algorithm 1, step 2) solves the projected pencil
// (Y^T A Y) E = (Y^T B Y) E Lambda.  The library reduces it with the Cholesky
// factor of the column-scaled Gram matrix Y^T B Y (CholQR) and diagonalises the
// resulting standard symmetric matrix with Jacobi rotations.
//
// Jacobi is chosen for the GPU because (i) a round of disjoint rotations is
// embarrassingly parallel, (ii) it converges quadratically when the matrix is
// nearly diagonal -- which is what the projected matrix becomes as subspace
// iteration converges -- and (iii) it is accurate to a small multiple of the
// unit roundoff.  The block variant pairs JB-wide column blocks (JB = 16) in a
// round-robin tournament, applies one inner sweep of rotations to every
// JP x JP pair subproblem (JP = 2 JB = 32) in LDS (one workgroup each, waves
// specialised so that a round costs one barrier: the next round's rotations,
// this round's update, the accumulation of U), and applies the resulting
// orthogonal JP x JP factors to the rest of the matrix and to the eigenvector
// accumulator with MFMA, in one launch per outer round.  Sweeps repeat until no
// rotation is applied or a cap of 40 sweeps is reached (then reported).
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <utility>
#include <vector>

namespace chfsi {

namespace {

constexpr int NB = 64;          // Cholesky / TRSM block
constexpr int JB = 16;          // Jacobi column block
constexpr int JP = 2 * JB;      // Jacobi pair subproblem size
constexpr int LDJ = JP + 1;     // padded LDS leading dimension

// ---------------------------------------------------------------------------
// Cholesky of the diagonal block (jb <= 64) in LDS; right-looking, one barrier
// per column: step k subtracts a_ik a_jk / d_k (d_k = a_kk at step k) from the
// trailing lower triangle, the columns are scaled by 1/sqrt(d_k) at the end.
// Threads form a 16 x 16 grid over the trailing triangle (no index division).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_potrf_diag(double* A, int64_t lda, int jb, int* info,
                                                    int j0, double piv_tol) {
  __shared__ double a[NB * (NB + 1)];
  constexpr int L = NB + 1;
  if (*info != 0) return;
  for (int idx = threadIdx.x; idx < jb * jb; idx += 256) {
    const int i = idx % jb, j = idx / jb;
    a[i + j * L] = A[i + j * lda];
  }
  __syncthreads();
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  for (int k = 0; k < jb; ++k) {
    const double d = a[k + k * L];
    if (!(d > piv_tol) || !isfinite(d)) {  // the same decision in every thread
      if (threadIdx.x == 0) atomicCAS(info, 0, j0 + k + 1);
      return;
    }
    const double inv = 1.0 / d;
    for (int j = k + 1 + ty; j < jb; j += 16) {
      const double ljk = a[j + k * L] * inv;
      for (int i = j + tx; i < jb; i += 16) a[i + j * L] -= a[i + k * L] * ljk;
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < jb * jb; idx += 256) {
    const int i = idx % jb, j = idx / jb;
    const double dj = sqrt(a[j + j * L]);
    A[i + j * lda] = i > j ? a[i + j * L] / dj : (i == j ? dj : 0.0);
  }
}

// Cholesky of the diagonal block (jb <= NB) and the inverse of its factor in
// one wave: lane i holds row i in registers (the block padded to NB x NB with
// the identity).  Step k: the pivot d = a_kk is read from lane k, g = 1/sqrt(d)
// comes from the hardware estimate and two Newton steps, lane i forms
// l_ik = a_ik g (l_kk = d g) and puts it in LDS (two alternating buffers), and
// every lane subtracts l_ik l_jk from its row (the l_jk are LDS broadcasts).
// Then lane c forms column c of L^{-1} by forward substitution with the
// pivots' g, reading the rows of L from LDS in 16-byte pairs; the sum of each
// step runs in four partial sums (j mod 4), which shortens the chain of
// dependent FP64 operations fourfold.  Writes L (upper part of the block
// zeroed) and L^{-1} (NB x NB, ld NB, identity-padded) to Li.  The steps are
// expanded from templates, so every register index is a constant.  Measured
// at b = 320 (five blocks per factorisation): see the kernel table.
constexpr int LDR = NB + 2;     // row stride of L in LDS (16-byte aligned rows)

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane(unsigned(u), lane);
  const unsigned hi = __builtin_amdgcn_readlane(unsigned(u >> 32), lane);
  return __longlong_as_double((static_cast<unsigned long long>(hi) << 32) | lo);
}

// 1/sqrt(x) for normal x > 0: the hardware estimate and two Newton steps
__device__ __forceinline__ double rsqrt_newton(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-(x * y), y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-(x * y), y, 1.0);
  return fma(0.5 * y, e, y);
}

template <int K>
__device__ __forceinline__ bool chol_step(double (&r)[NB], double (*col)[NB], double* invd,
                                          double piv_tol) {
  const int i = threadIdx.x;
  const double d = readlane_f64(r[K], K);
  if (!(d > piv_tol) || !isfinite(d)) return false;   // the same decision in every lane
  const double g = rsqrt_newton(d);
  const double l = i == K ? d * g : r[K] * g;
  r[K] = l;
  col[K & 1][i] = l;
  if (i == 0) invd[K] = g;
  __syncthreads();
#pragma unroll
  for (int j = K + 1; j < NB; ++j) r[j] = fma(-l, col[K & 1][j], r[j]);
  return true;
}

template <int K>
__device__ __forceinline__ void trtri_step(double (&x)[NB], const double* lt, const double* invd) {
  double s[4] = {(int(threadIdx.x) == K) ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < K; ++j) s[j & 3] = fma(-lt[K * LDR + j], x[j], s[j & 3]);
  x[K] = ((s[0] + s[1]) + (s[2] + s[3])) * invd[K];
}

template <int... Ks>
__device__ __forceinline__ int chol_all(std::integer_sequence<int, Ks...>, double (&r)[NB],
                                        double (*col)[NB], double* invd, double piv_tol) {
  int failed = -1;
  // left to right; a failed pivot stops the remaining steps
  ((failed < 0 && !chol_step<Ks>(r, col, invd, piv_tol) ? (failed = Ks) : 0), ...);
  return failed;
}

template <int... Ks>
__device__ __forceinline__ void trtri_all(std::integer_sequence<int, Ks...>, double (&x)[NB],
                                          const double* lt, const double* invd) {
  (trtri_step<Ks>(x, lt, invd), ...);
}

__global__ __launch_bounds__(64) void k_potrf_trtri_diag(double* A, int64_t lda, int jb,
                                                         int* info, int j0, double* Li,
                                                         double piv_tol) {
  __shared__ __attribute__((aligned(16))) double col[2][NB];
  __shared__ __attribute__((aligned(16))) double lt[NB * LDR];
  __shared__ double invd[NB];
  if (*info != 0) return;
  const int i = threadIdx.x;
  double r[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j)
    r[j] = (i < jb && j < jb) ? A[i + j * lda] : (i == j ? 1.0 : 0.0);
  const int failed = chol_all(std::make_integer_sequence<int, NB>{}, r, col, invd, piv_tol);
  if (failed >= 0) {
    if (i == 0) atomicCAS(info, 0, j0 + failed + 1);
    return;
  }
  // L (lower, zero above): row i to LDS (row-major) and to the block
#pragma unroll
  for (int j = 0; j < NB; ++j) lt[i * LDR + j] = j <= i ? r[j] : 0.0;
  if (i < jb) {
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (j < jb) A[i + j * lda] = j <= i ? r[j] : 0.0;
  }
  __syncthreads();
  // column i of L^{-1}: x_k = (delta_ki - sum_{j<k} l_kj x_j) / l_kk
  double x[NB];
  trtri_all(std::make_integer_sequence<int, NB>{}, x, lt, invd);
#pragma unroll
  for (int k = 0; k < NB; ++k) Li[k + i * NB] = x[k];
}

// Inverse of one lower-triangular diagonal block (jb <= NB) of L: one wave,
// lane c forms column c of L^{-1} by forward substitution in registers
// (entries above the diagonal are zero).  Block blockIdx.x starts at row and
// column j0 + blockIdx.x * NB.
__global__ __launch_bounds__(64) void k_trtri_diag(const double* L, int64_t ldl, int64_t b,
                                                   int64_t j0, double* Li, const int* info) {
  __shared__ double l[NB * (NB + 1)];
  constexpr int LD = NB + 1;
  if (info && *info != 0) return;
  const int64_t o = j0 + int64_t(blockIdx.x) * NB;
  const int jb = int(b - o < NB ? b - o : NB);
  for (int idx = threadIdx.x; idx < NB * NB; idx += 64) {
    const int i = idx % NB, j = idx / NB;
    l[i + j * LD] = (i < jb && j < jb) ? L[(o + i) + (o + j) * ldl] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  const int c = threadIdx.x;
  double x[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    double s = (k == c) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < k; ++j) s -= l[k + j * LD] * x[j];
    x[k] = s / l[k + k * LD];
  }
  double* out = Li + int64_t(blockIdx.x) * NB * NB;
#pragma unroll
  for (int k = 0; k < NB; ++k) out[k + c * NB] = x[k];
}

__global__ __launch_bounds__(256) void k_zero_upper(double* A, int64_t lda, int64_t b) {
  const int64_t total = b * b;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t i = idx % b, j = idx / b;
    if (i < j) A[i + j * lda] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Jacobi
// ---------------------------------------------------------------------------
// round-robin ("circle") schedule: n players (even), round r in [0, n-1),
// slot 0 fixed, slots 1..n-1 rotate; pair k joins slots k and n-1-k.
__device__ __forceinline__ int rr_slot(int slot, int r, int n) {
  return slot == 0 ? 0 : 1 + (slot - 1 + r) % (n - 1);
}

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// Block indices of pair k in round r of the block tournament (nblk blocks).
__device__ __forceinline__ void block_pair(int k, int r, int nblk, int* I, int* J) {
  int a = rr_slot(k, r, nblk), b = rr_slot(nblk - 1 - k, r, nblk);
  *I = a < b ? a : b;
  *J = a < b ? b : a;
}

// index of local row l (0..JP-1) of pair (I,J) in the padded matrix
__device__ __forceinline__ int pair_index(int l, int I, int J) {
  return l < JB ? I * JB + l : J * JB + (l - JB);
}

// ---------------------------------------------------------------------------
// Pair subproblem, wave-specialised (one sweep of JP - 1 rounds, one barrier
// per round).
// Round r of the circle schedule pairs slots (k, JP-1-k), k < JP/2; between
// rounds every index moves from slot s to slot sigma(s) = s - 1 (1 -> JP-1,
// slot 0 fixed).  The subproblem is therefore stored by slot, not by index:
// round r reads LDS buffer r % 2 and writes the shifted entries into buffer
// (r + 1) % 2, so every thread touches the same addresses in every round and
// no index arithmetic remains inside the loop.  Only the lower triangle (in
// slot order) is kept.  The rotation of pair k acts on (first, second) =
// (slot k, slot JP-1-k): J = [[c, s], [-s, c]], a <- J^T a J.
//  * wave 0, lane k < JP/2: the rotation of pair k in the NEXT round.  The
//    three entries it needs after this round are formed from this round's
//    buffer and rotations with the same arithmetic (rot_block, same operand
//    order) as the update waves, so they are bit-identical to what those
//    waves store.
//  * waves 2..4 (k1 >= k2 of 16 x 16 pair blocks, 136 threads): this round's
//    two-sided update of one 2 x 2 block each.
//  * wave 1, lane i < JP: row i of the accumulated rotation U in registers,
//    by index (the round loop is unrolled, so the indices of each round's
//    pairs are constants).
// ---------------------------------------------------------------------------
constexpr int kHalf = JP / 2;       // rotations per round
constexpr int kRounds = JP - 1;     // rounds per sweep
constexpr int kPairThreads = 5 * 64;

// lower-triangle LDS offset of symmetric entry (i, j) (slot coordinates)
__device__ __forceinline__ int sym_idx(int i, int j) { return i >= j ? i + j * LDJ : j + i * LDJ; }
// slot of an index after one round, and before it
__device__ __forceinline__ int slot_next(int s) { return s == 0 ? 0 : (s == 1 ? JP - 1 : s - 1); }
__device__ __forceinline__ int slot_prev(int s) { return s == 0 ? 0 : (s == JP - 1 ? 1 : s + 1); }
// pair of slot s, and whether s is the pair's first slot
__device__ __forceinline__ int slot_pair(int s) { return s < kHalf ? s : JP - 1 - s; }

// out = J1^T X J2 for the 2 x 2 block X (rows first/second of pair 1,
// columns first/second of pair 2); explicit fma so that every caller rounds
// alike
__device__ __forceinline__ void rot_block(double x11, double x12, double x21, double x22,
                                          double c1, double s1, double c2, double s2,
                                          double* o11, double* o12, double* o21, double* o22) {
  const double y11 = fma(c1, x11, -(s1 * x21)), y12 = fma(c1, x12, -(s1 * x22));
  const double y21 = fma(s1, x11, c1 * x21), y22 = fma(s1, x12, c1 * x22);
  *o11 = fma(c2, y11, -(s2 * y12));
  *o12 = fma(s2, y11, c2 * y12);
  *o21 = fma(c2, y21, -(s2 * y22));
  *o22 = fma(s2, y21, c2 * y22);
}

// 1/sqrt(x) for normal x > 0: the hardware estimate and two Newton steps
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-(x * y), y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-(x * y), y, 1.0);
  return fma(0.5 * y, e, y);
}

// rotation (c, s) with J^T [[app, apq], [apq, aqq]] J diagonal (apq != 0):
// t = tan(phi) = sign(d) e / (|d| + sqrt(d^2 + e^2)), d = aqq - app, e = 2 apq,
// c = 1 / sqrt(1 + t^2), s = t c -- written with g = |d| + sqrt(d^2 + e^2) as
// c = g / sqrt(g^2 + e^2), s = sign(d) e / sqrt(g^2 + e^2), two square roots
// and no division.  Outside the range where d^2 + e^2 is a normal number the
// textbook form with divisions is used.
__device__ __forceinline__ void jacobi_cs(double app, double aqq, double apq, double* c,
                                          double* s) {
  const double d = aqq - app, e = 2.0 * apq;
  const double h2 = fma(d, d, e * e);
  if (h2 > 1e-300 && h2 < 1e300) {
    const double h = h2 * rsqrt_nr(h2);
    const double g = fabs(d) + h;
    const double r = rsqrt_nr(fma(g, g, e * e));
    *c = g * r;
    *s = (d < 0.0 ? -e : e) * r;
    return;
  }
  const double theta = d / e;
  const double t = fabs(theta) > 1e150
                       ? 0.5 / theta
                       : copysign(1.0, theta) / (fabs(theta) + sqrt(theta * theta + 1.0));
  *c = 1.0 / sqrt(t * t + 1.0);
  *s = t * (*c);
}

// LDS of one pair subproblem: the slot-ordered lower triangle (ping-pong
// buffers), the rotations of the current and next round, the wave maxima
struct PairSmem {
  double buf[2][JP * LDJ];
  double2 cs[2][kHalf];
  double wmax[kPairThreads / 64];
  int nrot_total;
};

// One inner sweep of the pair subproblem held in S.buf[0] (lower triangle,
// local order = slot order of round 0); `mx` is this thread's largest
// off-diagonal magnitude among the entries it stored.  Skips (skip_out = 1)
// when the subproblem is already diagonal to the threshold, else writes the
// accumulated JP x JP rotation to Uo (skip_out = 0) and adds its rotation
// count to the sweep counter.
__device__ __forceinline__ void pair_solve_core(PairSmem& S, double mx, const double* scale,
                                                double tol, double* Uo, int* skip_out,
                                                int* counter) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  auto& buf = S.buf;
  auto& cs = S.cs;
  auto& wmax = S.wmax;
  int& nrot_total = S.nrot_total;
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if (lane == 0) wmax[wave] = mx;
  if (tid == 0) nrot_total = 0;
  __syncthreads();
  mx = wmax[0];
#pragma unroll
  for (int w = 1; w < kPairThreads / 64; ++w) mx = fmax(mx, wmax[w]);
  const double thresh = tol * (*scale);
  if (!(mx > thresh)) {
    if (tid == 0) *skip_out = 1;
    return;
  }
  if (wave == 0 && lane < kHalf) {
    const int f = lane, s = JP - 1 - lane;
    const double apq = buf[0][sym_idx(s, f)];
    double c = 1.0, sn = 0.0;
    if (fabs(apq) > thresh) jacobi_cs(buf[0][sym_idx(f, f)], buf[0][sym_idx(s, s)], apq, &c, &sn);
    cs[0][lane] = make_double2(c, sn);
  }
  __syncthreads();
  if (wave == 0) {
    // next-round pair `lane` = this round's slots x (first) and y (second)
    const int k = lane < kHalf ? lane : 0;
    const int x = slot_prev(k), y = slot_prev(JP - 1 - k);
    const int kx = slot_pair(x), ky = slot_pair(y);
    // diagonal blocks of kx and ky: first/second slots and which output
    const int fx = kx, sx = JP - 1 - kx, fy = ky, sy = JP - 1 - ky;
    const int ax_ff = sym_idx(fx, fx), ax_sf = sym_idx(sx, fx), ax_ss = sym_idx(sx, sx);
    const int ay_ff = sym_idx(fy, fy), ay_sf = sym_idx(sy, fy), ay_ss = sym_idx(sy, sy);
    const bool x_first = x == fx, y_first = y == fy;
    // off-diagonal (y, x): block (K1, K2) = rows of the pair with the larger index
    const bool xrow = kx > ky;
    const int K1 = xrow ? kx : ky, K2 = xrow ? ky : kx;
    const int f1 = K1, s1 = JP - 1 - K1, f2 = K2, s2 = JP - 1 - K2;
    const int b11 = sym_idx(f1, f2), b12 = sym_idx(f1, s2), b21 = sym_idx(s1, f2),
              b22 = sym_idx(s1, s2);
    const int rowv = xrow ? x : y, colv = xrow ? y : x;
    const int osel = (rowv == f1 ? 0 : 2) + (colv == f2 ? 0 : 1);
    int count = 0;
    for (int r = 0; r < kRounds; ++r) {
      const double* a = buf[r & 1];
      const double2* t = cs[r & 1];
      if (lane < kHalf) {
        const unsigned long long m = __ballot(t[lane].y != 0.0);
        if (r + 1 < kRounds) {
          const double2 tx = t[kx], ty = t[ky], t1 = t[K1], t2 = t[K2];
          double o11, o12, o21, o22;
          const double xsf = a[ax_sf];
          rot_block(a[ax_ff], xsf, xsf, a[ax_ss], tx.x, tx.y, tx.x, tx.y, &o11, &o12, &o21, &o22);
          const double app = x_first ? o11 : o22;
          const double ysf = a[ay_sf];
          rot_block(a[ay_ff], ysf, ysf, a[ay_ss], ty.x, ty.y, ty.x, ty.y, &o11, &o12, &o21, &o22);
          const double aqq = y_first ? o11 : o22;
          rot_block(a[b11], a[b12], a[b21], a[b22], t1.x, t1.y, t2.x, t2.y, &o11, &o12, &o21,
                    &o22);
          const double apq = osel == 0 ? o11 : (osel == 1 ? o12 : (osel == 2 ? o21 : o22));
          double c = 1.0, sn = 0.0;
          if (fabs(apq) > thresh) jacobi_cs(app, aqq, apq, &c, &sn);
          cs[(r + 1) & 1][lane] = make_double2(c, sn);
        }
        count += __popcll(m);
      }
      __syncthreads();
    }
    if (lane == 0) nrot_total = count;
  } else if (wave >= 2) {
    // block (k1, k2), k1 >= k2, of the 16 x 16 pair blocks (136 of 192 threads)
    const int idx = tid - 128;
    int k1 = 0, k2 = 0;
    {
      int rem = idx;
      while (k1 < kHalf && rem > k1) {
        rem -= k1 + 1;
        ++k1;
      }
      k2 = rem;
    }
    const bool active = idx < kHalf * (kHalf + 1) / 2;
    const int f1 = k1, s1 = JP - 1 - k1, f2 = k2, s2 = JP - 1 - k2;
    const int i11 = sym_idx(f1, f2), i12 = sym_idx(f1, s2), i21 = sym_idx(s1, f2),
              i22 = sym_idx(s1, s2);
    const int o11i = sym_idx(slot_next(f1), slot_next(f2)),
              o12i = sym_idx(slot_next(f1), slot_next(s2)),
              o21i = sym_idx(slot_next(s1), slot_next(f2)),
              o22i = sym_idx(slot_next(s1), slot_next(s2));
    for (int r = 0; r < kRounds; ++r) {
      if (active) {
        const double* a = buf[r & 1];
        double* o = buf[(r + 1) & 1];
        const double2 t1 = cs[r & 1][k1], t2 = cs[r & 1][k2];
        double v11, v12, v21, v22;
        if (k1 == k2) {
          const double x21 = a[i21];
          rot_block(a[i11], x21, x21, a[i22], t1.x, t1.y, t1.x, t1.y, &v11, &v12, &v21, &v22);
          o[o11i] = v11;
          o[o22i] = v22;
          o[o21i] = t1.y != 0.0 ? 0.0 : x21;
        } else {
          rot_block(a[i11], a[i12], a[i21], a[i22], t1.x, t1.y, t2.x, t2.y, &v11, &v12, &v21,
                    &v22);
          o[o11i] = v11;
          o[o12i] = v12;
          o[o21i] = v21;
          o[o22i] = v22;
        }
      }
      __syncthreads();
    }
  } else {
    double ur[JP];
#pragma unroll
    for (int j = 0; j < JP; ++j) ur[j] = (j == lane) ? 1.0 : 0.0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      if (lane < JP) {
#pragma unroll
        for (int k = 0; k < kHalf; ++k) {
          // indices in slots k and JP-1-k at round r
          const int p = (k == 0) ? 0 : 1 + (k - 1 + r) % (JP - 1);
          const int q = 1 + (JP - 2 - k + r) % (JP - 1);
          const double2 t = cs[r & 1][k];
          const double up = ur[p], uq = ur[q];
          ur[p] = fma(t.x, up, -(t.y * uq));
          ur[q] = fma(t.y, up, t.x * uq);
        }
      }
      __syncthreads();
    }
    // row `lane` of U into LDS (the subproblem itself is no longer needed)
    if (lane < JP) {
#pragma unroll
      for (int j = 0; j < JP; ++j) buf[0][lane + j * LDJ] = ur[j];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < JP * JP; idx += kPairThreads) {
    const int i = idx % JP, j = idx / JP;
    Uo[i + j * JP] = buf[0][i + j * LDJ];
  }
  if (tid == 0) {
    *skip_out = 0;
    if (nrot_total > 0) atomicAdd(counter, nrot_total);
  }
}

// One workgroup per pair of the outer round: gather the JP x JP subproblem,
// skip it when already diagonal (to the threshold), else one Jacobi sweep.
// Writes U (JP x JP) and skip[pair] (1 = U is the identity).
__global__ __launch_bounds__(kPairThreads) void k_jacobi_pair_solve(
    const double* A, int64_t lda, int nblk, int round, const double* scale, double tol, double* U,
    int* skip, int* counter) {
  __shared__ PairSmem S;
  const int tid = threadIdx.x;
  int I, J;
  block_pair(blockIdx.x, round, nblk, &I, &J);
  // round 0 has index s in slot s
  double mx = 0.0;
  for (int idx = tid; idx < JP * JP; idx += kPairThreads) {
    const int i = idx % JP, j = idx / JP;
    if (i < j) continue;
    const double v = A[pair_index(i, I, J) + int64_t(pair_index(j, I, J)) * lda];
    S.buf[0][i + j * LDJ] = v;
    if (i != j) mx = fmax(mx, fabs(v));
  }
  pair_solve_core(S, mx, scale, tol, U + int64_t(blockIdx.x) * JP * JP, skip + blockIdx.x,
                  counter);
}


// out = op(X) * Y for JP x JP matrices in LDS (ld LDJ) on FP64 MFMA
// (v_mfma_f64_16x16x4f64: lane l supplies X(l%16, l/16) and Y(l/16, l%16);
// output element r of lane l is row l/16 + 4r, column l%16).  Each of the
// four waves computes one JP/2 x JP/2 quadrant as NT x NT tiles of 16 x 16.
// TX: X is read transposed.
constexpr int NT = JP / 32;
template <bool TX>
__device__ __forceinline__ void lds_mm(const double* X, const double* Y, double out[NT][NT][4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int qm = (wave & 1) * (JP / 2), qn = (wave >> 1) * (JP / 2);
  const int l16 = lane & 15, g = lane >> 4;
  f64x4_t acc[NT][NT];
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f64x4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < JP; k0 += 4) {
    const int k = k0 + g;
    double xa[NT], yb[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int m = qm + i * 16 + l16;
      xa[i] = TX ? X[k + m * LDJ] : X[m + k * LDJ];
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) yb[j] = Y[k + (qn + j * 16 + l16) * LDJ];
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[i], yb[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) out[i][j][r] = acc[i][j][r];
}

// row / column (local) of output element r of tile (i, j) held by this lane
__device__ __forceinline__ int mm_row(int i, int r) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave & 1) * (JP / 2) + i * 16 + (lane >> 4) + 4 * r;
}
__device__ __forceinline__ int mm_col(int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave >> 1) * (JP / 2) + j * 16 + (lane & 15);
}

__device__ __forceinline__ void lds_mm_store(double* Z, const double v[NT][NT][4]) {
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) Z[mm_row(i, r) + mm_col(j) * LDJ] = v[i][j][r];
}

__device__ __forceinline__ void load_u_or_identity(double* dst, const double* U, bool identity) {
  for (int idx = threadIdx.x; idx < JP * JP; idx += 256) {
    const int i = idx % JP, j = idx / JP;
    dst[i + j * LDJ] = identity ? (i == j ? 1.0 : 0.0) : U[i + j * JP];
  }
}

// The outer round's rotations, one launch: blockIdx.y < npairs updates the
// matrix block pair (P, Q) = (blockIdx.x, blockIdx.y), P >= Q:
// A[SP, SQ] <- U_P^T A[SP, SQ] U_Q, written with its transpose into A[SQ, SP];
// blockIdx.y >= npairs updates JP rows (chunk blockIdx.y - npairs) of the
// eigenvector accumulator: V[rows, SP] <- V[rows, SP] U_P.
__global__ __launch_bounds__(256) void k_jacobi_apply(double* A, int64_t lda, double* V,
                                                      int64_t ldv, int nblk, int npairs,
                                                      int round, const double* U,
                                                      const int* skip) {
  __shared__ double m[JP * LDJ];
  __shared__ double up[JP * LDJ];
  __shared__ double uq[JP * LDJ];
  const int P = blockIdx.x;
  int IP, JPb;
  block_pair(P, round, nblk, &IP, &JPb);
  double t[NT][NT][4];
  if (int(blockIdx.y) >= npairs) {
    if (skip[P]) return;
    const int64_t r0 = int64_t(blockIdx.y - npairs) * JP;
    for (int idx = threadIdx.x; idx < JP * JP; idx += 256) {
      const int i = idx % JP, j = idx / JP;
      m[i + j * LDJ] = V[r0 + i + int64_t(pair_index(j, IP, JPb)) * ldv];
    }
    load_u_or_identity(up, U + int64_t(P) * JP * JP, false);
    __syncthreads();
    lds_mm<false>(m, up, t);
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          V[r0 + mm_row(i, r) + int64_t(pair_index(mm_col(j), IP, JPb)) * ldv] = t[i][j][r];
    return;
  }
  const int Q = blockIdx.y;
  if (P < Q) return;
  const bool sp = skip[P] != 0, sq = skip[Q] != 0;
  if (sp && sq) return;
  int IQ, JQ;
  block_pair(Q, round, nblk, &IQ, &JQ);
  for (int idx = threadIdx.x; idx < JP * JP; idx += 256) {
    const int i = idx % JP, j = idx / JP;
    m[i + j * LDJ] = A[pair_index(i, IP, JPb) + int64_t(pair_index(j, IQ, JQ)) * lda];
  }
  load_u_or_identity(up, U + int64_t(P) * JP * JP, sp);
  load_u_or_identity(uq, U + int64_t(Q) * JP * JP, sq);
  __syncthreads();
  lds_mm<true>(up, m, t);         // U_P^T M
  __syncthreads();
  lds_mm_store(m, t);
  __syncthreads();
  lds_mm<false>(m, uq, t);        // (U_P^T M) U_Q
  __syncthreads();
  lds_mm_store(m, t);
  __syncthreads();
  for (int idx = threadIdx.x; idx < JP * JP; idx += 256) {
    const int i = idx % JP, j = idx / JP;
    A[pair_index(i, IP, JPb) + int64_t(pair_index(j, IQ, JQ)) * lda] = m[i + j * LDJ];
  }
  if (P != Q) {
    for (int idx = threadIdx.x; idx < JP * JP; idx += 256) {
      const int i = idx % JP, j = idx / JP;
      A[pair_index(i, IQ, JQ) + int64_t(pair_index(j, IP, JPb)) * lda] = m[j + i * LDJ];
    }
  }
}

// ---------------------------------------------------------------------------
// Pipelined outer rounds: one launch carries the pair solves of round r and
// the rotations of round r - 1.  The pair workgroups do not wait for the
// rotated matrix: each forms the three 16 x 16 blocks of it that its
// subproblem needs from the matrix before round r - 1 and that round's
// factors, with the same products in the same order as the rotation
// workgroups (so the entries are bit-identical to the ones those store),
// while the rotation workgroups write the rotated matrix into the other
// buffer.  A sweep of R rounds takes R + 1 launches instead of 2 R, and the
// rotations leave the critical path.
// ---------------------------------------------------------------------------

// pair of round r that holds block x, and x's offset (0 or JB) in it
__device__ __forceinline__ void block_locate(int x, int r, int nblk, int* pair, int* off) {
  const int n1 = nblk - 1;
  const int s = x == 0 ? 0 : 1 + ((x - 1 - r) % n1 + n1) % n1;
  const int k = s < nblk / 2 ? s : nblk - 1 - s;
  int I, J;
  block_pair(k, r, nblk, &I, &J);
  *pair = k;
  *off = x == I ? 0 : JB;
}

constexpr int LDZ = JB + 1;   // leading dimension of a 16-row slice in LDS

// rows oR..oR+15 of U_R^T M (both 16-column halves), M = A[S_R, S_C] (pair R
// rows (IR, JR), pair C columns (IC, JC)); operands from global memory with the
// values and the k order of lds_mm<true>(U_R, M).  idR: U_R is the identity.
__device__ __forceinline__ void rot_rows(const double* A, int64_t lda, const double* UR, bool idR,
                                         int oR, int IR, int JR, int IC, int JC, f64x4_t* acc0,
                                         f64x4_t* acc1) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, g = lane >> 4;
  const int m = oR + l16;
  const int64_t col0 = int64_t(pair_index(l16, IC, JC)) * lda;
  const int64_t col1 = int64_t(pair_index(JB + l16, IC, JC)) * lda;
  double xa[JP / 4], y0[JP / 4], y1[JP / 4];
#pragma unroll
  for (int t = 0; t < JP / 4; ++t) {
    const int k = 4 * t + g;
    const int64_t row = pair_index(k, IR, JR);
    xa[t] = idR ? (k == m ? 1.0 : 0.0) : UR[k + m * JP];
    y0[t] = A[row + col0];
    y1[t] = A[row + col1];
  }
  f64x4_t a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < JP / 4; ++t) {
    a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[t], y0[t], a0, 0, 0, 0);
    a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[t], y1[t], a1, 0, 0, 0);
  }
  *acc0 = a0;
  *acc1 = a1;
}

// U_C[:, oC..oC+15] in the lane order of the B operand of rot_cols
__device__ __forceinline__ void load_ucols(const double* UC, bool idC, int oC, double (&yb)[JP / 4]) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, g = lane >> 4;
  const int n = oC + l16;
#pragma unroll
  for (int t = 0; t < JP / 4; ++t) {
    const int k = 4 * t + g;
    yb[t] = idC ? (k == n ? 1.0 : 0.0) : UC[k + n * JP];
  }
}

// the 16 x 16 tile Z U_C[:, oC..oC+15] for a 16-row slice Z (LDS, ld LDZ),
// with the values and the k order of lds_mm<false>(Z, U_C)
__device__ __forceinline__ f64x4_t rot_cols(const double* Z, const double (&yb)[JP / 4]) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, g = lane >> 4;
  f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < JP / 4; ++t) {
    const int k = 4 * t + g;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Z[l16 + k * LDZ], yb[t], acc, 0, 0, 0);
  }
  return acc;
}

union RoundSmem {
  struct {
    PairSmem ps;
    double z[3][JP * LDZ];
  } pair;
  struct {
    double m[JP * LDJ];
    double up[JP * LDJ];
    double uq[JP * LDJ];
  } apply;
};

// Workgroups [0, npairs) (when rcur >= 0): pair solves of round rcur on the
// matrix after round rprev (rprev < 0: Pin itself).  The rest (when
// rprev >= 0): round rprev's rotations as in k_jacobi_apply, Pin -> Pout (a
// block both of whose factors are identities is copied), V in place.
__global__ __launch_bounds__(kPairThreads) void k_jacobi_round(
    const double* __restrict__ Pin, double* __restrict__ Pout, int64_t lda, double* V,
    int64_t ldv, int nblk, int npairs, int rprev, const double* Uprev, const int* skipprev,
    int rcur, double* Ucur, int* skipcur, const double* scale, double tol, int* counter) {
  __shared__ RoundSmem sm;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int npw = rcur >= 0 ? npairs : 0;
  if (int(blockIdx.x) < npw) {
    PairSmem& S = sm.pair.ps;
    int I, J;
    block_pair(blockIdx.x, rcur, nblk, &I, &J);
    double mx = 0.0;
    if (rprev < 0) {
      for (int idx = tid; idx < JP * JP; idx += kPairThreads) {
        const int i = idx % JP, j = idx / JP;
        if (i < j) continue;
        const double v = Pin[pair_index(i, I, J) + int64_t(pair_index(j, I, J)) * lda];
        S.buf[0][i + j * LDJ] = v;
        if (i != j) mx = fmax(mx, fabs(v));
      }
    } else {
      int pI, oI, pJ, oJ;
      block_locate(I, rprev, nblk, &pI, &oI);
      block_locate(J, rprev, nblk, &pJ, &oJ);
      // tile 0: (I, I); tile 1: (J, J); tile 2: the (J, I) block, formed as
      // the rotation workgroup of the pair with the larger index forms it
      const bool jrow = pJ > pI;
      auto tile = [&](int t, int* R, int* oR, int* C, int* oC) {
        if (t == 0) { *R = pI; *oR = oI; *C = pI; *oC = oI; }
        else if (t == 1) { *R = pJ; *oR = oJ; *C = pJ; *oC = oJ; }
        else if (jrow) { *R = pJ; *oR = oJ; *C = pI; *oC = oI; }
        else { *R = pI; *oR = oI; *C = pJ; *oC = oJ; }
      };
      // waves 0..2: tile `wave`; the right factor of the second product is
      // loaded with the first product's operands
      const int l16 = lane & 15, g = lane >> 4;
      const int t = wave;
      int R = 0, oR = 0, C = 0, oC = 0;
      double ucol[JP / 4];
      if (wave < 3) {
        tile(t, &R, &oR, &C, &oC);
        int IR, JR, IC, JC;
        block_pair(R, rprev, nblk, &IR, &JR);
        block_pair(C, rprev, nblk, &IC, &JC);
        load_ucols(Uprev + int64_t(C) * JP * JP, skipprev[C] != 0, oC, ucol);
        f64x4_t a0, a1;
        rot_rows(Pin, lda, Uprev + int64_t(R) * JP * JP, skipprev[R] != 0, oR, IR, JR, IC, JC,
                 &a0, &a1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          sm.pair.z[t][(g + 4 * r) + l16 * LDZ] = a0[r];
          sm.pair.z[t][(g + 4 * r) + (JB + l16) * LDZ] = a1[r];
        }
      }
      __syncthreads();
      if (wave < 3) {
        const f64x4_t acc = rot_cols(sm.pair.z[t], ucol);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = g + 4 * r, bcol = l16;   // element (a, bcol) of the tile
          int i, j;                              // local (slot) coordinates
          if (t == 0) { i = a; j = bcol; }
          else if (t == 1) { i = JB + a; j = JB + bcol; }
          else if (jrow) { i = JB + a; j = bcol; }
          else { i = JB + bcol; j = a; }
          if (i < j) continue;
          S.buf[0][i + j * LDJ] = acc[r];
          if (i != j) mx = fmax(mx, fabs(acc[r]));
        }
      }
    }
    pair_solve_core(S, mx, scale, tol, Ucur + int64_t(blockIdx.x) * JP * JP,
                    skipcur + blockIdx.x, counter);
    return;
  }
  if (rprev < 0) return;
  // rotations of round rprev
  const int a = int(blockIdx.x) - npw;
  const int P = a % npairs, y = a / npairs;
  int IP, JPb;
  block_pair(P, rprev, nblk, &IP, &JPb);
  double* m = sm.apply.m;
  double* up = sm.apply.up;
  double* uq = sm.apply.uq;
  double t[NT][NT][4];
  if (y >= npairs) {
    if (skipprev[P]) return;
    const int64_t r0 = int64_t(y - npairs) * JP;
    for (int idx = tid; idx < JP * JP; idx += kPairThreads) {
      const int i = idx % JP, j = idx / JP;
      m[i + j * LDJ] = V[r0 + i + int64_t(pair_index(j, IP, JPb)) * ldv];
      up[i + j * LDJ] = Uprev[int64_t(P) * JP * JP + i + j * JP];
    }
    __syncthreads();
    if (wave < 4) {
      lds_mm<false>(m, up, t);
#pragma unroll
      for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            V[r0 + mm_row(i, r) + int64_t(pair_index(mm_col(j), IP, JPb)) * ldv] = t[i][j][r];
    }
    return;
  }
  const int Q = y;
  if (P < Q) return;
  const bool sp = skipprev[P] != 0, sq = skipprev[Q] != 0;
  int IQ, JQ;
  block_pair(Q, rprev, nblk, &IQ, &JQ);
  if (sp && sq) {
    for (int idx = tid; idx < JP * JP; idx += kPairThreads) {
      const int i = idx % JP, j = idx / JP;
      const int64_t o1 = pair_index(i, IP, JPb) + int64_t(pair_index(j, IQ, JQ)) * lda;
      Pout[o1] = Pin[o1];
      if (P != Q) {
        const int64_t o2 = pair_index(i, IQ, JQ) + int64_t(pair_index(j, IP, JPb)) * lda;
        Pout[o2] = Pin[o2];
      }
    }
    return;
  }
  for (int idx = tid; idx < JP * JP; idx += kPairThreads) {
    const int i = idx % JP, j = idx / JP;
    m[i + j * LDJ] = Pin[pair_index(i, IP, JPb) + int64_t(pair_index(j, IQ, JQ)) * lda];
    up[i + j * LDJ] = sp ? (i == j ? 1.0 : 0.0) : Uprev[int64_t(P) * JP * JP + i + j * JP];
    uq[i + j * LDJ] = sq ? (i == j ? 1.0 : 0.0) : Uprev[int64_t(Q) * JP * JP + i + j * JP];
  }
  __syncthreads();
  if (wave < 4) lds_mm<true>(up, m, t);         // U_P^T M
  __syncthreads();
  if (wave < 4) lds_mm_store(m, t);
  __syncthreads();
  if (wave < 4) lds_mm<false>(m, uq, t);        // (U_P^T M) U_Q
  __syncthreads();
  if (wave < 4) lds_mm_store(m, t);
  __syncthreads();
  for (int idx = tid; idx < JP * JP; idx += kPairThreads) {
    const int i = idx % JP, j = idx / JP;
    Pout[pair_index(i, IP, JPb) + int64_t(pair_index(j, IQ, JQ)) * lda] = m[i + j * LDJ];
    if (P != Q)
      Pout[pair_index(j, IQ, JQ) + int64_t(pair_index(i, IP, JPb)) * lda] = m[i + j * LDJ];
  }
}

// padded copy: P (bp x bp) = [A 0; 0 0]; V = I
__global__ __launch_bounds__(256) void k_jacobi_setup(const double* A, int64_t lda, int64_t b,
                                                      double* P, double* V, int64_t bp) {
  const int64_t total = bp * bp;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t i = idx % bp, j = idx / bp;
    P[idx] = (i < b && j < b) ? A[i + j * lda] : 0.0;
    V[idx] = (i == j) ? 1.0 : 0.0;
  }
}

// Frobenius norm of a b x b matrix: per-workgroup partial sums of squares
// (k_fro_part, one column range each), then one workgroup adds the partials
// in a fixed order (deterministic)
constexpr int kFroParts = 64;
__global__ __launch_bounds__(256) void k_fro_part(const double* A, int64_t lda, int64_t b,
                                                  double* part) {
  __shared__ double red[256];
  double s = 0.0;
  const int64_t c0 = b * blockIdx.x / kFroParts, c1 = b * (blockIdx.x + 1) / kFroParts;
  for (int64_t idx = threadIdx.x; idx < (c1 - c0) * b; idx += 256) {
    const double v = A[idx % b + (c0 + idx / b) * lda];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(64) void k_fro_final(const double* part, double* out) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < kFroParts; ++i) s += part[i];
    *out = sqrt(s) > 0 ? sqrt(s) : 1.0;
  }
}

// largest off-diagonal magnitude of the bp x bp matrix: per-workgroup column
// ranges (k_offmax_part), then out[0] = 1 if it is at most thresh_rel * scal[0]
// (the Frobenius norm), else 0
__global__ __launch_bounds__(256) void k_offmax_part(const double* P, int64_t bp, double* part) {
  __shared__ double red[256];
  double m = 0.0;
  const int64_t c0 = bp * blockIdx.x / kFroParts, c1 = bp * (blockIdx.x + 1) / kFroParts;
  for (int64_t idx = threadIdx.x; idx < (c1 - c0) * bp; idx += 256) {
    const int64_t i = idx % bp, j = c0 + idx / bp;
    if (i != j) m = fmax(m, fabs(P[i + j * bp]));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(64) void k_offmax_final(const double* part, const double* scal,
                                                     double thresh_rel, int* done) {
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int i = 0; i < kFroParts; ++i) m = fmax(m, part[i]);
    *done = (m <= thresh_rel * scal[0]) ? 1 : 0;
  }
}

// ascending sort of the diagonal (first b entries) by rank counting, then
// gather eigenvector columns; the diagonal is staged through LDS in chunks
__global__ __launch_bounds__(256) void k_jacobi_rank(const double* P, int64_t bp, int64_t b,
                                                     double* w, int* perm) {
  constexpr int kChunk = 1024;
  __shared__ double dg[kChunk];
  const int64_t i = blockIdx.x * int64_t(256) + threadIdx.x;
  const double di = i < b ? P[i + i * bp] : 0.0;
  int64_t rank = 0;
  for (int64_t c0 = 0; c0 < b; c0 += kChunk) {
    const int cn = int(b - c0 < kChunk ? b - c0 : kChunk);
    __syncthreads();
    for (int t = threadIdx.x; t < cn; t += 256) dg[t] = P[(c0 + t) + (c0 + t) * bp];
    __syncthreads();
    if (i < b) {
      // eight independent counts, so that the LDS reads are not serialised
      int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      int t = 0;
      for (; t + 8 <= cn; t += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double dj = dg[t + u];
          cnt[u] += (dj < di) || (dj == di && c0 + t + u < i);
        }
      }
      for (; t < cn; ++t) {
        const double dj = dg[t];
        cnt[0] += (dj < di) || (dj == di && c0 + t < i);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) rank += cnt[u];
    }
  }
  if (i < b) {
    w[rank] = di;
    perm[rank] = int(i);
  }
}

__global__ __launch_bounds__(256) void k_jacobi_gather(const double* V, int64_t bp, int64_t b,
                                                       const int* perm, double* out,
                                                       int64_t ldo) {
  const int64_t total = b * b;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t i = idx % b, r = idx / b;
    out[i + r * ldo] = V[i + int64_t(perm[r]) * bp];
  }
}

inline int64_t grid_for(int64_t total) {
  int64_t g = (total + 255) / 256;
  return std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

}  // namespace

size_t potrf_workspace_bytes(int64_t b) { return gemm_workspace_bytes(b, b, NB, sizeof(double)); }

size_t tri_workspace_bytes(int64_t b, int64_t nrhs) {
  const int64_t nblk = (b + NB - 1) / NB;
  return size_t(nblk * NB * NB + NB * std::max(b, nrhs)) * sizeof(double);
}

// Blocked right-looking Cholesky.  Per diagonal block: factor it in LDS,
// invert it (kept in tri for trsm_lower_left), form the panel below as a GEMM
// with the inverse, then update the trailing matrix with a GEMM.
// one-wave Cholesky-and-inverse of the diagonal blocks (knob CHFSI_POTRF_FUSED=0:
// the 256-thread Cholesky and a separate inverse)
static bool potrf_fused() {
  const char* e = std::getenv("CHFSI_POTRF_FUSED");
  return !(e && std::atoi(e) == 0);
}

hipError_t potrf_lower(double* A, int64_t lda, int64_t b, int* info, hipStream_t st,
                       const Workspace& ws, double* tri, double piv_tol) {
  hipError_t e = hipSuccess;
  const int64_t nblk = (b + NB - 1) / NB;
  double* tmp = tri + nblk * NB * NB;
  for (int64_t j0 = 0; j0 < b; j0 += NB) {
    const int jb = int(std::min<int64_t>(NB, b - j0));
    double* Li = tri + (j0 / NB) * NB * NB;
    if (potrf_fused()) {
      k_potrf_trtri_diag<<<1, 64, 0, st>>>(A + j0 + j0 * lda, lda, jb, info, int(j0), Li,
                                           piv_tol);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
      k_potrf_diag<<<1, 256, 0, st>>>(A + j0 + j0 * lda, lda, jb, info, int(j0), piv_tol);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      k_trtri_diag<<<1, 64, 0, st>>>(A, lda, b, j0, Li, info);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int64_t rows = b - j0 - jb;
    if (rows <= 0) break;
    {   // tmp (rows x jb) = A21 L11^{-T}; A21 <- tmp
      GemmDesc<double> g;
      g.M = rows;
      g.N = jb;
      g.K = jb;
      g.A = A + (j0 + jb) + j0 * lda;
      g.sam = 1;
      g.sak = lda;
      g.B = Li;           // B(k, n) = L11^{-1}(n, k)
      g.sbn = 1;
      g.sbk = NB;
      g.C = tmp;
      g.ldc = rows;
      if ((e = gemm<double>(g, st, ws, 1)) != hipSuccess) return e;
      if ((e = copy_block(tmp, rows, A + (j0 + jb) + j0 * lda, lda, rows, jb, st)) != hipSuccess)
        return e;
    }
    // A22 -= L21 L21^T
    GemmDesc<double> g;
    g.M = rows;
    g.N = rows;
    g.K = jb;
    g.A = A + (j0 + jb) + j0 * lda;
    g.sam = 1;
    g.sak = lda;
    g.B = A + (j0 + jb) + j0 * lda;
    g.sbn = 1;
    g.sbk = lda;
    g.C = A + (j0 + jb) + (j0 + jb) * lda;
    g.ldc = lda;
    g.epi.alpha = -1.0;
    g.epi.beta = 1.0;
    g.epi.C1 = g.C;
    g.epi.ldc1 = lda;
    if ((e = gemm<double>(g, st, ws, 1)) != hipSuccess) return e;
  }
  k_zero_upper<<<grid_for(b * b), 256, 0, st>>>(A, lda, b);
  return hipGetLastError();
}

// X <- L^{-1} X by block forward substitution with the diagonal blocks'
// inverses (computed here unless inverses_ready, i.e. left in tri by
// potrf_lower for the same L).
hipError_t trsm_lower_left(const double* L, int64_t ldl, double* X, int64_t ldx, int64_t b,
                           int64_t nrhs, hipStream_t st, const Workspace& ws, double* tri,
                           bool inverses_ready) {
  hipError_t e = hipSuccess;
  const int64_t nblk = (b + NB - 1) / NB;
  double* tmp = tri + nblk * NB * NB;
  if (!inverses_ready) {
    k_trtri_diag<<<dim3(unsigned(nblk)), 64, 0, st>>>(L, ldl, b, 0, tri, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int64_t j0 = 0; j0 < b; j0 += NB) {
    const int jb = int(std::min<int64_t>(NB, b - j0));
    {   // tmp (jb x nrhs) = L_jj^{-1} X_j; X_j <- tmp
      GemmDesc<double> g;
      g.M = jb;
      g.N = nrhs;
      g.K = jb;
      g.A = tri + (j0 / NB) * NB * NB;
      g.sam = 1;
      g.sak = NB;
      g.B = X + j0;
      g.sbk = 1;
      g.sbn = ldx;
      g.C = tmp;
      g.ldc = jb;
      if ((e = gemm<double>(g, st, ws, 1)) != hipSuccess) return e;
      if ((e = copy_block(tmp, jb, X + j0, ldx, jb, nrhs, st)) != hipSuccess) return e;
    }
    const int64_t rows = b - j0 - jb;
    if (rows <= 0) break;
    GemmDesc<double> g;
    g.M = rows;
    g.N = nrhs;
    g.K = jb;
    g.A = L + (j0 + jb) + j0 * ldl;
    g.sam = 1;
    g.sak = ldl;
    g.B = X + j0;
    g.sbk = 1;
    g.sbn = ldx;
    g.C = X + j0 + jb;
    g.ldc = ldx;
    g.epi.alpha = -1.0;
    g.epi.beta = 1.0;
    g.epi.C1 = g.C;
    g.epi.ldc1 = ldx;
    if ((e = gemm<double>(g, st, ws, 1)) != hipSuccess) return e;
  }
  return hipSuccess;
}

static int64_t jacobi_padded(int64_t b) { return std::max<int64_t>(JP, (b + JP - 1) / JP * JP); }

size_t syev_workspace_bytes(int64_t b) {
  const int64_t bp = jacobi_padded(b);
  const int64_t npairs = bp / JP;
  return size_t(3 * bp * bp + 2 * npairs * JP * JP + 16 + kFroParts) * sizeof(double) +
         size_t(b + 64 + 2 * npairs) * sizeof(int);
}

// pipelined outer rounds (knob CHFSI_JACOBI_PIPE=0: a pair-solve launch and a
// rotation launch per round; read at every call, so that tests can compare both)
static bool jacobi_pipelined() {
  const char* e = std::getenv("CHFSI_JACOBI_PIPE");
  return !(e && std::atoi(e) == 0);
}

hipError_t syev_jacobi(double* A, int64_t lda, int64_t b, double* w, double* V, int64_t ldv,
                       hipStream_t st, const Workspace& ws, int* sweeps_out,
                       int* unconverged_out, int* pinned_flags, hipEvent_t ev) {
  const int64_t bp = jacobi_padded(b);
  const int nblk = int(bp / JB);     // even
  const int npairs = nblk / 2;
  if (ws.bytes < syev_workspace_bytes(b)) return hipErrorInvalidValue;
  double* P = static_cast<double*>(ws.ptr);
  double* Vp = P + bp * bp;
  double* P2 = Vp + bp * bp;                      // the pipelined rounds' second buffer
  double* U = P2 + bp * bp;                       // two sets of npairs JP x JP factors
  double* scal = U + 2 * int64_t(npairs) * JP * JP;   // [0]: Frobenius norm
  int* counter = reinterpret_cast<int*>(scal + 16 + kFroParts);
  int* perm = counter + 64;
  int* skip = perm + b;                           // two sets of npairs flags
  hipError_t e;
  k_jacobi_setup<<<grid_for(bp * bp), 256, 0, st>>>(A, lda, b, P, Vp, bp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_fro_part<<<kFroParts, 256, 0, st>>>(A, lda, b, scal + 16);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_fro_final<<<1, 64, 0, st>>>(scal + 16, scal);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const double tol = 1e-15;
  // sweep cap (knob CHFSI_JACOBI_MAX_SWEEPS, for tests of the cap's report)
  int max_outer = 40;
  if (const char* e = std::getenv("CHFSI_JACOBI_MAX_SWEEPS")) max_outer = std::max(1, std::atoi(e));
  int sweeps = 0;
  int host_count = 0;
  bool converged = false;
  const bool pipe = jacobi_pipelined();
  const int R = nblk - 1;                          // rounds per sweep
  const unsigned napply = unsigned(npairs) * unsigned(npairs + bp / JP);
  const int64_t usz = int64_t(npairs) * JP * JP;
  // launch r of the pipelined sweep: pair solves of round r (on the matrix
  // after round r - 1, formed in the pair workgroups) and round r - 1's
  // rotations P -> P2; launch R applies round R - 1
  auto launch = [&](int r) -> hipError_t {
    const bool solve = r < R, rotate = r > 0;
    const int cu = r & 1, pu = (r - 1) & 1;
    k_jacobi_round<<<dim3((solve ? unsigned(npairs) : 0u) + (rotate ? napply : 0u)), kPairThreads,
                     0, st>>>(
        P, P2, bp, Vp, bp, nblk, npairs, rotate ? r - 1 : -1, rotate ? U + pu * usz : nullptr,
        rotate ? skip + pu * npairs : nullptr, solve ? r : -1, solve ? U + cu * usz : nullptr,
        solve ? skip + cu * npairs : nullptr, scal, tol, counter);
    const hipError_t le = hipGetLastError();
    if (le == hipSuccess && rotate) std::swap(P, P2);
    return le;
  };
  // With a pinned flag buffer and an event, the first two launches of the
  // next sweep are queued before the convergence flags of this one are read
  // back, so the device does not idle while the host waits.  After
  // convergence those launches change nothing: every pair subproblem is below
  // the threshold (skipped), the rotation workgroups copy the matrix into the
  // other buffer, and only that buffer swap is undone.
  const bool early = pipe && pinned_flags && ev && R >= 2;
  int started = 0;   // launches of the current sweep already queued
  for (; sweeps < max_outer; ++sweeps) {
    if (started == 0 && (e = fill_zero(counter, sizeof(int), st)) != hipSuccess) return e;
    if (pipe) {
      for (int r = started; r <= R; ++r)
        if ((e = launch(r)) != hipSuccess) return e;
      started = 0;
    } else {
      for (int r = 0; r < R; ++r) {
        k_jacobi_pair_solve<<<dim3(npairs), kPairThreads, 0, st>>>(P, bp, nblk, r, scal, tol, U,
                                                                   skip, counter);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_jacobi_apply<<<dim3(npairs, unsigned(npairs + bp / JP)), 256, 0, st>>>(
            P, bp, Vp, bp, nblk, npairs, r, U, skip);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
    }
    // converged when the sweep rotated nothing, or when no off-diagonal entry
    // is left above the threshold (every pair of a further sweep would skip)
    k_offmax_part<<<kFroParts, 256, 0, st>>>(P, bp, scal + 16);
    k_offmax_final<<<1, 64, 0, st>>>(scal + 16, scal, tol, counter + 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (early) {
      if ((e = hipMemcpyAsync(pinned_flags, counter, 2 * sizeof(int), hipMemcpyDeviceToHost,
                              st)) != hipSuccess)
        return e;
      if ((e = hipEventRecord(ev, st)) != hipSuccess) return e;
      if (sweeps + 1 < max_outer) {
        if ((e = fill_zero(counter, sizeof(int), st)) != hipSuccess) return e;
        for (int r = 0; r < 2; ++r)
          if ((e = launch(r)) != hipSuccess) return e;
        started = 2;
      }
      if ((e = hipEventSynchronize(ev)) != hipSuccess) return e;
      host_count = pinned_flags[0];
      if (host_count == 0 || pinned_flags[1] != 0) {
        if (started == 2) std::swap(P, P2);   // launch 1 copied the matrix into P2
        started = 0;
        converged = true;
        ++sweeps;
        break;
      }
      continue;
    }
    int host_flags[2] = {0, 0};
    if ((e = hipMemcpyAsync(host_flags, counter, 2 * sizeof(int), hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    host_count = host_flags[0];
    if (host_count == 0 || host_flags[1] != 0) {
      converged = true;
      ++sweeps;
      break;
    }
  }
  k_jacobi_rank<<<dim3(unsigned((b + 255) / 256)), 256, 0, st>>>(P, bp, b, w, perm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_jacobi_gather<<<grid_for(b * b), 256, 0, st>>>(Vp, bp, b, perm, V, ldv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (sweeps_out) *sweeps_out = sweeps;
  // the tolerance was not met within the cap
  if (unconverged_out) *unconverged_out = converged ? 0 : 1;
  return hipSuccess;
}

}  // namespace chfsi
