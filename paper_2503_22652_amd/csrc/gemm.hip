// MFMA GEMM for gfx950 with a fused three-term epilogue.
//
// This kernel evaluates the matrix multi-vector products of the Chebyshev
// filter -- the dominant cost of the method (paper, Section 3, opening
// paragraph) -- together with the rest of the recurrence step: for the
// residual filter (Algorithm 3, loop body)
//     R_X <- a_k A (D^{-1} R_Y) + b_k R_Y + c_k R_X + a_k Y Lambda_Y
// is one launch (kscale = D^{-1}, C1 = R_Y, C2 = R_X, C3 = Y, colscale3 =
// Lambda_Y).  The same kernel provides the FP64 products of the Rayleigh-Ritz
// step (operator application, Gram matrices, rotations).
//
// Design (CDNA4):
//  * 256 threads = four 64-wide waves arranged WM x WN; each wave owns a
//    (BM/WM) x (BN/WN) sub-tile made of 16x16 MFMA tiles
//    (v_mfma_f32_16x16x4f32 or v_mfma_f64_16x16x4f64).
//  * Operands are staged through LDS in a k-contiguous layout [row][k] with a
//    small pad.  Within one BK slice the four 16-lane groups of a wave take
//    disjoint k ranges (group g owns k = g*BK/4 ... g*BK/4 + BK/4 - 1), so
//    every lane fetches its operand fragments with 16-byte LDS reads; the sum
//    over the slice is unchanged because A and B use the same k assignment.
//  * Two LDS stages with register prefetch: one barrier per k slice.
//  * Deterministic split-K: partial tiles go to scratch and a second kernel
//    adds them in split order and applies the epilogue, so results never depend
//    on scheduling.
//  * Tile order is remapped so that consecutive logical tiles (same rows of A,
//    neighbouring column tiles) land on the same XCD and share its L2.
#include "internal.h"

#include <algorithm>
#include <cstdlib>

namespace chfsi {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

// Operand layout of both 16x16x4 instructions: lane l supplies A(l%16, l/16)
// and B(l/16, l%16).  Output element r of lane l sits in column l%16; its row
// differs: the f32 form keeps four consecutive rows per lane group
// (row 4*(l/16) + r), the f64 form interleaves them (row l/16 + 4*r).
template <>
struct Mfma<float> {
  using acc_t = f32x4;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int lgrp, int r) { return lgrp * 4 + r; }
};

template <>
struct Mfma<double> {
  using acc_t = f64x4;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int lgrp, int r) { return lgrp + 4 * r; }
};

// 16-byte native vector of T
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  static constexpr int W = 4;
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec16<double> {
  static constexpr int W = 2;
  typedef double type __attribute__((ext_vector_type(2)));
};

struct KernelArgsCommon {
  int64_t M, N, K;
  int64_t sam, sak, sbk, sbn, ldc;
  int batch, splits;
  int64_t kchunk;           // k range per split (multiple of BK)
  int64_t bsA, bsB, bsC, bsC1;
  int vecA, vecB;           // 16-byte vector loads allowed along the contiguous dim
  int tiles_m, tiles_n;
  int lower;                // skip tiles strictly above the diagonal
};

template <typename T>
struct KernelArgs {
  KernelArgsCommon c;
  const T* A;
  const T* B;
  const T* kscale;
  T* C;
  T* partial;
  Epilogue<T> epi;
  // optional second output of the vectorised split-K reduction: out16 (M x N,
  // ld M) = bfloat16(scale16 .* C), the next BF16 product's right operand
  unsigned short* out16 = nullptr;
  const T* scale16 = nullptr;
};

// float -> bfloat16, round to nearest even (NaN stays a quiet NaN)
__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ int xcd_remap(int h, int G) {
  // Dispatch is round-robin over 8 XCDs: WG h runs on XCD h % 8.  Give each
  // XCD a contiguous range of logical tile ids.
  const int xcd = h & 7, slot = h >> 3;
  const int full = G >> 3, rem = G & 7;
  return (xcd < rem) ? xcd * (full + 1) + slot : rem * (full + 1) + (xcd - rem) * full + slot;
}

template <typename T>
__device__ __forceinline__ T apply_epilogue(const Epilogue<T>& e, T acc, int64_t m, int64_t n) {
  T v = e.alpha * acc;
  if (e.rowscale) v *= e.rowscale[m];
  if (e.C1) v += e.beta * e.C1[m + n * e.ldc1];
  if (e.C2) v += e.gamma * e.C2[m + n * e.ldc2];
  if (e.C3) {
    T f = e.delta;
    if (e.colscale3) f *= e.colscale3[n];
    v += f * e.C3[m + n * e.ldc3];
  }
  return v;
}

// Load a ROWS x BK tile of a "row operand" (row r, depth k) into registers.
// KCONTIG: element (r,k) at base[r*sr + k]; else at base[r + k*sr].
// KS: multiply every element by kscale[k] on the way in.
template <typename T, int ROWS, int BK, bool KCONTIG, bool KS>
struct TileLoader {
  static constexpr int W = Vec16<T>::W;
  static constexpr int TOT = ROWS * BK / W;       // vectors per tile
  static constexpr int NV = (TOT + 255) / 256;     // vectors per thread
  static_assert((ROWS * BK) % W == 0, "tile not divisible into vectors");
  static_assert(KCONTIG ? (BK % W == 0) : (ROWS % W == 0), "vector along the contiguous dim");
  using vec_t = typename Vec16<T>::type;
  vec_t r[NV];

  // Unchecked 16-byte loads: the whole tile lies inside the operand.
  __device__ __forceinline__ void load_fast(const T* __restrict__ base, int64_t sr, int64_t r0,
                                            int64_t k0, const T* __restrict__ kscale) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int v = threadIdx.x + i * 256;
      if (TOT % 256 != 0 && v >= TOT) break;
      if constexpr (KCONTIG) {
        const int row = v / (BK / W);
        const int kk = (v % (BK / W)) * W;
        r[i] = *reinterpret_cast<const vec_t*>(base + (r0 + row) * sr + k0 + kk);
      } else {
        const int kk = v / (ROWS / W);
        const int row = (v % (ROWS / W)) * W;
        r[i] = *reinterpret_cast<const vec_t*>(base + r0 + row + (k0 + kk) * sr);
      }
    }
  }

  // Element-wise loads with bounds checks (edge tiles, ragged k, unaligned).
  __device__ __forceinline__ void load_checked(const T* __restrict__ base, int64_t sr, int64_t r0,
                                            int64_t rmax, int64_t k0, int64_t kmax,
                                            const T* __restrict__ kscale) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int v = threadIdx.x + i * 256;
      if (TOT % 256 != 0 && v >= TOT) break;
      if constexpr (KCONTIG) {
        const int row = v / (BK / W);
        const int kk = (v % (BK / W)) * W;
        const int64_t gr = r0 + row, gk = k0 + kk;
        for (int j = 0; j < W; ++j) {
          const bool ok = gr < rmax && gk + j < kmax;
          r[i][j] = ok ? base[gr * sr + gk + j] : T(0);
        }
      } else {
        const int kk = v / (ROWS / W);
        const int row = (v % (ROWS / W)) * W;
        const int64_t gr = r0 + row, gk = k0 + kk;
        for (int j = 0; j < W; ++j) {
          const bool ok = gk < kmax && gr + j < rmax;
          r[i][j] = ok ? base[gr + j + gk * sr] : T(0);
        }
      }
    }
  }

  template <int LDK>
  __device__ __forceinline__ void store(T* __restrict__ lds) const {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int v = threadIdx.x + i * 256;
      if (TOT % 256 != 0 && v >= TOT) break;
      const vec_t x = r[i];
      if constexpr (KCONTIG) {
        const int row = v / (BK / W);
        const int kk = (v % (BK / W)) * W;
        *reinterpret_cast<vec_t*>(lds + row * LDK + kk) = x;
      } else {
        const int kk = v / (ROWS / W);
        const int row = (v % (ROWS / W)) * W;
#pragma unroll
        for (int j = 0; j < W; ++j) lds[(row + j) * LDK + kk] = x[j];
      }
    }
  }
};

// CHECK = false: every tile is interior and every k slice is full (M, N
// multiples of the tile, K a multiple of BK, 16-byte aligned operands) -- the
// host launches this variant only then; it carries no bounds checks at all.
template <typename T, int BM, int BN, int BK, int MINW, bool AK, bool BKC, bool KS, bool CHECK>
__global__ __launch_bounds__(256, MINW) void gemm_kernel(KernelArgs<T> args) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc_t;
  constexpr int WM = 2, WN = 2;
  constexpr int PAD = 16 / sizeof(T);
  constexpr int LDK = BK + PAD;
  constexpr int KG = BK / 4;                 // k values per lane group per slice
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile must be a multiple of 16");
  static_assert((KG * sizeof(T)) % 16 == 0, "fragment reads are 16-byte vectors");

  __shared__ __attribute__((aligned(16))) T As[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][BN * LDK];
  // k-scaling factors (B(k,n) *= kscale[k]) of each staged slice
  __shared__ __attribute__((aligned(16))) T Ks[2][KS ? BK : 1];

  const KernelArgsCommon& c = args.c;
  const int G = gridDim.x;
  const int t = xcd_remap(blockIdx.x, G);
  const int tiles_mn = c.tiles_m * c.tiles_n;
  const int n_tile = t % c.tiles_n;
  const int m_tile = (t / c.tiles_n) % c.tiles_m;
  const int zs = t / tiles_mn;                  // batch * splits + split
  const int split = zs % c.splits;
  const int bz = zs / c.splits;

  const T* __restrict__ A = args.A + bz * c.bsA;
  const T* __restrict__ B = args.B + bz * c.bsB;
  const T* __restrict__ ks = args.kscale;
  const int64_t m0 = int64_t(m_tile) * BM;
  const int64_t n0 = int64_t(n_tile) * BN;
  if (c.lower && n0 >= m0 + BM) return;        // whole tile above the diagonal
  const int64_t kbeg = int64_t(split) * c.kchunk;
  const int64_t kend = std::min<int64_t>(c.K, kbeg + c.kchunk);
  const int nk = kend > kbeg ? int((kend - kbeg + BK - 1) / BK) : 0;
  // slices [0, nfull) of an interior tile need no bounds checks
  const bool interior = !CHECK || (c.vecA && c.vecB && m0 + BM <= c.M && n0 + BN <= c.N);
  const int nfull = !CHECK ? nk : (interior ? int((kend - kbeg) / BK) : 0);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lrow = lane & 15;
  const int lgrp = lane >> 4;

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = T(0);

  using LA = TileLoader<T, BM, BK, AK, false>;
  using LB = TileLoader<T, BN, BK, BKC, false>;
  LA la0, la1;
  LB lb0, lb1;
  T kv0 = T(0), kv1 = T(0);        // one k-scaling factor per thread < BK, per set
  const int64_t sA = AK ? c.sam : c.sak;
  const int64_t sB = BKC ? c.sbn : c.sbk;

  auto load = [&](LA& la, LB& lb, T& kv, int s) __attribute__((always_inline)) {
    const int64_t k0 = kbeg + int64_t(s) * BK;
    if (!CHECK || s < nfull) {
      la.load_fast(A, sA, m0, k0, nullptr);
      lb.load_fast(B, sB, n0, k0, nullptr);
    } else {
      la.load_checked(A, sA, m0, c.M, k0, kend, nullptr);
      lb.load_checked(B, sB, n0, c.N, k0, kend, nullptr);
    }
    if constexpr (KS) {
      if (threadIdx.x < BK)
        kv = (!CHECK || k0 + threadIdx.x < kend) ? ks[k0 + threadIdx.x] : T(0);
    }
  };
  auto stage_ks = [&](T kv, int stg) __attribute__((always_inline)) {
    if constexpr (KS) {
      if (threadIdx.x < BK) Ks[stg][threadIdx.x] = kv;
    }
  };

  auto compute = [&](const T* __restrict__ as, const T* __restrict__ bs,
                     const T* __restrict__ kss) __attribute__((always_inline)) {
    T af[TM][KG];
    T bf[TN][KG];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const T* p = as + (wm * WTM + i * 16 + lrow) * LDK + lgrp * KG;
#pragma unroll
      for (int q = 0; q < KG; q += Vec16<T>::W) {
        const typename Vec16<T>::type x = *reinterpret_cast<const typename Vec16<T>::type*>(p + q);
#pragma unroll
        for (int j = 0; j < Vec16<T>::W; ++j) af[i][q + j] = x[j];
      }
    }
#pragma unroll
    for (int i = 0; i < TN; ++i) {
      const T* p = bs + (wn * WTN + i * 16 + lrow) * LDK + lgrp * KG;
#pragma unroll
      for (int q = 0; q < KG; q += Vec16<T>::W) {
        const typename Vec16<T>::type x = *reinterpret_cast<const typename Vec16<T>::type*>(p + q);
#pragma unroll
        for (int j = 0; j < Vec16<T>::W; ++j) bf[i][q + j] = x[j];
      }
    }
    if constexpr (KS) {
      T kf[KG];
#pragma unroll
      for (int q = 0; q < KG; q += Vec16<T>::W) {
        const typename Vec16<T>::type x =
            *reinterpret_cast<const typename Vec16<T>::type*>(kss + lgrp * KG + q);
#pragma unroll
        for (int j = 0; j < Vec16<T>::W; ++j) kf[q + j] = x[j];
      }
#pragma unroll
      for (int i = 0; i < TN; ++i)
#pragma unroll
        for (int q = 0; q < KG; ++q) bf[i][q] *= kf[q];
    }
#pragma unroll
    for (int s = 0; s < KG; ++s)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MF::mma(af[i][s], bf[j][s], acc[i][j]);
  };

  // Two register sets: slice s lives in set s%2 from its load (two slices
  // ahead of its use) until it is written to LDS stage s%2.
  if (nk > 0) {
    load(la0, lb0, kv0, 0);
    if (nk > 1) load(la1, lb1, kv1, 1);
    la0.template store<LDK>(As[0]);
    lb0.template store<LDK>(Bs[0]);
    stage_ks(kv0, 0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; kt += 2) {
    // even slice: compute stage 0, refill set 0 with slice kt+2, stage slice kt+1
    if (kt + 2 < nk) load(la0, lb0, kv0, kt + 2);
    compute(As[0], Bs[0], Ks[0]);
    if (kt + 1 < nk) {
      la1.template store<LDK>(As[1]);
      lb1.template store<LDK>(Bs[1]);
      stage_ks(kv1, 1);
    }
    __syncthreads();
    if (kt + 1 >= nk) break;
    // odd slice: compute stage 1, refill set 1 with slice kt+3, stage slice kt+2
    if (kt + 3 < nk) load(la1, lb1, kv1, kt + 3);
    compute(As[1], Bs[1], Ks[1]);
    if (kt + 2 < nk) {
      la0.template store<LDK>(As[0]);
      lb0.template store<LDK>(Bs[0]);
      stage_ks(kv0, 0);
    }
    __syncthreads();
  }

  // Output fragment layout of the 16x16 MFMA: lane l, element r holds
  // row MF::out_row(l/16, r), column l%16 of the tile.
  if (c.splits == 1) {
    T* C = args.C + bz * c.bsC;
    Epilogue<T> e = args.epi;
    if (e.C1) e.C1 += bz * c.bsC1;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t n = n0 + wn * WTN + j * 16 + lrow;
        if (CHECK && n >= c.N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = m0 + wm * WTM + i * 16 + MF::out_row(lgrp, r);
          if (!CHECK || m < c.M) C[m + n * c.ldc] = apply_epilogue(e, acc[i][j][r], m, n);
        }
      }
  } else {
    T* P = args.partial + int64_t(zs) * c.M * c.N;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t n = n0 + wn * WTN + j * 16 + lrow;
        if (CHECK && n >= c.N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = m0 + wm * WTM + i * 16 + MF::out_row(lgrp, r);
          if (!CHECK || m < c.M) P[m + n * c.M] = acc[i][j][r];
        }
      }
  }
}

// Sum split-K partials in split order, then apply the epilogue; four rows per
// thread with 16-byte accesses (M and every leading dimension multiples of 4,
// 16-byte aligned bases; batch 1).
// grid: x over 1024-row chunks, y over columns (grid-stride beyond gridDim.y)
__global__ __launch_bounds__(256) void splitk_reduce4_kernel(KernelArgs<float> args) {
  const KernelArgsCommon& c = args.c;
  const int64_t MN = c.M * c.N;
  const int64_t m = (int64_t(blockIdx.x) * 256 + threadIdx.x) * 4;
  if (m >= c.M) return;
  const Epilogue<float> ep = args.epi;
  f32x4 sc16 = {1.f, 1.f, 1.f, 1.f};
  if (args.out16 && args.scale16) sc16 = *reinterpret_cast<const f32x4*>(args.scale16 + m);
  for (int64_t n = blockIdx.y; n < c.N; n += gridDim.y) {
    const float* P = args.partial + m + n * c.M;
    f32x4 s = *reinterpret_cast<const f32x4*>(P);
    for (int q = 1; q < c.splits; ++q) s += *reinterpret_cast<const f32x4*>(P + q * MN);
    f32x4 v = ep.alpha * s;
    if (ep.rowscale) v *= *reinterpret_cast<const f32x4*>(ep.rowscale + m);
    if (ep.C1) v += ep.beta * *reinterpret_cast<const f32x4*>(ep.C1 + m + n * ep.ldc1);
    if (ep.C2) v += ep.gamma * *reinterpret_cast<const f32x4*>(ep.C2 + m + n * ep.ldc2);
    if (ep.C3) {
      float f = ep.delta;
      if (ep.colscale3) f *= ep.colscale3[n];
      v += f * *reinterpret_cast<const f32x4*>(ep.C3 + m + n * ep.ldc3);
    }
    *reinterpret_cast<f32x4*>(args.C + m + n * c.ldc) = v;
    if (args.out16) {
      const f32x4 w = v * sc16;
      const uint32_t lo = uint32_t(f32_to_bf16_rne(w[0])) | (uint32_t(f32_to_bf16_rne(w[1])) << 16);
      const uint32_t hi = uint32_t(f32_to_bf16_rne(w[2])) | (uint32_t(f32_to_bf16_rne(w[3])) << 16);
      *reinterpret_cast<uint2*>(args.out16 + m + n * c.M) = make_uint2(lo, hi);
    }
  }
}

static dim3 reduce4_grid(int64_t M, int64_t N) {
  return dim3(unsigned((M / 4 + 255) / 256), unsigned(std::min<int64_t>(N, 65535)));
}

static bool reduce4_ok(const KernelArgs<float>& a, int batch) {
  auto al = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
  const Epilogue<float>& e = a.epi;
  return batch == 1 && a.c.M % 4 == 0 && a.c.ldc % 4 == 0 && al(a.C) && al(a.partial) &&
         (!e.rowscale || al(e.rowscale)) && (!e.C1 || (al(e.C1) && e.ldc1 % 4 == 0)) &&
         (!e.C2 || (al(e.C2) && e.ldc2 % 4 == 0)) && (!e.C3 || (al(e.C3) && e.ldc3 % 4 == 0));
}

// Sum split-K partials in split order, then apply the epilogue.
template <typename T>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(KernelArgs<T> args) {
  const KernelArgsCommon& c = args.c;
  const int64_t MN = c.M * c.N;
  const int64_t total = MN * c.batch;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t bz = idx / MN;
    const int64_t e = idx - bz * MN;
    const int64_t m = e % c.M, n = e / c.M;
    const T* P = args.partial + bz * c.splits * MN + e;
    T s = T(0);
    for (int q = 0; q < c.splits; ++q) s += P[q * MN];
    Epilogue<T> ep = args.epi;
    if (ep.C1) ep.C1 += bz * c.bsC1;
    T* C = args.C + bz * c.bsC;
    C[m + n * c.ldc] = apply_epilogue(ep, s, m, n);
  }
}

// ---------------------------------------------------------------------------
// FP64 Gram product C = A B over a long k range (A: M x K, B: K x N, both
// k-contiguous; M = N; only tiles reaching the diagonal or below): the
// Rayleigh-Ritz Gram matrices Y^T W of the grid pencils.
//
// A 256 x 128 tile per workgroup of eight waves (4 x 2, 64 x 64 each on
// v_mfma_f64_16x16x4f64), one workgroup per CU.  Split-K over the eight XCDs:
// every workgroup of one k-range runs on one XCD, and with at most 32 tiles
// per k-range (M <= 1280) all of them are resident at once on that XCD's 32
// CUs, start together and march through k at the same pace, so each k-slice
// of Y and W is fetched into that XCD's L2 about once and read there by every
// tile that needs it.  (With 128 x 64 tiles, 109 tiles per k-range at
// b = 1200 cannot all be resident; the late ones re-read their panels.)
// Measured at 128^3 x 1200: 76 GB of L2 fills per Gram product (operands
// 40 GB) against 336 GB, 76 ms against 84 ms: two waves per SIMD and one
// slice of prefetch (a second register set does not fit) leave it at half
// the FP64 MFMA peak.  Partial sums go to the split-K buffer; the reduction
// applies the epilogue.
// ---------------------------------------------------------------------------
constexpr int kGramBM = 256, kGramBN = 128, kGramBK = 16, kGramLDK = kGramBK + 2;

__global__ __launch_bounds__(512, 1) void gram_f64_kernel(KernelArgs<double> args, int ntiles) {
  using MF = Mfma<double>;
  typedef double f64x2 __attribute__((ext_vector_type(2)));
  __shared__ __attribute__((aligned(16))) double As[2][kGramBM * kGramLDK];
  __shared__ __attribute__((aligned(16))) double Bs[2][kGramBN * kGramLDK];
  const KernelArgsCommon& c = args.c;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int split = t / ntiles;
  int tile = t - split * ntiles;
  // lower tiles in row-major order: row i holds n-tiles 0 .. min(2 (i + 1), tiles_n) - 1
  int mi = 0;
  for (;;) {
    const int cnt = min(2 * (mi + 1), c.tiles_n);
    if (tile < cnt) break;
    tile -= cnt;
    ++mi;
  }
  const int64_t m0 = int64_t(mi) * kGramBM, n0 = int64_t(tile) * kGramBN;
  const int64_t kbeg = int64_t(split) * c.kchunk;
  const int64_t kend = min(c.K, kbeg + c.kchunk);
  const int nk = kend > kbeg ? int((kend - kbeg) / kGramBK) : 0;
  const double* __restrict__ A = args.A;
  const double* __restrict__ B = args.B;
  const int64_t lda = c.sam, ldb = c.sbn;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 3, wn = wave >> 2;
  const int l16 = lane & 15, lg = lane >> 4;

  f64x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  // staging: A slice 256 rows x 16 k (4 vectors of 2 doubles per thread),
  // B slice 128 rows x 16 k (2 per thread); rows past M (N) read as zero.
  // One register set, loaded a slice ahead (two sets do not fit the 256
  // registers of two waves per SIMD).
  f64x2 ra[4], rb[2];
  auto load = [&](int s) __attribute__((always_inline)) {
    const int64_t k0 = kbeg + int64_t(s) * kGramBK;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int v = threadIdx.x + q * 512, row = v >> 3, kk = (v & 7) * 2;
      const int64_t gr = m0 + row;
      ra[q] = gr < c.M ? *reinterpret_cast<const f64x2*>(A + gr * lda + k0 + kk) : f64x2{0.0, 0.0};
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int v = threadIdx.x + q * 512, row = v >> 3, kk = (v & 7) * 2;
      const int64_t gr = n0 + row;
      rb[q] = gr < c.N ? *reinterpret_cast<const f64x2*>(B + gr * ldb + k0 + kk) : f64x2{0.0, 0.0};
    }
  };
  auto store = [&](int stg) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int v = threadIdx.x + q * 512, row = v >> 3, kk = (v & 7) * 2;
      *reinterpret_cast<f64x2*>(&As[stg][row * kGramLDK + kk]) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int v = threadIdx.x + q * 512, row = v >> 3, kk = (v & 7) * 2;
      *reinterpret_cast<f64x2*>(&Bs[stg][row * kGramLDK + kk]) = rb[q];
    }
  };
  auto compute = [&](int stg) __attribute__((always_inline)) {
    const double* as = &As[stg][(wm * 64 + l16) * kGramLDK + lg];
    const double* bs = &Bs[stg][(wn * 64 + l16) * kGramLDK + lg];
#pragma unroll
    for (int k4 = 0; k4 < kGramBK; k4 += 4) {
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = as[i * 16 * kGramLDK + k4];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = bs[j * 16 * kGramLDK + k4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = MF::mma(af[i], bf[j], acc[i][j]);
    }
  };

  if (nk > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load(kt + 1);
    compute(kt & 1);
    if (kt + 1 < nk) store((kt + 1) & 1);
    __syncthreads();
  }

  double* P = args.partial + int64_t(split) * c.M * c.N;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t n = n0 + wn * 64 + j * 16 + l16;
      if (n >= c.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 64 + i * 16 + MF::out_row(lg, r);
        if (m < c.M) P[m + n * c.M] = acc[i][j][r];
      }
    }
}

// The Gram kernel for the shapes it takes (a long k range, lower only,
// k-contiguous 16-byte aligned operands, K and the split length multiples of
// 16, 1024 < M = N <= 1280 (20-30 tiles per k-range: enough workgroups to
// fill the GPU, few enough to be resident together), room for the partial
// sums); returns false otherwise.
// Knob CHFSI_GRAM_KERNEL=0 turns it off.
static bool gram_launch(const GemmDesc<double>& d, hipStream_t st, const Workspace& ws,
                        hipError_t* err) {
  static const bool on = [] {
    const char* e = std::getenv("CHFSI_GRAM_KERNEL");
    return !(e && std::atoi(e) == 0);
  }();
  if (!on || !d.lower_only || d.batch != 1 || d.kscale || d.sak != 1 || d.sbk != 1) return false;
  if (d.M != d.N || d.M > 1280 || d.M <= 1024 || d.K < 16 * d.M || d.K % (kGramBK * 8) != 0)
    return false;
  if (reinterpret_cast<uintptr_t>(d.A) % 16 || reinterpret_cast<uintptr_t>(d.B) % 16 ||
      d.sam % 2 || d.sbn % 2)
    return false;
  constexpr int splits = 8;   // one k-range per XCD
  const size_t need = size_t(splits) * d.M * d.N * sizeof(double);
  if (need > ws.bytes || ws.ptr == nullptr) return false;
  KernelArgs<double> a;
  KernelArgsCommon& c = a.c;
  c.M = d.M;
  c.N = d.N;
  c.K = d.K;
  c.sam = d.sam;
  c.sak = 1;
  c.sbk = 1;
  c.sbn = d.sbn;
  c.ldc = d.ldc;
  c.batch = 1;
  c.bsA = c.bsB = c.bsC = c.bsC1 = 0;
  c.lower = 1;
  c.tiles_m = int((d.M + kGramBM - 1) / kGramBM);
  c.tiles_n = int((d.N + kGramBN - 1) / kGramBN);
  c.kchunk = d.K / splits;   // a multiple of 16
  c.splits = splits;
  int ntiles = 0;
  for (int i = 0; i < c.tiles_m; ++i) ntiles += std::min(2 * (i + 1), c.tiles_n);
  a.A = d.A;
  a.B = d.B;
  a.kscale = nullptr;
  a.C = d.C;
  a.epi = d.epi;
  a.partial = static_cast<double*>(ws.ptr);
  if (d.ev_begin && (*err = hipEventRecord(d.ev_begin, st)) != hipSuccess) return true;
  gram_f64_kernel<<<dim3(unsigned(ntiles * splits)), dim3(512), 0, st>>>(a, ntiles);
  if ((*err = hipGetLastError()) != hipSuccess) return true;
  const int64_t total = d.M * d.N;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
  splitk_reduce_kernel<double><<<dim3(blocks), dim3(256), 0, st>>>(a);
  if ((*err = hipGetLastError()) != hipSuccess) return true;
  if (d.ev_end && (*err = hipEventRecord(d.ev_end, st)) != hipSuccess) return true;
  *err = hipSuccess;
  return true;
}

// ---------------------------------------------------------------------------
// configurations and dispatch
// ---------------------------------------------------------------------------
struct Cfg {
  int BM, BN, BK, occ;   // occ: resident workgroups per CU assumed by the planner
};

// Tile shapes.  FP32 shapes are used for the filter products (both operands
// k-contiguous); every other layout uses the last (generic) entry.
static const Cfg kCfgF32[] = {{128, 128, 32, 1}, {128, 160, 16, 1}, {128, 64, 32, 2},
                              {64, 160, 16, 2},  {128, 160, 32, 1}, {64, 320, 16, 1},
                              {64, 64, 32, 4}};
static const Cfg kCfgF64[] = {{128, 128, 16, 1}, {128, 64, 16, 2}, {64, 64, 16, 3}};
static constexpr int kNumF32 = 7, kNumF64 = 3;
static constexpr int kNumCU = 256;

[[maybe_unused]] static int choose_splits(int64_t tiles, int64_t K, int BK, int slots) {
  // enough work items to fill every resident slot a few times, but keep at
  // least 8 k-slices per split
  int s = 1;
  const int64_t max_s = std::max<int64_t>(1, K / (8 * BK));
  while (tiles * s < 2 * slots && s * 2 <= max_s && s < 64) s *= 2;
  return s;
}

// Tile/split choice.  Measured on MI355X (rocprofv3 + HIP events, the filter
// shape M = K = 8192, N = 320): 64 x 64 tiles at high occupancy with enough
// split-K work items to give every CU ~16 workgroups beat the larger tiles
// (FP32 k-scaled: 64x64x32 / 8 splits 118 TFLOP/s vs 128x160 95; FP64:
// 64x64x16 / 4 splits 58-61 TFLOP/s).  Larger tiles remain selectable through
// force_config for other shapes.
//
// FP64 products with a long reduction (K >= 16 max(M, N), M, N >= 128: the
// Gram matrices Y^T W of Rayleigh-Ritz) use 128 x 64 tiles and 8 k-splits.
// The tile -> XCD remap then gives each XCD one k-range, whose panels every
// tile on that XCD shares in its L2.  Measured on the 128^3 x 1200 grid
// pencil (whole Rayleigh-Ritz, same process): 128x64 / 8 splits 375 ms,
// 64x64 / 8 402 ms, 128x128 / 8 403 ms; 4 splits 456-593 ms; 16-64 splits
// 610-990 ms (a k-range per XCD no longer holds).  Tuning knobs (read per
// call): CHFSI_GEMM64_LONG_CFG (0 = 128x128, 1 = 128x64, 2 = 64x64) and
// CHFSI_GEMM64_LONG_SPLITS (power of two, at most 64).
static int env_int(const char* name, int dflt) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : dflt;
}

template <typename T>
static void plan_impl(int64_t M, int64_t N, int64_t K, int batch, bool filter_layout, int* config,
                      int* splits) {
  (void)filter_layout;
  const int ncfg = sizeof(T) == 4 ? kNumF32 : kNumF64;
  // the long-K rule also serves the complex Gram products (two batched
  // b x b blocks; knob CHFSI_GEMM64_LONG_BATCHED = 0 gives them the general plan)
  const bool long_batched = env_int("CHFSI_GEMM64_LONG_BATCHED", 1) > 0 && batch <= 2;
  if (sizeof(T) == 8 && (batch == 1 || long_batched) && M >= 128 && N >= 128 &&
      K >= 16 * std::max(M, N)) {
    int lcfg = env_int("CHFSI_GEMM64_LONG_CFG", 1);
    if (lcfg < 0 || lcfg >= kNumF64) lcfg = 1;
    const int lsplits = env_int("CHFSI_GEMM64_LONG_SPLITS", 8);
    const Cfg& w = kCfgF64[lcfg];
    const int64_t max_s = std::max<int64_t>(1, K / (8 * w.BK));
    int s = 1;
    while (s * 2 <= lsplits && s * 2 <= max_s && s < 64) s *= 2;
    *config = lcfg;
    *splits = s;
    return;
  }
  // FP64 products with a large output (M N >= 2^24, e.g. the grid rotation
  // X = Y Q): knob CHFSI_GEMM64_BIG_CFG (0 = 128x128, 1 = 128x64, 2 = 64x64)
  int gcfg = ncfg - 1;
  if (sizeof(T) == 8 && M * N >= (int64_t(1) << 24)) {
    const int bc = env_int("CHFSI_GEMM64_BIG_CFG", ncfg - 1);
    if (bc >= 0 && bc < ncfg) gcfg = bc;
  }
  const Cfg& f = (sizeof(T) == 4 ? kCfgF32 : kCfgF64)[gcfg];
  const int64_t tiles = ((M + f.BM - 1) / f.BM) * ((N + f.BN - 1) / f.BN) * batch;
  const int64_t target = int64_t(kNumCU) * (sizeof(T) == 4 ? 16 : 8);
  const int64_t max_s = std::max<int64_t>(1, K / (8 * f.BK));
  int s = 1;
  while (tiles * s < target && s * 2 <= max_s && s < 64) s *= 2;
  *config = gcfg;
  *splits = s;
}

template <typename T>
void gemm_plan(int64_t M, int64_t N, int64_t K, int batch, int* config, int* splits) {
  plan_impl<T>(M, N, K, batch, true, config, splits);
}

size_t gemm_workspace_bytes(int64_t M, int64_t N, int64_t K, size_t elem) {
  (void)K;
  return size_t(64) * size_t(M) * size_t(N) * elem;
}

template <typename T, int BM, int BN, int BK, int MINW, bool FILTER_ONLY = false>
static hipError_t launch_cfg(const GemmDesc<T>& d, hipStream_t st, const Workspace& ws,
                             int splits) {
  KernelArgs<T> a;
  KernelArgsCommon& c = a.c;
  c.M = d.M;
  c.N = d.N;
  c.K = d.K;
  c.sam = d.sam;
  c.sak = d.sak;
  c.sbk = d.sbk;
  c.sbn = d.sbn;
  c.ldc = d.ldc;
  c.batch = d.batch;
  c.bsA = d.bsA;
  c.bsB = d.bsB;
  c.bsC = d.bsC;
  c.bsC1 = d.bsC1;
  c.tiles_m = int((d.M + BM - 1) / BM);
  c.lower = d.lower_only ? 1 : 0;
  c.tiles_n = int((d.N + BN - 1) / BN);
  const bool AK = (d.sak == 1);
  const bool BKC = (d.sbk == 1);
  constexpr int W = 16 / sizeof(T);
  const int64_t ldA = AK ? d.sam : d.sak;
  const int64_t ldB = BKC ? d.sbn : d.sbk;
  c.vecA = (reinterpret_cast<uintptr_t>(d.A) % 16 == 0) && (ldA % W == 0) &&
           (d.batch == 1 || d.bsA % W == 0);
  c.vecB = (reinterpret_cast<uintptr_t>(d.B) % 16 == 0) && (ldB % W == 0) &&
           (d.batch == 1 || d.bsB % W == 0) &&
           (d.kscale == nullptr || reinterpret_cast<uintptr_t>(d.kscale) % 16 == 0);
  if (splits > 1) {
    int64_t kchunk = (d.K + splits - 1) / splits;
    kchunk = (kchunk + BK - 1) / BK * BK;
    splits = int((d.K + kchunk - 1) / kchunk);
    c.kchunk = kchunk;
  } else {
    c.kchunk = (d.K + BK - 1) / BK * BK;
    if (c.kchunk == 0) c.kchunk = BK;
  }
  c.splits = std::max(splits, 1);
  a.A = d.A;
  a.B = d.B;
  a.kscale = d.kscale;
  a.C = d.C;
  a.epi = d.epi;
  a.partial = nullptr;
  if (c.splits > 1) {
    const size_t need = size_t(c.splits) * d.batch * d.M * d.N * sizeof(T);
    if (need > ws.bytes || ws.ptr == nullptr) {
      c.splits = 1;
      c.kchunk = (d.K + BK - 1) / BK * BK;
    } else {
      a.partial = static_cast<T*>(ws.ptr);
    }
  }
  const int64_t grid = int64_t(c.tiles_m) * c.tiles_n * c.splits * d.batch;
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  if (d.ev_begin) {
    hipError_t e0 = hipEventRecord(d.ev_begin, st);
    if (e0 != hipSuccess) return e0;
  }
  const bool KS = d.kscale != nullptr;
  // the unchecked variant needs whole tiles, whole k slices and aligned operands
  const bool aligned = c.vecA && c.vecB && d.M % BM == 0 && d.N % BN == 0 && d.K % BK == 0 &&
                       c.kchunk % BK == 0;
  if (AK && BKC) {
    if (aligned) {
      if (KS)
        gemm_kernel<T, BM, BN, BK, MINW, true, true, true, false><<<dim3(grid), dim3(256), 0, st>>>(a);
      else
        gemm_kernel<T, BM, BN, BK, MINW, true, true, false, false><<<dim3(grid), dim3(256), 0, st>>>(a);
    } else {
      if (KS)
        gemm_kernel<T, BM, BN, BK, MINW, true, true, true, true><<<dim3(grid), dim3(256), 0, st>>>(a);
      else
        gemm_kernel<T, BM, BN, BK, MINW, true, true, false, true><<<dim3(grid), dim3(256), 0, st>>>(a);
    }
  } else if (KS || FILTER_ONLY) {
    return hipErrorInvalidValue;   // k-scaling is only used with k-contiguous operands
  } else if constexpr (FILTER_ONLY) {
    return hipErrorInvalidValue;
  } else if (AK && !BKC) {
    gemm_kernel<T, BM, BN, BK, MINW, true, false, false, true><<<dim3(grid), dim3(256), 0, st>>>(a);
  } else if (!AK && BKC) {
    gemm_kernel<T, BM, BN, BK, MINW, false, true, false, true><<<dim3(grid), dim3(256), 0, st>>>(a);
  } else {
    gemm_kernel<T, BM, BN, BK, MINW, false, false, false, true><<<dim3(grid), dim3(256), 0, st>>>(a);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if (c.splits > 1) {
    const int64_t total = d.M * d.N * d.batch;
    bool done = false;
    if constexpr (sizeof(T) == 4) {
      if (reduce4_ok(a, d.batch)) {
        splitk_reduce4_kernel<<<reduce4_grid(d.M, d.N), dim3(256), 0, st>>>(a);
        done = true;
      }
    }
    if (!done) {
      const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
      splitk_reduce_kernel<T><<<dim3(blocks), dim3(256), 0, st>>>(a);
    }
    err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  // the profiling interval ends after the split-K reduction, which carries the
  // fused epilogue: it times the whole recurrence step
  if (d.ev_end) {
    err = hipEventRecord(d.ev_end, st);
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

// Launchers for the FP32 filter shapes (both operands k-contiguous only).
template <int BM, int BN, int BK, int MINW>
static hipError_t launch_f32_filter(const GemmDesc<float>& d, hipStream_t st, const Workspace& ws,
                                    int splits) {
  return launch_cfg<float, BM, BN, BK, MINW, true>(d, st, ws, splits);
}

template <typename T>
hipError_t gemm(const GemmDesc<T>& d, hipStream_t st, const Workspace& ws, int force_splits,
                int force_config) {
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  if (d.sam != 1 && d.sak != 1) return hipErrorInvalidValue;
  if (d.sbk != 1 && d.sbn != 1) return hipErrorInvalidValue;
  if (d.batch > 1 && (d.epi.C2 || d.epi.C3 || d.epi.rowscale)) return hipErrorInvalidValue;
  const bool filter_layout = (d.sak == 1) && (d.sbk == 1);
  int cfg, splits;
  plan_impl<T>(d.M, d.N, d.K, d.batch, filter_layout, &cfg, &splits);
  const int ncfg = sizeof(T) == 4 ? kNumF32 : kNumF64;
  if (force_config >= 0 && force_config < ncfg && (sizeof(T) == 8 || filter_layout))
    cfg = force_config;
  if (force_splits > 0) splits = force_splits;
  if (d.K <= 0) splits = 1;
  if constexpr (sizeof(T) == 8) {
    hipError_t gerr = hipSuccess;
    if (force_config < 0 && force_splits <= 0 && gram_launch(d, st, ws, &gerr)) return gerr;
  }
  if constexpr (sizeof(T) == 4) {
    if (!filter_layout) return launch_cfg<float, 64, 64, 32, 4>(d, st, ws, splits);
    switch (cfg) {
      case 0: return launch_f32_filter<128, 128, 32, 1>(d, st, ws, splits);
      case 1: return launch_f32_filter<128, 160, 16, 1>(d, st, ws, splits);
      case 2: return launch_f32_filter<128, 64, 32, 2>(d, st, ws, splits);
      case 3: return launch_f32_filter<64, 160, 16, 2>(d, st, ws, splits);
      case 4: return launch_f32_filter<128, 160, 32, 1>(d, st, ws, splits);
      case 5: return launch_f32_filter<64, 320, 16, 1>(d, st, ws, splits);
      default: return launch_f32_filter<64, 64, 32, 4>(d, st, ws, splits);
    }
  } else {
    switch (cfg) {
      case 0: return launch_cfg<T, 128, 128, 16, 1>(d, st, ws, splits);
      case 1: return launch_cfg<T, 128, 64, 16, 2>(d, st, ws, splits);
      default: return launch_cfg<T, 64, 64, 16, 3>(d, st, ws, splits);
    }
  }
}

// ---------------------------------------------------------------------------
// BF16 product for the dense residual filter: C = epilogue(A16 * B16), A16
// the operator rounded once to bfloat16 and B16 = bfloat16(D^{-1} R_Y) (both
// k-contiguous, 16-byte vector loads), products on v_mfma_f32_16x16x32_bf16
// with FP32 accumulation, the FP32 three-term epilogue (or split-K partials)
// as in gemm_kernel.  Lane l supplies A(l%16, 8 k-values of group l/16) and
// the same k-values of B(., l%16); output element r of lane l is row
// 4 (l/16) + r, column l%16 of the 16 x 16 tile.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));

template <int BM, int BN, int BK, bool CHECK>
__global__ __launch_bounds__(256, 2) void gemm_bf16_kernel(KernelArgs<float> args,
                                                           const unsigned short* __restrict__ A16,
                                                           const unsigned short* __restrict__ B16) {
  constexpr int WM = 2, WN = 2, WTM = BM / WM, WTN = BN / WN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int LDK = BK + 8;                  // bf16 elements per LDS row (16-byte pad)
  constexpr int NVA = BM * BK / 8 / 256;       // 8-element vectors per thread
  constexpr int NVB = BN * BK / 8 / 256;
  static_assert(NVA * 8 * 256 == BM * BK && NVB * 8 * 256 == BN * BK, "tile / thread mismatch");
  static_assert(BK % 32 == 0 && WTM % 16 == 0 && WTN % 16 == 0, "tile shape");
  __shared__ __attribute__((aligned(16))) unsigned short As[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][BN * LDK];

  const KernelArgsCommon& c = args.c;
  const int G = gridDim.x;
  const int t = xcd_remap(blockIdx.x, G);
  const int tiles_mn = c.tiles_m * c.tiles_n;
  const int n_tile = t % c.tiles_n;
  const int m_tile = (t / c.tiles_n) % c.tiles_m;
  const int split = t / tiles_mn;
  const int64_t m0 = int64_t(m_tile) * BM, n0 = int64_t(n_tile) * BN;
  const int64_t kbeg = int64_t(split) * c.kchunk;
  const int64_t kend = std::min<int64_t>(c.K, kbeg + c.kchunk);
  const int nk = kend > kbeg ? int((kend - kbeg + BK - 1) / BK) : 0;
  const int64_t lda = c.sam, ldb = c.sbn;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lrow = lane & 15, lgrp = lane >> 4;

  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  struct Regs {
    u16x8_t a[NVA];
    u16x8_t b[NVB];
  };
  Regs r0, r1;
  // one operand tile: ROWS rows (m or n) x BK k-values, 8 k-values per vector
  auto load_tile = [&](u16x8_t* R, int NV, const unsigned short* __restrict__ X, int64_t ldx,
                       int64_t r0_, int64_t rmax, int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int v = threadIdx.x + i * 256;
      const int row = v / (BK / 8), kk = (v % (BK / 8)) * 8;
      const int64_t gr = r0_ + row, gk = k0 + kk;
      if (!CHECK) {
        R[i] = *reinterpret_cast<const u16x8_t*>(X + gr * ldx + gk);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
          R[i][j] = (gr < rmax && gk + j < kend) ? X[gr * ldx + gk + j] : (unsigned short)0;
      }
    }
  };
  auto load = [&](Regs& R, int s) __attribute__((always_inline)) {
    const int64_t k0 = kbeg + int64_t(s) * BK;
    load_tile(R.a, NVA, A16, lda, m0, c.M, k0);
    load_tile(R.b, NVB, B16, ldb, n0, c.N, k0);
  };
  auto store = [&](const Regs& R, int stg) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < NVA; ++i) {
      const int v = threadIdx.x + i * 256;
      *reinterpret_cast<u16x8_t*>(&As[stg][(v / (BK / 8)) * LDK + (v % (BK / 8)) * 8]) = R.a[i];
    }
#pragma unroll
    for (int i = 0; i < NVB; ++i) {
      const int v = threadIdx.x + i * 256;
      *reinterpret_cast<u16x8_t*>(&Bs[stg][(v / (BK / 8)) * LDK + (v % (BK / 8)) * 8]) = R.b[i];
    }
  };
  auto compute = [&](int stg) __attribute__((always_inline)) {
#pragma unroll
    for (int k0 = 0; k0 < BK; k0 += 32) {
      bf16x8_t af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        af[i] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u16x8_t*>(
                                                 &As[stg][(wm * WTM + i * 16 + lrow) * LDK + k0 +
                                                          lgrp * 8]));
#pragma unroll
      for (int j = 0; j < TN; ++j)
        bf[j] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u16x8_t*>(
                                                 &Bs[stg][(wn * WTN + j * 16 + lrow) * LDK + k0 +
                                                          lgrp * 8]));
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  };

  // two register sets: slice s is loaded two slices ahead of its use
  if (nk > 0) {
    load(r0, 0);
    if (nk > 1) load(r1, 1);
    store(r0, 0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; kt += 2) {
    if (kt + 2 < nk) load(r0, kt + 2);
    compute(0);
    if (kt + 1 < nk) store(r1, 1);
    __syncthreads();
    if (kt + 1 >= nk) break;
    if (kt + 3 < nk) load(r1, kt + 3);
    compute(1);
    if (kt + 2 < nk) store(r0, 0);
    __syncthreads();
  }

  if (c.splits == 1) {
    const Epilogue<float> e = args.epi;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t n = n0 + wn * WTN + j * 16 + lrow;
        if (CHECK && n >= c.N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = m0 + wm * WTM + i * 16 + lgrp * 4 + r;
          if (!CHECK || m < c.M) args.C[m + n * c.ldc] = apply_epilogue(e, acc[i][j][r], m, n);
        }
      }
  } else {
    float* P = args.partial + int64_t(split) * c.M * c.N;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t n = n0 + wn * WTN + j * 16 + lrow;
        if (CHECK && n >= c.N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = m0 + wm * WTM + i * 16 + lgrp * 4 + r;
          if (!CHECK || m < c.M) P[m + n * c.M] = acc[i][j][r];
        }
      }
  }
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

// BF16 product on v_mfma_f32_32x32x16_bf16 for aligned shapes (M % 128 == 0,
// N % (64 TN) == 0, K and the split length multiples of 64, 16-byte aligned
// operands with leading dimensions multiples of 8).  A 32 x 32 x 16 product
// reads one 16-byte fragment of each operand per lane for 32 x 32 x 16 x 2
// flops, half the operand traffic per flop of the 16 x 16 x 32 form.
//  * Workgroup tile 128 x 64 TN, four waves as 2 (m) x 2 (n), each wave
//    64 x 32 TN (2 x TN accumulator tiles of 32 x 32).
//  * The right operand (N x K, K contiguous) is staged through LDS in 64-deep
//    slices, double-buffered; its rows are 128 bytes with the 16-byte chunks
//    XOR-swizzled by (row & 7), so that the eight rows a fragment read touches
//    at once fall on distinct banks.
//  * The left operand (M x K, K contiguous) goes from global memory straight
//    into registers, two slices ahead: lane l (row l % 32, half h = l / 32)
//    takes k = h*32 + 8s .. +8 at step s of a slice, i.e. 64 contiguous bytes
//    per row and slice.  The right operand's fragments use the same order of
//    k, which leaves every dot product's terms unchanged.
template <int TN>
__global__ __launch_bounds__(256, 1) void gemm_bf16_wide_kernel(
    KernelArgs<float> args, const unsigned short* __restrict__ A16,
    const unsigned short* __restrict__ B16) {
  constexpr int BM = 128, BN = 64 * TN, BK = 64, TM = 2;
  constexpr int NVB = BN * BK / 8 / 256;       // 16-byte right-operand vectors per thread
  static_assert(NVB * 8 * 256 == BN * BK, "tile / thread mismatch");
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][BN * BK];

  const KernelArgsCommon& c = args.c;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int tiles_mn = c.tiles_m * c.tiles_n;
  const int n_tile = t % c.tiles_n;
  const int m_tile = (t / c.tiles_n) % c.tiles_m;
  const int split = t / tiles_mn;
  const int64_t m0 = int64_t(m_tile) * BM, n0 = int64_t(n_tile) * BN;
  const int64_t kbeg = int64_t(split) * c.kchunk;
  const int64_t kend = std::min<int64_t>(c.K, kbeg + c.kchunk);
  const int nk = kend > kbeg ? int((kend - kbeg) / BK) : 0;
  const int64_t lda = c.sam, ldb = c.sbn;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l32 = lane & 31, h = lane >> 5;

  const unsigned short* Ap[TM];
#pragma unroll
  for (int i = 0; i < TM; ++i) Ap[i] = A16 + (m0 + wm * 64 + i * 32 + l32) * lda + kbeg + h * 32;

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  u16x8_t a0[TM][4], a1[TM][4], a2[TM][4];
  u16x8_t bst[NVB];
  auto load_a = [&](u16x8_t (&R)[TM][4], int s) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        R[i][q] = *reinterpret_cast<const u16x8_t*>(Ap[i] + int64_t(s) * BK + q * 8);
  };
  auto load_b = [&](int s) __attribute__((always_inline)) {
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const int idx = threadIdx.x + v * 256, row = idx >> 3, ch = idx & 7;
      bst[v] = *reinterpret_cast<const u16x8_t*>(B16 + (n0 + row) * ldb + kbeg +
                                                  int64_t(s) * BK + ch * 8);
    }
  };
  auto store_b = [&](int stg) __attribute__((always_inline)) {
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const int idx = threadIdx.x + v * 256, row = idx >> 3, ch = idx & 7;
      *reinterpret_cast<u16x8_t*>(&Bs[stg][row * BK + ((ch ^ (row & 7)) << 3)]) = bst[v];
    }
  };
  auto compute = [&](int stg, const u16x8_t (&R)[TM][4]) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      bf16x8_t bf[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int row = wn * 32 * TN + j * 32 + l32, ch = 4 * h + s;
        bf[j] = __builtin_bit_cast(
            bf16x8_t, *reinterpret_cast<const u16x8_t*>(&Bs[stg][row * BK + ((ch ^ (row & 7)) << 3)]));
      }
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const bf16x8_t af = __builtin_bit_cast(bf16x8_t, R[i][s]);
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bf[j], acc[i][j], 0, 0, 0);
      }
    }
  };
  // one step of the slice loop: slice kt in stage kt & 1 with left-operand
  // registers RC; slice kt + 2 is loaded into RN, slice kt + 1's right operand
  // goes to the other stage
  auto step = [&](int kt, const u16x8_t (&RC)[TM][4], u16x8_t (&RN)[TM][4])
      __attribute__((always_inline)) {
    if (kt + 2 < nk) load_a(RN, kt + 2);
    compute(kt & 1, RC);
    if (kt + 1 < nk) store_b((kt + 1) & 1);
    __syncthreads();
    if (kt + 2 < nk) load_b(kt + 2);
  };

  if (nk > 0) {
    load_a(a0, 0);
    load_b(0);
    store_b(0);
    if (nk > 1) {
      load_a(a1, 1);
      load_b(1);
    }
  }
  __syncthreads();
  // three left-operand register sets rotate: slices kt, kt+1 in flight, kt+2 loading
  int kt = 0;
  for (; kt + 3 <= nk; kt += 3) {
    step(kt, a0, a2);
    step(kt + 1, a1, a0);
    step(kt + 2, a2, a1);
  }
  if (kt < nk) step(kt, a0, a2);
  if (kt + 1 < nk) step(kt + 1, a1, a0);

  // output element r of tile (i, j): row 8 (r / 4) + 4 h + r % 4, column l32
  if (c.splits == 1) {
    const Epilogue<float> e = args.epi;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t n = n0 + wn * 32 * TN + j * 32 + l32;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t m = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
          args.C[m + n * c.ldc] = apply_epilogue(e, acc[i][j][r], m, n);
        }
      }
  } else {
    float* P = args.partial + int64_t(split) * c.M * c.N;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t n = n0 + wn * 32 * TN + j * 32 + l32;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int64_t m = m0 + wm * 64 + i * 32 + 8 * g + 4 * h;
          *reinterpret_cast<f32x4*>(P + m + n * c.M) =
              f32x4{acc[i][j][4 * g], acc[i][j][4 * g + 1], acc[i][j][4 * g + 2],
                    acc[i][j][4 * g + 3]};
        }
      }
  }
}

// B16 (n x b, ld ldo) = bfloat16(kscale .* B) (nearest-even); grid x over
// 1024-row chunks (4 rows per thread when n % 4 == 0 and the pointers and
// leading dimensions allow 16-byte loads), y over columns
template <bool VEC>
__global__ __launch_bounds__(256) void k_scale_bf16(const float* __restrict__ B, int64_t ldb,
                                                    const float* __restrict__ ks, int64_t n,
                                                    int64_t b, unsigned short* __restrict__ out,
                                                    int64_t ldo) {
  const int64_t i0 = (int64_t(blockIdx.x) * 256 + threadIdx.x) * 4;
  if (i0 >= n) return;
  for (int64_t j = blockIdx.y; j < b; j += gridDim.y) {
    if constexpr (VEC) {
      f32x4 v = *reinterpret_cast<const f32x4*>(B + i0 + j * ldb);
      if (ks) v *= *reinterpret_cast<const f32x4*>(ks + i0);
      const uint32_t lo = uint32_t(f32_to_bf16_rne(v[0])) | (uint32_t(f32_to_bf16_rne(v[1])) << 16);
      const uint32_t hi = uint32_t(f32_to_bf16_rne(v[2])) | (uint32_t(f32_to_bf16_rne(v[3])) << 16);
      *reinterpret_cast<uint2*>(out + i0 + j * ldo) = make_uint2(lo, hi);
    } else {
      for (int64_t i = i0; i < std::min<int64_t>(n, i0 + 4); ++i)
        out[i + j * ldo] = f32_to_bf16_rne(B[i + j * ldb] * (ks ? ks[i] : 1.f));
    }
  }
}

// Split-K factor (after rounding the k-range to whole 64-deep slices) and
// k-range length of the BF16 product: enough work items for ~4 per CU,
// at least 8 slices per split, at most 16 splits.
// The 32 x 32 x 16 kernel (WIDE) runs one workgroup per CU: splits until the
// work items reach the CU count.
template <int BM, int BN, bool WIDE = false>
static int bf16_splits(int64_t M, int64_t N, int64_t K, int force_splits, int64_t* kchunk_out) {
  constexpr int BK = 64;
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  int splits = force_splits;
  if (splits <= 0) {
    splits = 1;
    const int64_t max_s = std::max<int64_t>(1, K / (8 * BK));
    const int64_t target = int64_t(kNumCU) * (WIDE ? 1 : 4);
    while (tiles * splits < target && splits * 2 <= max_s && splits < 16) splits *= 2;
  }
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + BK - 1) / BK * BK;
  if (kchunk == 0) kchunk = BK;
  splits = int((K + kchunk - 1) / kchunk);
  *kchunk_out = kchunk;
  return std::max(splits, 1);
}

template <int BM, int BN, bool WIDE = false>
static hipError_t gemm_bf16_launch(const GemmDesc<float>& d, const uint16_t* A16, int64_t lda16,
                                   uint16_t* B16, hipStream_t st, const Workspace& ws,
                                   int force_splits, bool b16_ready, uint16_t* next16,
                                   const float* next_scale, bool* next_ready) {
  constexpr int BK = 64;
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  if (d.sbk != 1 || d.batch != 1 || !A16 || !B16) return hipErrorInvalidValue;
  hipError_t err;
  // (the profiling interval covers the rounding pass and the product)
  if (d.ev_begin && (err = hipEventRecord(d.ev_begin, st)) != hipSuccess) return err;
  // the product's right operand in bfloat16, D^{-1} applied (ld = K), unless
  // the previous step's reduction already wrote it
  if (!b16_ready) {
    const dim3 grid(unsigned(((d.K + 3) / 4 + 255) / 256), unsigned(std::min<int64_t>(d.N, 65535)));
    auto al = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
    const bool vec = d.K % 4 == 0 && d.sbn % 4 == 0 && al(d.B) && al(B16) &&
                     (!d.kscale || al(d.kscale));
    if (vec)
      k_scale_bf16<true><<<grid, dim3(256), 0, st>>>(
          d.B, d.sbn, d.kscale, d.K, d.N, reinterpret_cast<unsigned short*>(B16), d.K);
    else
      k_scale_bf16<false><<<grid, dim3(256), 0, st>>>(
          d.B, d.sbn, d.kscale, d.K, d.N, reinterpret_cast<unsigned short*>(B16), d.K);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
  }
  KernelArgs<float> a;
  KernelArgsCommon& c = a.c;
  c.M = d.M;
  c.N = d.N;
  c.K = d.K;
  c.sam = lda16;
  c.sak = 1;
  c.sbk = 1;
  c.sbn = d.K;
  c.ldc = d.ldc;
  c.batch = 1;
  c.bsA = c.bsB = c.bsC = c.bsC1 = 0;
  c.lower = 0;
  c.tiles_m = int((d.M + BM - 1) / BM);
  c.tiles_n = int((d.N + BN - 1) / BN);
  const int64_t tiles = int64_t(c.tiles_m) * c.tiles_n;
  int64_t kchunk = 0;
  const int splits = bf16_splits<BM, BN, WIDE>(d.M, d.N, d.K, force_splits, &kchunk);
  c.kchunk = kchunk;
  c.splits = splits;
  a.A = nullptr;
  a.B = nullptr;
  a.kscale = nullptr;
  a.C = d.C;
  a.epi = d.epi;
  a.partial = nullptr;
  if (c.splits > 1) {
    const size_t need = size_t(c.splits) * d.M * d.N * sizeof(float);
    if (need > ws.bytes || ws.ptr == nullptr) {
      c.splits = 1;
      c.kchunk = (d.K + BK - 1) / BK * BK;
    } else {
      a.partial = static_cast<float*>(ws.ptr);
    }
  }
  const int64_t grid = tiles * c.splits;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  const bool aligned = d.M % BM == 0 && d.N % BN == 0 && d.K % BK == 0 && c.kchunk % BK == 0 &&
                       reinterpret_cast<uintptr_t>(A16) % 16 == 0 && lda16 % 8 == 0 &&
                       reinterpret_cast<uintptr_t>(B16) % 16 == 0;
  const unsigned short* a16 = reinterpret_cast<const unsigned short*>(A16);
  const unsigned short* b16 = reinterpret_cast<const unsigned short*>(B16);
  if constexpr (WIDE) {
    static_assert(BM == 128 && BN % 64 == 0, "wide tile shape");
    if (!aligned) return hipErrorInvalidValue;
    gemm_bf16_wide_kernel<BN / 64><<<dim3(unsigned(grid)), dim3(256), 0, st>>>(a, a16, b16);
  } else if (aligned) {
    gemm_bf16_kernel<BM, BN, BK, false><<<dim3(unsigned(grid)), dim3(256), 0, st>>>(a, a16, b16);
  } else {
    gemm_bf16_kernel<BM, BN, BK, true><<<dim3(unsigned(grid)), dim3(256), 0, st>>>(a, a16, b16);
  }
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if (next_ready) *next_ready = false;
  if (c.splits > 1) {
    const int64_t total = d.M * d.N;
    if (reduce4_ok(a, 1)) {
      // the next step's right operand, rounded here from the values just formed
      auto al = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
      if (next16 && al(next16) && (!next_scale || al(next_scale))) {
        a.out16 = reinterpret_cast<unsigned short*>(next16);
        a.scale16 = next_scale;
        if (next_ready) *next_ready = true;
      }
      splitk_reduce4_kernel<<<reduce4_grid(d.M, d.N), dim3(256), 0, st>>>(a);
    } else {
      const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
      splitk_reduce_kernel<float><<<dim3(blocks), dim3(256), 0, st>>>(a);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  // the profiling interval ends after the reduction, which carries the epilogue
  if (d.ev_end && (err = hipEventRecord(d.ev_end, st)) != hipSuccess) return err;
  return hipSuccess;
}

// tile shape of the BF16 product (knob CHFSI_BF16_TILE: 0 = 64x64, 1 = 64x160
// (default), 2 = 128x64).  Measured at 8192 x 320 x 8192 on MI355X: 0.093,
// 0.084 and 0.086 ms per product with split-K 4.
static int bf16_tile() {
  static const int tile = [] {
    const char* e = std::getenv("CHFSI_BF16_TILE");
    return e ? std::atoi(e) : 1;
  }();
  return tile;
}

// the 32 x 32 x 16 kernel for shapes it takes (knob CHFSI_BF16_WIDE=0: off)
static bool bf16_wide() {
  static const bool on = [] {
    const char* e = std::getenv("CHFSI_BF16_WIDE");
    return !(e && std::atoi(e) == 0);
  }();
  return on;
}

hipError_t gemm_bf16_filter(const GemmDesc<float>& d, const uint16_t* A16, int64_t lda16,
                            uint16_t* B16, hipStream_t st, const Workspace& ws,
                            int force_splits, bool b16_ready, uint16_t* next16,
                            const float* next_scale, bool* next_ready) {
  if (next_ready) *next_ready = false;
  // the fused rounding writes an M x N block with ld M into the K x N buffer
  if (next16 && d.M != d.K) next16 = nullptr;
  const bool wide_ok = bf16_wide() && d.sbk == 1 && d.batch == 1 && A16 && B16 &&
                       d.M % 128 == 0 && d.K % 64 == 0 && lda16 % 8 == 0 &&
                       reinterpret_cast<uintptr_t>(A16) % 16 == 0 &&
                       reinterpret_cast<uintptr_t>(B16) % 16 == 0;
  if (wide_ok && d.N % 320 == 0)
    return gemm_bf16_launch<128, 320, true>(d, A16, lda16, B16, st, ws, force_splits, b16_ready,
                                                   next16, next_scale, next_ready);
  if (wide_ok && d.N % 128 == 0)
    return gemm_bf16_launch<128, 128, true>(d, A16, lda16, B16, st, ws, force_splits, b16_ready,
                                                   next16, next_scale, next_ready);
  switch (bf16_tile()) {
    case 1: return gemm_bf16_launch<64, 160>(d, A16, lda16, B16, st, ws, force_splits, b16_ready,
                                                   next16, next_scale, next_ready);
    case 2: return gemm_bf16_launch<128, 64>(d, A16, lda16, B16, st, ws, force_splits, b16_ready,
                                                   next16, next_scale, next_ready);
    default: return gemm_bf16_launch<64, 64>(d, A16, lda16, B16, st, ws, force_splits, b16_ready,
                                                   next16, next_scale, next_ready);
  }
}

size_t gemm_bf16_workspace_bytes(int64_t M, int64_t N) {
  return size_t(16) * size_t(M) * size_t(N) * sizeof(float);
}

size_t gemm_bf16_plan_bytes(int64_t M, int64_t N, int64_t K, int force_splits) {
  int64_t kc = 0;
  int s;
  switch (bf16_tile()) {
    case 1: s = bf16_splits<64, 160>(M, N, K, force_splits, &kc); break;
    case 2: s = bf16_splits<128, 64>(M, N, K, force_splits, &kc); break;
    default: s = bf16_splits<64, 64>(M, N, K, force_splits, &kc); break;
  }
  return s > 1 ? size_t(s) * size_t(M) * size_t(N) * sizeof(float) : 0;
}

template hipError_t gemm<float>(const GemmDesc<float>&, hipStream_t, const Workspace&, int, int);
template hipError_t gemm<double>(const GemmDesc<double>&, hipStream_t, const Workspace&, int,
                                 int);
template void gemm_plan<float>(int64_t, int64_t, int64_t, int, int*, int*);
template void gemm_plan<double>(int64_t, int64_t, int64_t, int, int*, int*);

}  // namespace chfsi
