// Periodic 27-point grid operators for the sparse generalized problems
// (the finite-element setting of the paper's Section 4.2: a mass matrix B and
// a Hamiltonian A = 0.5 K + potential on a tensor-product grid, with the
// mass-lumped diagonal approximation D of B used only in the filter).
//
// An operator is S z + field term, where S is a 27-point stencil with
// arbitrary coefficients and the field term is diag(V) z (mode 1) or the
// mass-weighted 1/2 (diag(V) M + M diag(V)) z (mode 2).  Mode 2 is evaluated
// per neighbour as sum_o (c_o + m_o (V_r + V_{r+o})/2) z_{r+o}, with three
// accumulators (S z, M z, M (V z)).
//
// Blocks are column-major (grid index x + nx*(y + ny*z) fastest, then the
// column), so a wave covers 64 consecutive x points of one column and every
// neighbour row it reads is a contiguous, cache-line aligned run.
//
// Filter steps fuse the whole recurrence update (Algorithm 3 loop body, or
// Algorithm 2) into the operator kernel, so each step streams R_Y, R_X and the
// forcing block once: the HBM-bound form the method's reduced-precision
// storage is meant to speed up.
#include "stencil_api.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>

namespace chfsi {

namespace {

struct Coefs {
  float c[27];
  float m[27];
};
struct CoefsD {
  double c[27];
  double m[27];
};

struct Grid {
  int nx, ny, nz;
  int mode;
  const double* V;
};

inline int64_t grid_for(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g < 1) g = 1;
  return g > 262144 ? 262144 : g;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(uint32_t(h) << 16);
}

// round-to-nearest-even float -> bfloat16 (NaN stays NaN)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// Operator application at point r of one column.  `col` points at the
// column's first element.  Returns S z (+ field term), in accumulator type A.
template <typename A, typename CT, typename LoadF>
__device__ __forceinline__ A apply_point(const CT& cf, const Grid& g, int x, int y, int z,
                                         LoadF load) {
  A acc = A(0), accm = A(0), accv = A(0);
  const A Vr = (g.mode == 2) ? A(g.V[x + int64_t(g.nx) * (y + int64_t(g.ny) * z)]) : A(0);
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    int zz = z + dz;
    zz = zz < 0 ? zz + g.nz : (zz >= g.nz ? zz - g.nz : zz);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      int yy = y + dy;
      yy = yy < 0 ? yy + g.ny : (yy >= g.ny ? yy - g.ny : yy);
      const int64_t row = int64_t(g.nx) * (yy + int64_t(g.ny) * zz);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        int xx = x + dx;
        xx = xx < 0 ? xx + g.nx : (xx >= g.nx ? xx - g.nx : xx);
        const int o = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
        const A v = load(row + xx);
        acc += A(cf.c[o]) * v;
        if (g.mode == 2) {
          accm += A(cf.m[o]) * v;
          accv += A(cf.m[o]) * (A(g.V[row + xx]) * v);
        }
      }
    }
  }
  if (g.mode == 2) acc += A(0.5) * (Vr * accm + accv);
  if (g.mode == 1) acc += A(g.V[x + int64_t(g.nx) * (y + int64_t(g.ny) * z)]) * load(x + int64_t(g.nx) * (y + int64_t(g.ny) * z));
  return acc;
}

__global__ __launch_bounds__(256) void k_apply_f64(CoefsD cf, Grid g, const double* X, int64_t ldx,
                                                   double* Y, int64_t ldy, int64_t n, int64_t b) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t j = idx / n, i = idx - j * n;
    const int x = int(i % g.nx), y = int((i / g.nx) % g.ny), z = int(i / (int64_t(g.nx) * g.ny));
    const double* col = X + j * ldx;
    Y[i + j * ldy] = apply_point<double>(cf, g, x, y, z, [&](int64_t k) { return col[k]; });
  }
}

__global__ __launch_bounds__(256) void k_rstep_f64(CoefsD cf, Grid g, const double* dinv,
                                                   const double* RY, double* RX, const double* Yf,
                                                   int64_t ldf, const double* colcoef,
                                                   StencilStep s, int64_t n, int64_t b) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t j = idx / n, i = idx - j * n;
    const int x = int(i % g.nx), y = int((i / g.nx) % g.ny), z = int(i / (int64_t(g.nx) * g.ny));
    const double* col = RY + j * n;
    const double av = apply_point<double>(cf, g, x, y, z, [&](int64_t k) {
      return dinv ? dinv[k] * col[k] : col[k];
    });
    const int64_t e = i + j * n;
    RX[e] = s.alpha * av + s.beta * RY[e] + s.gamma * RX[e] + s.delta * colcoef[j] * Yf[i + j * ldf];
  }
}

__global__ __launch_bounds__(256) void k_rstep_f32(Coefs cf, Grid g, const float* dinv,
                                                   const float* RY, float* RX, const float* Yf,
                                                   const float* colcoef, float a, float bb,
                                                   float cc, float dd, int64_t n, int64_t b) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t j = idx / n, i = idx - j * n;
    const int x = int(i % g.nx), y = int((i / g.nx) % g.ny), z = int(i / (int64_t(g.nx) * g.ny));
    const float* col = RY + j * n;
    const float av = apply_point<float>(cf, g, x, y, z,
                                        [&](int64_t k) { return dinv ? dinv[k] * col[k] : col[k]; });
    const int64_t e = i + j * n;
    RX[e] = a * av + bb * RY[e] + cc * RX[e] + dd * colcoef[j] * Yf[e];
  }
}

__global__ __launch_bounds__(256) void k_rstep_bf16(Coefs cf, Grid g, const float* dinv,
                                                    const uint16_t* RY, uint16_t* RX,
                                                    const uint16_t* Yf, const float* colcoef,
                                                    float a, float bb, float cc, float dd,
                                                    int64_t n, int64_t b) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t j = idx / n, i = idx - j * n;
    const int x = int(i % g.nx), y = int((i / g.nx) % g.ny), z = int(i / (int64_t(g.nx) * g.ny));
    const uint16_t* col = RY + j * n;
    const float av = apply_point<float>(cf, g, x, y, z,
                                        [&](int64_t k) {
                                          const float u = bf16_to_f32(col[k]);
                                          return dinv ? dinv[k] * u : u;
                                        });
    const int64_t e = i + j * n;
    const float v = a * av + bb * bf16_to_f32(RY[e]) + cc * bf16_to_f32(RX[e]) +
                    dd * colcoef[j] * bf16_to_f32(Yf[e]);
    RX[e] = f32_to_bf16(v);
  }
}

__global__ __launch_bounds__(256) void k_cstep_f64(CoefsD cf, Grid g, const double* dinv,
                                                   const double* src, int64_t lds,
                                                   const double* prev, int64_t ldp, double* dst,
                                                   StencilStep s, int64_t n, int64_t b) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t j = idx / n, i = idx - j * n;
    const int x = int(i % g.nx), y = int((i / g.nx) % g.ny), z = int(i / (int64_t(g.nx) * g.ny));
    const double* col = src + j * lds;
    double av = apply_point<double>(cf, g, x, y, z, [&](int64_t k) { return col[k]; });
    if (dinv) av *= dinv[i];
    double v = s.alpha * av + s.beta * col[i];
    if (prev) v += s.gamma * prev[i + j * ldp];
    dst[i + j * n] = v;
  }
}

__global__ __launch_bounds__(256) void k_init_bf16(const double* R, int64_t ldr, int64_t n,
                                                   int64_t b, double scale, uint16_t* RY,
                                                   uint16_t* RX, uint16_t* Yc) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t j = idx / n, i = idx - j * n;
    const double r = R[i + j * ldr];
    RY[idx] = f32_to_bf16(float(scale * r));
    RX[idx] = 0;
    Yc[idx] = f32_to_bf16(float(r));
  }
}

__global__ __launch_bounds__(256) void k_recon_bf16(const uint16_t* RY, const double* dinv,
                                                    const double* X, int64_t ldx,
                                                    const double* lamY, double* Yp, int64_t ldy,
                                                    int64_t n, int64_t b) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(256) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int64_t j = idx / n, i = idx - j * n;
    double r = double(bf16_to_f32(RY[idx]));
    if (dinv) r *= dinv[i];
    Yp[i + j * ldy] = r + X[i + j * ldx] * lamY[j];
  }
}

// ---------------------------------------------------------------------------
// Separable (class-symmetric) 27-point kernels, z-marching.
//
// The tensor-product Q1 stiffness and mass stencils have one coefficient per
// class of offsets (0: centre, 1: the 6 faces, 2: the 12 edges, 3: the 8
// corners).  Their class sums follow from per-plane partial sums
//   P0 = u(x,y),  P1 = u(x±1,y) + u(x,y±1),  P2 = u(x±1,y±1)   (in-plane)
// combined across z:
//   s0 = P0(z),               s1 = P1(z) + P0(z-1) + P0(z+1),
//   s2 = P2(z) + P1(z±1),      s3 = P2(z-1) + P2(z+1).
// A workgroup owns one column and a slab of TY full x-rows and walks the whole
// periodic z range; each plane (with its two halo rows) is staged once in LDS,
// every thread keeps the partials of its points for planes z-1, z, z+1 in
// registers, so an element costs 8 LDS reads per operand (u, and V*u for the
// mass-weighted potential) instead of 27.
// ---------------------------------------------------------------------------
enum StencilKind { SK_APPLY = 0, SK_RSTEP = 1, SK_CSTEP = 2, SK_RESID = 3 };

template <typename S>
__device__ __forceinline__ float ld_f(const S* p, int64_t i);
template <>
__device__ __forceinline__ float ld_f<float>(const float* p, int64_t i) {
  return p[i];
}
template <>
__device__ __forceinline__ float ld_f<uint16_t>(const uint16_t* p, int64_t i) {
  return bf16_to_f32(p[i]);
}
template <typename S, typename F>
__device__ __forceinline__ F ld_s(const S* p, int64_t i) {
  if constexpr (sizeof(S) == 2)
    return F(bf16_to_f32(reinterpret_cast<const uint16_t*>(p)[i]));
  else
    return F(p[i]);
}
template <typename S, typename F>
__device__ __forceinline__ void st_s(S* p, int64_t i, F v) {
  if constexpr (sizeof(S) == 2)
    reinterpret_cast<uint16_t*>(p)[i] = f32_to_bf16(float(v));
  else
    p[i] = S(v);
}

template <typename F>
struct SepArgs {
  int nx, ny, nz, ty, ntiles_y;
  int z0, nzs;               // output planes [z0, z0 + nzs)
  int64_t out_off;           // output row index = grid index - out_off
  int mode;                  // field mode
  F cA[4], cM[4];            // class coefficients of S and of the mass stencil
  F cB[4];                   // SK_RESID: class coefficients of B (b_identity: B = I)
  int b_identity;
  const double* V;
  const void* dinv;          // length n, F-typed (FP32 for FP32/BF16 storage, FP64 for FP64)
  const void* src;           // operand block (APPLY: X, RSTEP: R_Y, CSTEP: src)
  int64_t lds_src;
  void* out;                 // APPLY: Y, RSTEP: R_X (in place), CSTEP: dst
  int64_t ld_out;
  const void* prev;          // CSTEP: previous iterate (may alias out)
  int64_t ld_prev;
  const void* forcing;       // RSTEP: Y copy
  int64_t ld_forcing;
  const F* colcoef;          // RSTEP: Lambda_Y per column
  F alpha, beta, gamma, delta;
};

// points per thread per plane: 4 for FP32 arithmetic, 2 for FP64
template <typename F>
constexpr int sep_pt() { return sizeof(F) == 4 ? 4 : 2; }

template <typename S, typename F, int KIND>
__global__ __launch_bounds__(256) void k_stencil_sep(SepArgs<F> a) {
  constexpr int SEP_MAXPT = sep_pt<F>();
  extern __shared__ __attribute__((aligned(16))) unsigned char sep_smem[];
  F* lds = reinterpret_cast<F*>(sep_smem);
  const int nx = a.nx, ny = a.ny, nz = a.nz, TY = a.ty;
  const int rows = TY + 2;
  const int plane_sz = rows * nx;            // one operand plane incl. halo rows
  const int64_t n = int64_t(nx) * ny * nz;
  const int j = blockIdx.x / a.ntiles_y;      // column
  const int ytile = blockIdx.x - j * a.ntiles_y;
  const int y0 = ytile * TY;
  const int npts = nx * min(TY, ny - y0);     // points of this slab per plane
  const bool field2 = a.mode == 2;
  const S* src = static_cast<const S*>(a.src) + int64_t(j) * a.lds_src;
  const F* dinv = static_cast<const F*>(a.dinv);

  // LDS: buffer b (0/1) holds u at [b*2*plane_sz] and w = V*u at +plane_sz
  auto stage = [&](int buf, int z) {
    F* u = lds + buf * 2 * plane_sz;
    F* w = u + plane_sz;
    const int64_t zoff = int64_t(z) * nx * ny;
    for (int idx = threadIdx.x; idx < plane_sz; idx += 256) {
      const int r = idx / nx, x = idx - r * nx;
      int y = y0 - 1 + r;
      y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
      const int64_t i = zoff + int64_t(y) * nx + x;
      F v = ld_s<S, F>(src, i);
      if (KIND == SK_RSTEP && dinv) v *= dinv[i];
      u[idx] = v;
      if (field2) w[idx] = F(a.V[i]) * v;
    }
  };

  // per-point partial sums for planes z-1 (0), z (1), z+1 (2)
  F pu[3][SEP_MAXPT][3], pw[3][SEP_MAXPT][3];
  auto partials = [&](int buf, F (&P)[SEP_MAXPT][3], F (&Q)[SEP_MAXPT][3]) {
    const F* u = lds + buf * 2 * plane_sz;
    const F* w = u + plane_sz;
#pragma unroll
    for (int q = 0; q < SEP_MAXPT; ++q) {
      const int pt = threadIdx.x + q * 256;
      if (pt >= npts) break;
      const int yy = pt / nx, x = pt - yy * nx;
      const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
      const int rc = (yy + 1) * nx, rm = yy * nx, rp = (yy + 2) * nx;
      P[q][0] = u[rc + x];
      P[q][1] = u[rc + xm] + u[rc + xp] + u[rm + x] + u[rp + x];
      P[q][2] = u[rm + xm] + u[rm + xp] + u[rp + xm] + u[rp + xp];
      if (field2) {
        Q[q][0] = w[rc + x];
        Q[q][1] = w[rc + xm] + w[rc + xp] + w[rm + x] + w[rp + x];
        Q[q][2] = w[rm + xm] + w[rm + xp] + w[rp + xm] + w[rp + xp];
      }
    }
  };

  const int zb = a.z0, ze = a.z0 + a.nzs;
  stage(0, zb == 0 ? nz - 1 : zb - 1);
  stage(1, zb);
  __syncthreads();
  partials(0, pu[0], pw[0]);
  partials(1, pu[1], pw[1]);
  __syncthreads();
  for (int z = zb; z < ze; ++z) {
    const int buf = (z - zb) & 1;            // plane z+1 goes to the buffer of z-1
    stage(buf, z + 1 < nz ? z + 1 : 0);
    __syncthreads();
    partials(buf, pu[2], pw[2]);
    const int64_t zoff = int64_t(z) * nx * ny + int64_t(y0) * nx;
#pragma unroll
    for (int q = 0; q < SEP_MAXPT; ++q) {
      const int pt = threadIdx.x + q * 256;
      if (pt >= npts) break;
      const F s0 = pu[1][q][0];
      const F s1 = pu[1][q][1] + pu[0][q][0] + pu[2][q][0];
      const F s2 = pu[1][q][2] + pu[0][q][1] + pu[2][q][1];
      const F s3 = pu[0][q][2] + pu[2][q][2];
      F av = a.cA[0] * s0 + a.cA[1] * s1 + a.cA[2] * s2 + a.cA[3] * s3;
      const int64_t i = zoff + pt;           // grid index of this point
      if (a.mode == 1) av += F(a.V[i]) * s0;
      if (field2) {
        const F t0 = pw[1][q][0];
        const F t1 = pw[1][q][1] + pw[0][q][0] + pw[2][q][0];
        const F t2 = pw[1][q][2] + pw[0][q][1] + pw[2][q][1];
        const F t3 = pw[0][q][2] + pw[2][q][2];
        const F mu = a.cM[0] * s0 + a.cM[1] * s1 + a.cM[2] * s2 + a.cM[3] * s3;
        const F mw = a.cM[0] * t0 + a.cM[1] * t1 + a.cM[2] * t2 + a.cM[3] * t3;
        av += F(0.5) * (F(a.V[i]) * mu + mw);
      }
      if constexpr (KIND == SK_APPLY) {
        st_s<S, F>(static_cast<S*>(a.out) + int64_t(j) * a.ld_out, i - a.out_off, av);
      } else if constexpr (KIND == SK_RESID) {
        // r = A x - lambda_j B x from the same class sums
        const F bx = a.b_identity ? s0 : a.cB[0] * s0 + a.cB[1] * s1 + a.cB[2] * s2 + a.cB[3] * s3;
        st_s<S, F>(static_cast<S*>(a.out) + int64_t(j) * a.ld_out, i - a.out_off,
                   av - a.colcoef[j] * bx);
      } else if constexpr (KIND == SK_RSTEP) {
        S* RX = static_cast<S*>(a.out) + int64_t(j) * a.ld_out;
        const S* Yf = static_cast<const S*>(a.forcing) + int64_t(j) * a.ld_forcing;
        const F v = a.alpha * av + a.beta * ld_s<S, F>(src, i) + a.gamma * ld_s<S, F>(RX, i) +
                    a.delta * a.colcoef[j] * ld_s<S, F>(Yf, i);
        st_s<S, F>(RX, i, v);
      } else {
        if (dinv) av *= dinv[i];
        F v = a.alpha * av + a.beta * ld_s<S, F>(src, i);
        if (a.prev)
          v += a.gamma * ld_s<S, F>(static_cast<const S*>(a.prev) + int64_t(j) * a.ld_prev, i);
        st_s<S, F>(static_cast<S*>(a.out) + int64_t(j) * a.ld_out, i, v);
      }
    }
    // roll the partials: z-1 <- z, z <- z+1
#pragma unroll
    for (int q = 0; q < SEP_MAXPT; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        pu[0][q][c] = pu[1][q][c];
        pu[1][q][c] = pu[2][q][c];
        pw[0][q][c] = pw[1][q][c];
        pw[1][q][c] = pw[2][q][c];
      }
    __syncthreads();
  }
  (void)n;
}

// ---------------------------------------------------------------------------
// Vectorised, software-pipelined z-marching kernel (class-symmetric
// coefficients, no diagonal scaling of the operand).
//
// Every plane p contributes to the outputs of planes p-1, p and p+1 through
// two class combinations of its in-plane partial sums P0, P1, P2:
//   centre     C = c0 P0 + c1 P1 + c2 P2      (p is the output plane)
//   neighbour  N = c1 P0 + c2 P1 + c3 P2      (p is one plane above or below)
// so out(z) = N(z-1) + C(z) + N(z+1) needs two running sums per operator and
// point.  Two such operators are carried: K (the stencil on u plus the
// stencil on w = V u) and M (the mass stencil on u, multiplied by V at the
// output point), which together give the mass-weighted potential
// 1/2 (diag(V) M + M diag(V)) u; the diagonal potential is M = identity.
// Linear terms of the step (beta * src, -lambda_j * B u) fold into the
// coefficients, so one pass gives every kind of update:
//   out = K + V * M + gamma * e1 + delta * colcoef[j] * e2.
//
// A workgroup owns CP columns, a slab of TY full x rows and a range of z
// planes.  Thread t owns PT consecutive x points of one slab row in all CP
// columns.  Each plane (the CP operand columns and, with the mass-weighted
// potential, w = V u of each, with one halo row on each side; the periodic x
// neighbours are read across the row) is staged into one of two LDS buffers from registers loaded
// one plane ahead; w is formed once per staged element, not once per use.  A
// single barrier per plane separates the writes from the reads, and the
// global loads of plane z+2 and of the epilogue operands of z+1 are in flight
// while plane z+1 is processed.  Workgroup ids are remapped so that the y-tiles of one column
// group (order 0), or the column groups of one y-tile (order 1), run on the
// same XCD, where the rows they share hit that XCD's L2.
// ---------------------------------------------------------------------------
// ZM_STEP: residual-filter step, e1 and e2 both present; ZM_CSTEP: plain
// Chebyshev step, e1 optional, no e2; ZM_BSTEP: ZM_STEP plus a precomputed
// correction at the grid's boundary points (Bloch-phase operators in the
// twisted frame: corr holds, per column, one value per boundary point in the
// enumeration of bloch.hip -- both z faces, the y = 0 / ny-1 rows of the
// inner planes, the x = 0 / nx-1 points of the inner rows).
enum ZmKind { ZM_APPLY = 0, ZM_RESID = 1, ZM_STEP = 2, ZM_CSTEP = 3, ZM_BSTEP = 4 };

template <typename F>
struct ZmArgs {
  int nx, ny, nz, ty, ntiles_y, b;
  int order;                 // workgroup -> tile order (see k_zmarch)
  int z0, nzs;               // output planes [z0, z0 + nzs)
  int use_w;                 // the stencil on w = V u is present (cw != 0)
  int64_t out_off;           // output row index = grid index - out_off
  F cu[4], cw[4], cm[4];     // class coefficients on u, on w = V u, and of M
  F cb[4];                   // ZM_RESID: B class coefficients (scaled by -lambda_j)
  const F* V;                // potential (has_v)
  const void* src;
  int64_t ld_src;
  void* out;
  int64_t ld_out;
  const void* e1;            // ZM_STEP / ZM_CSTEP: first extra stream (may alias out)
  int64_t ld_e1;
  F gamma;
  const void* e2;            // ZM_STEP: second extra stream, scaled per column
  int64_t ld_e2;
  F delta;
  const F* colcoef;          // ZM_STEP: per-column factor of e2; ZM_RESID: lambda_j
  const F* corr;             // ZM_BSTEP: boundary correction, column-major, ld ld_corr
  int64_t ld_corr;
  void* edge_out;            // ZM_BSTEP (may be null): the output's x = 0 and x = nx-1
                             // values, ((z ny + y) 2 + (x == nx-1)) per column, ld 2 ny nz
};

template <typename S, typename F, int PT>
__device__ __forceinline__ void zm_cvt(const S __attribute__((ext_vector_type(PT))) & v,
                                       F (&o)[PT]) {
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    if constexpr (sizeof(S) == 2)
      o[i] = F(__uint_as_float(uint32_t(v[i]) << 16));
    else
      o[i] = F(v[i]);
  }
}

// storage element of an output value (bfloat16: round to nearest even, by the
// hardware conversion)
template <typename S, typename F>
__device__ __forceinline__ S zm_store_elem(F v) {
  if constexpr (sizeof(S) == 2)
    return __builtin_bit_cast(uint16_t, static_cast<__bf16>(float(v)));
  else
    return S(v);
}

template <typename T>
__device__ __forceinline__ const T* zm_byte_off(const T* p, uint32_t bytes) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + bytes);
}

template <typename S, typename F, int PT, int CP, int NG, int KIND, bool HASV>
// (the BF16 Bloch step is held to 96 VGPRs, five waves per SIMD like the
// plain step; unconstrained it takes 97 and drops to four)
__global__ __launch_bounds__(256 * NG)
__attribute__((amdgpu_waves_per_eu(KIND == ZM_BSTEP && sizeof(S) == 2 ? 5 : 1)))
void k_zmarch(ZmArgs<F> a) {
  using SV = S __attribute__((ext_vector_type(PT)));
  using FV = F __attribute__((ext_vector_type(PT)));
  extern __shared__ __attribute__((aligned(16))) unsigned char zm_smem[];
  F* lds = reinterpret_cast<F*>(zm_smem);
  const int nx = a.nx, ny = a.ny, nz = a.nz, TY = a.ty;
  const int RS = nx + 8;                     // LDS row: [4..4+nx) = the grid row (16-byte aligned)
  const int plane = (TY + 2) * RS;
  // planes per buffer: u of every column slot, then (potential) w of every slot
  constexpr int NC = NG * CP;
  constexpr int NOPS = HASV ? 2 * NC : NC;
  constexpr bool ONE_COL = NG == 1 && CP == 1;   // every launched workgroup owns its column
  const int bufsz = NOPS * plane;
  const bool use_w = HASV && a.use_w != 0;

  // XCD-aware tile order: consecutive ids on one XCD take consecutive tiles
  const int nb = gridDim.x, bid = blockIdx.x;
  const int q8 = nb >> 3, r8 = nb & 7, xcd = bid & 7, loc = bid >> 3;
  const int t = xcd < r8 ? xcd * (q8 + 1) + loc : r8 * (q8 + 1) + (xcd - r8) * q8 + loc;
  // order 0: a column group's y-tiles are consecutive (they share halo rows);
  // order 1: the column groups of one y-tile are consecutive (they share the
  // potential's planes, which are 2 x the BF16 operand bytes)
  int cg, ytile;
  if (a.order == 0) {
    cg = t / a.ntiles_y;
    ytile = t - cg * a.ntiles_y;
  } else {
    const int ncg = nb / a.ntiles_y;
    ytile = t / ncg;
    cg = t - ytile * ncg;
  }
  const int y0 = ytile * TY, tyn = min(TY, ny - y0);
  // group g (256 threads) owns columns col0 .. col0 + ncol - 1
  const int g = NG == 1 ? 0 : int(threadIdx.x >> 8);
  const int col0 = (cg * NG + g) * CP;
  const int ncol = ONE_COL ? 1 : min(CP, a.b - col0);
  const int64_t pstride = int64_t(nx) * ny;

  const int tpr = nx / PT;
  const int tid = threadIdx.x & 255;
  const int my_row = tid / tpr, xq = (tid - my_row * tpr) * PT;
  const bool active = my_row < tyn && ncol > 0;

  // staging chunks: PT consecutive elements of one of the tyn+2 slab rows
  // (byte offsets within a plane: operand and potential element sizes).
  // Chunk 0 of a thread is its own output points (slab row my_row + 1), so the
  // potential it stages there is the one its output needs; chunk 1 covers the
  // halo rows 0 and tyn + 1 (threads below 2 * tpr).  Together they cover the
  // (tyn + 2) * tpr chunks once: tyn * tpr <= 256 and tpr <= 128.
  const int nchunk = (tyn + 2) * tpr;
  uint32_t boff_s[2], boff_f[2];
  int l_off[2];
  bool okc[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int k = m == 0 ? tid + tpr : (tid < tpr ? tid : tid + 256);
    okc[m] = k < nchunk;
    const int rr = okc[m] ? k / tpr : 0;
    const int xx = (k - rr * tpr) * PT;
    int y = y0 - 1 + rr;
    y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
    boff_s[m] = uint32_t(y * nx + xx) * uint32_t(sizeof(S));
    boff_f[m] = uint32_t(y * nx + xx) * uint32_t(sizeof(F));
    l_off[m] = rr * RS + 4 + xx;
  }
  // this thread's points and their periodic x neighbours within an LDS row
  const int x_mid = 4 + xq;
  const int x_lo = 4 + (xq == 0 ? nx - 1 : xq - 1);
  const int x_hi = 4 + (xq + PT == nx ? 0 : xq + PT);

  // Column base pointers are uniform within a group; every per-lane offset is
  // a 32-bit byte count added to a uniform plane offset (the host keeps a
  // column below 2^31 bytes), so the loads address base + 32-bit offset.
  const S* srcc[CP];
#pragma unroll
  for (int c = 0; c < CP; ++c)
    srcc[c] = static_cast<const S*>(a.src) + int64_t(col0 + c) * a.ld_src;
  const uint32_t own_b = uint32_t((y0 + my_row) * nx + xq) * uint32_t(sizeof(S));
  struct Staged {
    SV us[2][CP];
    FV vs[2];
  };
  auto load_plane = [&](int zp, Staged& R) __attribute__((always_inline)) {
    const uint32_t zo = uint32_t(zp) * uint32_t(pstride);
    const uint32_t zs = zo * uint32_t(sizeof(S)), zf = zo * uint32_t(sizeof(F));
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (!okc[m]) continue;
#pragma unroll
      for (int c = 0; c < CP; ++c)
        if (ONE_COL || c < ncol)
          R.us[m][c] = *reinterpret_cast<const SV*>(zm_byte_off(srcc[c], zs + boff_s[m]));
      if constexpr (HASV)
        if (m == 0 || use_w)
          R.vs[m] = *reinterpret_cast<const FV*>(zm_byte_off(a.V, zf + boff_f[m]));
    }
  };
  auto put = [&](F* pl, int m, const F (&v)[PT]) __attribute__((always_inline)) {
    FV w;
#pragma unroll
    for (int i = 0; i < PT; ++i) w[i] = v[i];
    *reinterpret_cast<FV*>(pl + l_off[m]) = w;
  };
  auto write_plane = [&](int buf, const Staged& R) __attribute__((always_inline)) {
    F* base = lds + buf * bufsz;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (!okc[m]) continue;
#pragma unroll
      for (int c = 0; c < CP; ++c) {
        F v[PT];
        if (ONE_COL || c < ncol) {
          zm_cvt<S, F, PT>(R.us[m][c], v);
        } else {
#pragma unroll
          for (int i = 0; i < PT; ++i) v[i] = F(0);
        }
        put(base + (g * CP + c) * plane, m, v);
        if constexpr (HASV) {
          if (use_w) {
            F w[PT];
#pragma unroll
            for (int i = 0; i < PT; ++i) w[i] = R.vs[m][i] * v[i];
            put(base + (NC + g * CP + c) * plane, m, w);
          }
        }
      }
    }
  };

  // per-column coefficients on u (RESID subtracts lambda_j times B's) and the
  // step's per-column factor of e2
  constexpr bool STEPK = KIND == ZM_STEP || KIND == ZM_BSTEP;
  F cu[CP][4], dcol[CP];
#pragma unroll
  for (int c = 0; c < CP; ++c) {
    const bool have = ONE_COL || c < ncol;
    const F lam = (KIND == ZM_RESID && have) ? a.colcoef[col0 + c] : F(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) cu[c][k] = KIND == ZM_RESID ? a.cu[k] - lam * a.cb[k] : a.cu[k];
    dcol[c] = (STEPK && have) ? a.delta * a.colcoef[col0 + c] : F(0);
  }

  // three rows x (PT + 2) values around this thread's points in one staged
  // plane (p: row y-1 of this thread's slab row)
  auto rows = [&](const F* p, F (&seg)[3][PT + 2]) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const FV mid = *reinterpret_cast<const FV*>(p + r * RS + x_mid);
      seg[r][0] = p[r * RS + x_lo];
#pragma unroll
      for (int i = 0; i < PT; ++i) seg[r][i + 1] = mid[i];
      seg[r][PT + 1] = p[r * RS + x_hi];
    }
  };
  // in-plane class sums: centre, the 4 face neighbours, the 4 corners
  auto sums = [&](const F (&s)[3][PT + 2], F (&p0)[PT], F (&p1)[PT], F (&p2)[PT])
      __attribute__((always_inline)) {
    F vs[PT + 2];
#pragma unroll
    for (int k = 0; k < PT + 2; ++k) vs[k] = s[0][k] + s[2][k];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      p0[i] = s[1][i + 1];
      p1[i] = s[1][i] + s[1][i + 2] + vs[i + 1];
      p2[i] = vs[i] + vs[i + 2];
    }
  };
  // centre and neighbour combinations of column c in one staged plane
  auto combos = [&](int buf, int c, F (&ck)[PT], F (&nk)[PT], F (&cmv)[PT], F (&nmv)[PT])
      __attribute__((always_inline)) {
    const int off = my_row * RS;               // row y-1 of this thread's points
    {
      F seg[3][PT + 2], p0[PT], p1[PT], p2[PT];
      rows(lds + buf * bufsz + (g * CP + c) * plane + off, seg);
      sums(seg, p0, p1, p2);
#pragma unroll
      for (int i = 0; i < PT; ++i) {
        ck[i] = cu[c][0] * p0[i] + cu[c][1] * p1[i] + cu[c][2] * p2[i];
        nk[i] = cu[c][1] * p0[i] + cu[c][2] * p1[i] + cu[c][3] * p2[i];
        if constexpr (HASV) {
          cmv[i] = a.cm[0] * p0[i] + a.cm[1] * p1[i] + a.cm[2] * p2[i];
          nmv[i] = a.cm[1] * p0[i] + a.cm[2] * p1[i] + a.cm[3] * p2[i];
        }
      }
    }
    if constexpr (HASV) {
      if (use_w) {
        F seg[3][PT + 2], p0[PT], p1[PT], p2[PT];
        rows(lds + buf * bufsz + (NC + g * CP + c) * plane + off, seg);
        sums(seg, p0, p1, p2);
#pragma unroll
        for (int i = 0; i < PT; ++i) {
          ck[i] += a.cw[0] * p0[i] + a.cw[1] * p1[i] + a.cw[2] * p2[i];
          nk[i] += a.cw[1] * p0[i] + a.cw[2] * p1[i] + a.cw[3] * p2[i];
        }
      }
    }
  };

  // epilogue operands of one output plane
  struct Extra {
    SV e1[CP], e2[CP];
  };
  const S* e1p = static_cast<const S*>(a.e1);
  const S* e2p = static_cast<const S*>(a.e2);
  const S* e1c[CP];
  const S* e2c[CP];
  S* outc[CP];
#pragma unroll
  for (int c = 0; c < CP; ++c) {
    e1c[c] = e1p ? e1p + int64_t(col0 + c) * a.ld_e1 : nullptr;
    e2c[c] = e2p ? e2p + int64_t(col0 + c) * a.ld_e2 : nullptr;
    outc[c] = static_cast<S*>(a.out) + int64_t(col0 + c) * a.ld_out;
  }
  constexpr bool HAS_E = STEPK || KIND == ZM_CSTEP;
  auto load_e = [&](int z, Extra& E) __attribute__((always_inline)) {
    if (!active) return;
    const uint32_t gb = uint32_t(z) * uint32_t(pstride) * uint32_t(sizeof(S)) + own_b;
    if constexpr (STEPK) {
#pragma unroll
      for (int c = 0; c < CP; ++c) {
        if (!ONE_COL && c >= ncol) continue;
        E.e1[c] = *reinterpret_cast<const SV*>(zm_byte_off(e1c[c], gb));
        E.e2[c] = *reinterpret_cast<const SV*>(zm_byte_off(e2c[c], gb));
      }
    } else if constexpr (KIND == ZM_CSTEP) {
      if (e1p) {
#pragma unroll
        for (int c = 0; c < CP; ++c) {
          if (!ONE_COL && c >= ncol) continue;
          E.e1[c] = *reinterpret_cast<const SV*>(zm_byte_off(e1c[c], gb));
        }
      }
    }
  };

  F accK[CP][PT], accKn[CP][PT], accM[CP][PT], accMn[CP][PT];
  // potential at this thread's points of the next output plane (from staging)
  FV vcur;
  const int zb = a.z0, ze = a.z0 + a.nzs;
  auto wz = [&](int z) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); };

  // The next plane and the next output's epilogue operands are loaded one
  // iteration ahead, into registers.
  Staged A;
  Extra EA;
  load_plane(wz(zb - 1), A);
  load_e(zb, EA);
  write_plane(0, A);
  load_plane(wz(zb), A);
  __syncthreads();
  if (active) {
#pragma unroll
    for (int c = 0; c < CP; ++c) {
      F ck[PT], nk[PT], cmv[PT], nmv[PT];
      combos(0, c, ck, nk, cmv, nmv);
#pragma unroll
      for (int i = 0; i < PT; ++i) {
        accK[c][i] = nk[i];
        accM[c][i] = HASV ? nmv[i] : F(0);
      }
    }
  }
  write_plane(1, A);
  if constexpr (HASV) vcur = A.vs[0];
  if (zb + 1 <= ze) load_plane(wz(zb + 1), A);
  __syncthreads();
  if (active) {
#pragma unroll
    for (int c = 0; c < CP; ++c) {
      F ck[PT], nk[PT], cmv[PT], nmv[PT];
      combos(1, c, ck, nk, cmv, nmv);
#pragma unroll
      for (int i = 0; i < PT; ++i) {
        accK[c][i] += ck[i];
        accKn[c][i] = nk[i];
        if constexpr (HASV) {
          accM[c][i] += cmv[i];
          accMn[c][i] = nmv[i];
        }
      }
    }
  }

  // one output plane: stage plane z+1 from R (and refill R with plane z+2),
  // combine, write out(z) with the operands in E (and refill E with z+1)
  auto step = [&](int z, Staged& R, Extra& E) __attribute__((always_inline)) {
    const int buf = (z - zb) & 1;            // plane z+1 goes where plane z-1 was
    write_plane(buf, R);
    F vc[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i) vc[i] = HASV ? F(vcur[i]) : F(0);
    if constexpr (HASV) vcur = R.vs[0];      // plane z+1, for the next output
    if (z + 2 <= ze) load_plane(wz(z + 2), R);
    __syncthreads();
    if (active) {
      // output byte offset: plane z of the grid, rows shifted by out_off
      const uint32_t ob =
          uint32_t(int64_t(z) * pstride - a.out_off) * uint32_t(sizeof(S)) + own_b;
#pragma unroll
      for (int c = 0; c < CP; ++c) {
        F ck[PT], nk[PT], cmv[PT], nmv[PT];
        combos(buf, c, ck, nk, cmv, nmv);
        if (ONE_COL || c < ncol) {
          F e1v[PT], e2v[PT], cv[PT];
#pragma unroll
          for (int i = 0; i < PT; ++i) cv[i] = F(0);
          if constexpr (KIND == ZM_BSTEP) {
            // boundary correction of this thread's points in plane z (32-bit
            // offsets: the boundary has fewer than 2^31 points; ld_corr is a
            // multiple of 4, so a full row's PT values are one aligned load)
            const int gy = y0 + my_row;
            const F* cc = a.corr + int64_t(col0 + c) * a.ld_corr;
            const uint32_t face = uint32_t(pstride);
            if (z == 0 || z == nz - 1 || gy == 0 || gy == ny - 1) {
              const uint32_t t0 =
                  z == 0        ? uint32_t(gy * nx + xq)
                  : z == nz - 1 ? face + uint32_t(gy * nx + xq)
                                : 2 * face + uint32_t((z - 1) * 2 * nx + (gy == 0 ? 0 : nx) + xq);
              const FV w = *reinterpret_cast<const FV*>(cc + t0);
#pragma unroll
              for (int i = 0; i < PT; ++i) cv[i] = w[i];
            } else if (xq == 0 || xq + PT == nx) {
              const uint32_t t0 = 2 * face + uint32_t(2 * nx * (nz - 2)) +
                                  uint32_t((z - 1) * 2 * (ny - 2) + 2 * (gy - 1));
              if (xq == 0) cv[0] = cc[t0];
              if (xq + PT == nx) cv[PT - 1] = cc[t0 + 1];
            }
          }
          if constexpr (STEPK) {
            zm_cvt<S, F, PT>(E.e1[c], e1v);
            zm_cvt<S, F, PT>(E.e2[c], e2v);
          } else if constexpr (KIND == ZM_CSTEP) {
            if (e1p) {
              zm_cvt<S, F, PT>(E.e1[c], e1v);
            } else {
#pragma unroll
              for (int i = 0; i < PT; ++i) e1v[i] = F(0);
            }
          }
          SV o;
#pragma unroll
          for (int i = 0; i < PT; ++i) {
            F v = accK[c][i] + nk[i];
            if constexpr (HASV) v += vc[i] * (accM[c][i] + nmv[i]);
            if constexpr (HAS_E) v += a.gamma * e1v[i];
            if constexpr (STEPK) v += dcol[c] * e2v[i];
            if constexpr (KIND == ZM_BSTEP) v += cv[i];
            o[i] = zm_store_elem<S, F>(v);
          }
          *reinterpret_cast<SV*>(reinterpret_cast<char*>(outc[c]) + ob) = o;
          if constexpr (KIND == ZM_BSTEP) {
            // the row-end values, for the next step's wrap correction
            if (a.edge_out && (xq == 0 || xq + PT == nx)) {
              S* eo = static_cast<S*>(a.edge_out) + int64_t(col0 + c) * (int64_t(2) * ny * nz);
              const uint32_t e = uint32_t((z * ny + y0 + my_row) * 2);
              if (xq == 0) eo[e] = o[0];
              if (xq + PT == nx) eo[e + 1] = o[PT - 1];
            }
          }
        }
#pragma unroll
        for (int i = 0; i < PT; ++i) {
          accK[c][i] = accKn[c][i] + ck[i];
          accKn[c][i] = nk[i];
          if constexpr (HASV) {
            accM[c][i] = accMn[c][i] + cmv[i];
            accMn[c][i] = nmv[i];
          }
        }
      }
    }
    if (z + 1 < ze) load_e(z + 1, E);
  };

  for (int z = zb; z < ze; ++z) step(z, A, EA);
}

// class-symmetric coefficients? (value depends only on the number of nonzero offsets)
bool class_symmetric(const double* c, double out[4]) {
  bool seen[4] = {false, false, false, false};
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int cls = (dz != 0) + (dy != 0) + (dx != 0);
        const double v = c[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
        if (!seen[cls]) {
          out[cls] = v;
          seen[cls] = true;
        } else if (v != out[cls]) {
          return false;
        }
      }
  return true;
}

// slab height: full x rows, at most sep_pt<F>() points per thread per plane
template <typename F>
int sep_ty(const chfsi_operator& op) {
  const int cap = 256 * sep_pt<F>();
  if (op.nx > cap) return 0;
  int ty = std::min(cap / op.nx, op.ny);
  return ty >= 1 ? ty : 0;
}

template <typename F>
bool sep_setup(const chfsi_operator& op, SepArgs<F>* a) {
  double cA[4], cM[4] = {0, 0, 0, 0};
  if (!class_symmetric(op.coef, cA)) return false;
  if (op.field_mode == 2 && !class_symmetric(op.coef_mass, cM)) return false;
  const int ty = sep_ty<F>(op);
  if (ty == 0) return false;
  a->nx = op.nx;
  a->ny = op.ny;
  a->nz = op.nz;
  a->z0 = 0;
  a->nzs = op.nz;
  a->out_off = 0;
  a->b_identity = 1;
  for (int i = 0; i < 4; ++i) a->cB[i] = F(0);
  a->ty = ty;
  a->ntiles_y = (op.ny + ty - 1) / ty;
  a->mode = op.field_mode;
  for (int i = 0; i < 4; ++i) {
    a->cA[i] = F(cA[i]);
    a->cM[i] = F(cM[i]);
  }
  a->V = op.field;
  a->dinv = nullptr;
  a->prev = nullptr;
  a->forcing = nullptr;
  a->colcoef = nullptr;
  a->alpha = F(1);
  a->beta = a->gamma = a->delta = F(0);
  return true;
}

template <typename S, typename F, int KIND>
hipError_t sep_launch(const SepArgs<F>& a, int64_t b, hipStream_t st) {
  const int64_t grid = int64_t(a.ntiles_y) * b;
  const size_t lds = size_t(2) * 2 * (a.ty + 2) * a.nx * sizeof(F);
  k_stencil_sep<S, F, KIND><<<dim3(unsigned(grid)), 256, lds, st>>>(a);
  return hipGetLastError();
}

// ---- vectorised z-march: set-up and launch --------------------------------
inline bool zm_aligned(const void* p, int64_t ld, size_t vec_bytes, int PT) {
  return p == nullptr || ((reinterpret_cast<uintptr_t>(p) % vec_bytes) == 0 && ld % PT == 0);
}

// Coefficients for out = alpha * op(u) + beta * u (+ extra streams).  Returns
// false when the operator is not class-symmetric or the grid does not fit the
// thread layout (nx a multiple of PT, at most 128 PT-chunks per row).
inline size_t zm_lds_bytes(int nx, int ty, int cp, bool hasv, size_t fbytes) {
  // two buffers of: u of every column, and with a potential w = V u of every column
  return size_t(2) * (hasv ? 2 * cp : cp) * (ty + 2) * (nx + 8) * fbytes;
}

template <typename F>
bool zm_setup(const chfsi_operator& op, int PT, int CP, double alpha, double beta, ZmArgs<F>* a) {
  double cA[4], cM[4] = {0, 0, 0, 0};
  if (!class_symmetric(op.coef, cA)) return false;
  if (op.field_mode == 2 && !class_symmetric(op.coef_mass, cM)) return false;
  if (op.nx % PT != 0 || op.nx / PT > 128 || op.nx < 2 * PT) return false;
  // per-lane byte offsets within a column are 32-bit
  if (int64_t(op.n) * int64_t(sizeof(double)) >= (int64_t(1) << 31)) return false;
  const int tpr = op.nx / PT;
  if (zm_lds_bytes(op.nx, std::min(256 / tpr, op.ny), CP, op.field_mode != 0, sizeof(F)) > 65536)
    return false;
  *a = ZmArgs<F>{};
  a->nx = op.nx;
  a->ny = op.ny;
  a->nz = op.nz;
  a->ty = std::min(256 / tpr, op.ny);
  a->ntiles_y = (op.ny + a->ty - 1) / a->ty;
  a->z0 = 0;
  a->nzs = op.nz;
  a->out_off = 0;
  a->use_w = op.field_mode == 2 ? 1 : 0;
  for (int k = 0; k < 4; ++k) {
    a->cu[k] = F(alpha * cA[k] + (k == 0 ? beta : 0.0));
    a->cw[k] = F(op.field_mode == 2 ? 0.5 * alpha * cM[k] : 0.0);
    a->cm[k] = F(op.field_mode == 2 ? 0.5 * alpha * cM[k]
                                    : (op.field_mode == 1 && k == 0 ? alpha : 0.0));
    a->cb[k] = F(0);
  }
  a->gamma = F(0);
  a->delta = F(0);
  return true;
}

// workgroup -> tile order (tuning knob CHFSI_STENCIL_ORDER = 1 or 2 selects
// order 0 or 1; unset = default)
int zm_order(bool hasv) {
  static const int v = [] {
    const char* e = std::getenv("CHFSI_STENCIL_ORDER");
    const int o = e ? std::atoi(e) : 0;
    return (o == 1 || o == 2) ? o : 0;
  }();
  if (v) return v - 1;
  return hasv ? 1 : 0;
}

template <typename S, typename F, int PT, int CP, int NG, int KIND>
hipError_t zm_launch_ng(const ZmArgs<F>& a, bool hasv, hipStream_t st) {
  const int per = CP * NG;
  const int64_t grid = int64_t((a.b + per - 1) / per) * a.ntiles_y;
  ZmArgs<F> ar = a;
  ar.order = zm_order(hasv);
  const size_t lds = zm_lds_bytes(a.nx, a.ty, per, hasv, sizeof(F));
  if (lds > 65536) return hipErrorInvalidValue;
  const dim3 gd{unsigned(grid)};
  if (hasv)
    k_zmarch<S, F, PT, CP, NG, KIND, true><<<gd, 256 * NG, lds, st>>>(ar);
  else
    k_zmarch<S, F, PT, CP, NG, KIND, false><<<gd, 256 * NG, lds, st>>>(ar);
  return hipGetLastError();
}

// Workgroup shape of the z-march: CP columns per thread, NG groups of 256
// threads sharing the staged potential (tuning knobs CHFSI_STENCIL_COLS and
// CHFSI_STENCIL_GROUPS; 0 = default).  Measured on MI355X at 128^3 x 1200
// columns with the mass-weighted potential: one column per thread gives the
// highest occupancy (108 VGPRs, 4 waves/SIMD); more columns per thread cost
// more in occupancy than they save.  Groups share the potential's plane
// without costing registers, but coupling 8 or 16 waves at every plane's
// barrier costs more than the saved potential reads (BF16: 1 group 5.98 ms,
// 2 groups 7.13 ms, 4 groups 6.94 ms per step).
struct ZmShape {
  int cp, ng;
};
int zm_env(const char* name) {
  const char* e = std::getenv(name);
  const int v = e ? std::atoi(e) : 0;
  return (v == 1 || v == 2 || v == 4) ? v : 0;
}
ZmShape zm_shape(bool lowp) {
  static const int cp = zm_env("CHFSI_STENCIL_COLS");
  static const int ng = zm_env("CHFSI_STENCIL_GROUPS");
  ZmShape sh{cp ? cp : 1, ng ? ng : 1};
  if (!lowp) {
    sh.cp = 1;
    sh.ng = std::min(sh.ng, 2);
  }
  if (sh.cp == 4) sh.ng = 1;
  if (sh.cp == 2) sh.ng = std::min(sh.ng, 2);
  return sh;
}

template <typename S, typename F, int PT, int KIND>
hipError_t zm_launch(const ZmArgs<F>& a, bool hasv, hipStream_t st) {
  const ZmShape sh = zm_shape(sizeof(F) == 4);
  if constexpr (sizeof(F) == 8) {
    // FP64: at most 2 groups (4 would cap the kernel at 128 VGPRs and spill)
    if (sh.ng == 1) return zm_launch_ng<S, F, PT, 1, 1, KIND>(a, hasv, st);
    return zm_launch_ng<S, F, PT, 1, 2, KIND>(a, hasv, st);
  } else if constexpr (PT == 2) {
    return zm_launch_ng<S, F, 2, 1, 1, KIND>(a, hasv, st);
  } else {
    if (sh.cp == 2) {
      if (sh.ng == 1) return zm_launch_ng<S, F, PT, 2, 1, KIND>(a, hasv, st);
      return zm_launch_ng<S, F, PT, 2, 2, KIND>(a, hasv, st);
    }
    if (sh.cp == 4) return zm_launch_ng<S, F, PT, 4, 1, KIND>(a, hasv, st);
    if (sh.ng == 1) return zm_launch_ng<S, F, PT, 1, 1, KIND>(a, hasv, st);
    if (sh.ng == 2) return zm_launch_ng<S, F, PT, 1, 2, KIND>(a, hasv, st);
    return zm_launch_ng<S, F, PT, 1, 4, KIND>(a, hasv, st);
  }
}

// points per thread of the FP32/BF16 filter steps (tuning knob CHFSI_STENCIL_PT)
int zm_pt_lowp() {
  static const int v = zm_env("CHFSI_STENCIL_PT");
  return v == 2 ? 2 : 4;
}

// columns sharing one workgroup's staged planes (for the LDS-size check)
int zm_per_wg(bool lowp) {
  const ZmShape sh = zm_shape(lowp);
  return sh.cp * sh.ng;
}

Grid make_grid(const chfsi_operator& op) {
  Grid g;
  g.nx = op.nx;
  g.ny = op.ny;
  g.nz = op.nz;
  g.mode = op.field_mode;
  g.V = op.field;
  return g;
}

CoefsD make_coefs_d(const chfsi_operator& op) {
  CoefsD c;
  for (int i = 0; i < 27; ++i) {
    c.c[i] = op.coef[i];
    c.m[i] = op.coef_mass[i];
  }
  return c;
}

Coefs make_coefs_f(const chfsi_operator& op) {
  Coefs c;
  for (int i = 0; i < 27; ++i) {
    c.c[i] = float(op.coef[i]);
    c.m[i] = float(op.coef_mass[i]);
  }
  return c;
}

}  // namespace

hipError_t stencil_check(const chfsi_operator& op) {
  if (op.nx < 3 || op.ny < 3 || op.nz < 3) return hipErrorInvalidValue;
  return hipSuccess;
}

double stencil_flops(const chfsi_operator& op) {
  // nominal: 2 flops per coefficient and the fused three-term update
  return 2.0 * 27.0 + 8.0 + (op.field_mode == 2 ? 4.0 * 27.0 : (op.field_mode == 1 ? 2.0 : 0.0));
}

hipError_t stencil_apply_f64(const chfsi_operator& op, const double* X, int64_t ldx, double* Y,
                             int64_t ldy, int64_t b, hipStream_t st) {
  ZmArgs<double> z;
  if (zm_setup(op, 2, zm_per_wg(false), 1.0, 0.0, &z) && zm_aligned(X, ldx, 16, 2) && zm_aligned(Y, ldy, 16, 2) &&
      zm_aligned(op.field, 0, 16, 2)) {
    z.b = int(b);
    z.V = op.field;
    z.src = X;
    z.ld_src = ldx;
    z.out = Y;
    z.ld_out = ldy;
    return zm_launch<double, double, 2, ZM_APPLY>(z, op.field_mode != 0, st);
  }
  SepArgs<double> a;
  if (sep_setup(op, &a)) {
    a.src = X;
    a.lds_src = ldx;
    a.out = Y;
    a.ld_out = ldy;
    return sep_launch<double, double, SK_APPLY>(a, b, st);
  }
  k_apply_f64<<<grid_for(op.n * b), 256, 0, st>>>(make_coefs_d(op), make_grid(op), X, ldx, Y, ldy,
                                                  op.n, b);
  return hipGetLastError();
}

hipError_t stencil_rchfsi_step_f64(const chfsi_operator& op, const double* dinv, const double* RY,
                                   double* RX, const double* Yf, int64_t ldf,
                                   const double* colcoef, StencilStep s, int64_t b,
                                   hipStream_t st, const BlochStep* bloch) {
  if (bloch && (b % 2 != 0 || bloch->ld_corr % 4 != 0)) return hipErrorInvalidValue;
  ZmArgs<double> z;
  if (!dinv && RX && Yf && zm_setup(op, 2, zm_per_wg(false), s.alpha, s.beta, &z) &&
      zm_aligned(RY, op.n, 16, 2) && zm_aligned(RX, op.n, 16, 2) && zm_aligned(Yf, ldf, 16, 2) &&
      zm_aligned(op.field, 0, 16, 2)) {
    z.b = int(b);
    z.V = op.field;
    z.src = RY;
    z.ld_src = op.n;
    z.out = RX;
    z.ld_out = op.n;
    z.e1 = RX;
    z.ld_e1 = op.n;
    z.gamma = s.gamma;
    z.e2 = Yf;
    z.ld_e2 = ldf;
    z.delta = s.delta;
    z.colcoef = colcoef;
    if (bloch) {
      double* corr = static_cast<double*>(bloch->corr);
      const hipError_t e = bloch_corr<double, double>(
          op, bloch->dinv, s.alpha, RY, op.n, static_cast<const double*>(bloch->edge_in), corr,
          bloch->ld_corr, b / 2, st);
      if (e != hipSuccess) return e;
      z.corr = corr;
      z.ld_corr = bloch->ld_corr;
      z.edge_out = bloch->edge_out;
      return zm_launch<double, double, 2, ZM_BSTEP>(z, op.field_mode != 0, st);
    }
    return zm_launch<double, double, 2, ZM_STEP>(z, op.field_mode != 0, st);
  }
  SepArgs<double> a;
  if (sep_setup(op, &a)) {
    a.dinv = dinv;
    a.src = RY;
    a.lds_src = op.n;
    a.out = RX;
    a.ld_out = op.n;
    a.forcing = Yf;
    a.ld_forcing = ldf;
    a.colcoef = colcoef;
    a.alpha = s.alpha;
    a.beta = s.beta;
    a.gamma = s.gamma;
    a.delta = s.delta;
    const hipError_t e = sep_launch<double, double, SK_RSTEP>(a, b, st);
    if (e != hipSuccess || !bloch) return e;
  } else {
    k_rstep_f64<<<grid_for(op.n * b), 256, 0, st>>>(make_coefs_d(op), make_grid(op), dinv, RY,
                                                    RX, Yf, ldf, colcoef, s, op.n, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || !bloch) return e;
  }
  return bloch_fix<double>(op, bloch->dinv, s.alpha, RY, op.n, RX, op.n, b / 2, st);
}

hipError_t stencil_rchfsi_step_f32(const chfsi_operator& op, const float* Vf, const float* dinv,
                                   const float* RY, float* RX, const float* Yf,
                                   const float* colcoef, StencilStep s, int64_t b, hipStream_t st,
                                   const BlochStep* bloch) {
  if (bloch && (b % 2 != 0 || bloch->ld_corr % 4 != 0)) return hipErrorInvalidValue;
  ZmArgs<float> z;
  const int pt = zm_pt_lowp();
  const size_t vb = size_t(pt) * sizeof(float);
  if (!dinv && RX && Yf && (op.field_mode == 0 || Vf) &&
      zm_setup(op, pt, zm_per_wg(true), s.alpha, s.beta, &z) && zm_aligned(RY, op.n, vb, pt) &&
      zm_aligned(RX, op.n, vb, pt) && zm_aligned(Yf, op.n, vb, pt) && zm_aligned(Vf, 0, vb, pt)) {
    z.b = int(b);
    z.V = Vf;
    z.src = RY;
    z.ld_src = op.n;
    z.out = RX;
    z.ld_out = op.n;
    z.e1 = RX;
    z.ld_e1 = op.n;
    z.gamma = float(s.gamma);
    z.e2 = Yf;
    z.ld_e2 = op.n;
    z.delta = float(s.delta);
    z.colcoef = colcoef;
    if (bloch) {
      float* corr = static_cast<float*>(bloch->corr);
      const hipError_t e = bloch_corr<float, float>(
          op, bloch->dinv, s.alpha, RY, op.n, static_cast<const float*>(bloch->edge_in), corr,
          bloch->ld_corr, b / 2, st);
      if (e != hipSuccess) return e;
      z.corr = corr;
      z.ld_corr = bloch->ld_corr;
      z.edge_out = bloch->edge_out;
      return pt == 2 ? zm_launch<float, float, 2, ZM_BSTEP>(z, op.field_mode != 0, st)
                     : zm_launch<float, float, 4, ZM_BSTEP>(z, op.field_mode != 0, st);
    }
    return pt == 2 ? zm_launch<float, float, 2, ZM_STEP>(z, op.field_mode != 0, st)
                   : zm_launch<float, float, 4, ZM_STEP>(z, op.field_mode != 0, st);
  }
  SepArgs<float> a;
  if (sep_setup(op, &a)) {
    a.dinv = dinv;
    a.src = RY;
    a.lds_src = op.n;
    a.out = RX;
    a.ld_out = op.n;
    a.forcing = Yf;
    a.ld_forcing = op.n;
    a.colcoef = colcoef;
    a.alpha = float(s.alpha);
    a.beta = float(s.beta);
    a.gamma = float(s.gamma);
    a.delta = float(s.delta);
    const hipError_t e = sep_launch<float, float, SK_RSTEP>(a, b, st);
    if (e != hipSuccess || !bloch) return e;
  } else {
    k_rstep_f32<<<grid_for(op.n * b), 256, 0, st>>>(make_coefs_f(op), make_grid(op), dinv, RY,
                                                    RX, Yf, colcoef, float(s.alpha),
                                                    float(s.beta), float(s.gamma),
                                                    float(s.delta), op.n, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || !bloch) return e;
  }
  return bloch_fix<float>(op, bloch->dinv, s.alpha, RY, op.n, RX, op.n, b / 2, st);
}

hipError_t stencil_rchfsi_step_bf16(const chfsi_operator& op, const float* Vf, const float* dinv,
                                    const void* RY, void* RX, const void* Yf,
                                    const float* colcoef, StencilStep s, int64_t b,
                                    hipStream_t st, const BlochStep* bloch) {
  if (bloch && (b % 2 != 0 || bloch->ld_corr % 4 != 0)) return hipErrorInvalidValue;
  const uint16_t* RY16 = static_cast<const uint16_t*>(RY);
  ZmArgs<float> z;
  const int pt = zm_pt_lowp();
  const size_t vb = size_t(pt) * 2, vf = size_t(pt) * sizeof(float);
  if (!dinv && RX && Yf && (op.field_mode == 0 || Vf) &&
      zm_setup(op, pt, zm_per_wg(true), s.alpha, s.beta, &z) && zm_aligned(RY, op.n, vb, pt) &&
      zm_aligned(RX, op.n, vb, pt) && zm_aligned(Yf, op.n, vb, pt) && zm_aligned(Vf, 0, vf, pt)) {
    z.b = int(b);
    z.V = Vf;
    z.src = RY;
    z.ld_src = op.n;
    z.out = RX;
    z.ld_out = op.n;
    z.e1 = RX;
    z.ld_e1 = op.n;
    z.gamma = float(s.gamma);
    z.e2 = Yf;
    z.ld_e2 = op.n;
    z.delta = float(s.delta);
    z.colcoef = colcoef;
    if (bloch) {
      float* corr = static_cast<float*>(bloch->corr);
      const hipError_t e = bloch_corr<uint16_t, float>(
          op, bloch->dinv, s.alpha, RY16, op.n, static_cast<const uint16_t*>(bloch->edge_in), corr,
          bloch->ld_corr, b / 2, st);
      if (e != hipSuccess) return e;
      z.corr = corr;
      z.ld_corr = bloch->ld_corr;
      z.edge_out = bloch->edge_out;
      return pt == 2 ? zm_launch<uint16_t, float, 2, ZM_BSTEP>(z, op.field_mode != 0, st)
                     : zm_launch<uint16_t, float, 4, ZM_BSTEP>(z, op.field_mode != 0, st);
    }
    return pt == 2 ? zm_launch<uint16_t, float, 2, ZM_STEP>(z, op.field_mode != 0, st)
                   : zm_launch<uint16_t, float, 4, ZM_STEP>(z, op.field_mode != 0, st);
  }
  SepArgs<float> a;
  if (sep_setup(op, &a)) {
    a.dinv = dinv;
    a.src = RY;
    a.lds_src = op.n;
    a.out = RX;
    a.ld_out = op.n;
    a.forcing = Yf;
    a.ld_forcing = op.n;
    a.colcoef = colcoef;
    a.alpha = float(s.alpha);
    a.beta = float(s.beta);
    a.gamma = float(s.gamma);
    a.delta = float(s.delta);
    const hipError_t e = sep_launch<uint16_t, float, SK_RSTEP>(a, b, st);
    if (e != hipSuccess || !bloch) return e;
  } else {
    k_rstep_bf16<<<grid_for(op.n * b), 256, 0, st>>>(
        make_coefs_f(op), make_grid(op), dinv, RY16, static_cast<uint16_t*>(RX),
        static_cast<const uint16_t*>(Yf), colcoef, float(s.alpha), float(s.beta),
        float(s.gamma), float(s.delta), op.n, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || !bloch) return e;
  }
  return bloch_fix<uint16_t>(op, bloch->dinv, s.alpha, RY16, op.n, static_cast<uint16_t*>(RX),
                             op.n, b / 2, st);
}

hipError_t stencil_chfsi_step_f64(const chfsi_operator& op, const double* dinv, const double* src,
                                  int64_t lds, const double* prev, int64_t ldp, double* dst,
                                  StencilStep s, int64_t b, hipStream_t st) {
  ZmArgs<double> z;
  if (!dinv && zm_setup(op, 2, zm_per_wg(false), s.alpha, s.beta, &z) && zm_aligned(src, lds, 16, 2) &&
      zm_aligned(prev, ldp, 16, 2) && zm_aligned(dst, op.n, 16, 2) &&
      zm_aligned(op.field, 0, 16, 2)) {
    z.b = int(b);
    z.V = op.field;
    z.src = src;
    z.ld_src = lds;
    z.out = dst;
    z.ld_out = op.n;
    z.e1 = prev;
    z.ld_e1 = ldp;
    z.gamma = s.gamma;
    return zm_launch<double, double, 2, ZM_CSTEP>(z, op.field_mode != 0, st);
  }
  SepArgs<double> a;
  if (sep_setup(op, &a)) {
    a.dinv = dinv;
    a.src = src;
    a.lds_src = lds;
    a.out = dst;
    a.ld_out = op.n;
    a.prev = prev;
    a.ld_prev = ldp;
    a.alpha = s.alpha;
    a.beta = s.beta;
    a.gamma = s.gamma;
    return sep_launch<double, double, SK_CSTEP>(a, b, st);
  }
  k_cstep_f64<<<grid_for(op.n * b), 256, 0, st>>>(make_coefs_d(op), make_grid(op), dinv, src, lds,
                                                  prev, ldp, dst, s, op.n, b);
  return hipGetLastError();
}

hipError_t rchfsi_init_bf16(const double* R, int64_t ldr, int64_t n, int64_t b, double scale,
                            void* RY, void* RX, void* Yc, hipStream_t st) {
  k_init_bf16<<<grid_for(n * b), 256, 0, st>>>(R, ldr, n, b, scale, static_cast<uint16_t*>(RY),
                                               static_cast<uint16_t*>(RX),
                                               static_cast<uint16_t*>(Yc));
  return hipGetLastError();
}

hipError_t rchfsi_reconstruct_bf16(const void* RY, const double* dinv, const double* X,
                                   int64_t ldx, const double* lamY, double* Yp, int64_t ldy,
                                   int64_t n, int64_t b, hipStream_t st) {
  k_recon_bf16<<<grid_for(n * b), 256, 0, st>>>(static_cast<const uint16_t*>(RY), dinv, X, ldx,
                                                lamY, Yp, ldy, n, b);
  return hipGetLastError();
}

// Y_slab = (op X)[rows of planes z0 .. z0+nzs-1]; Y_slab rows are indexed
// from the slab's first grid point.  Class-symmetric coefficients only.
hipError_t stencil_apply_slab_f64(const chfsi_operator& op, const double* X, int64_t ldx,
                                  double* Yslab, int64_t ldy, int64_t b, int z0, int nzs,
                                  hipStream_t st) {
  if (z0 < 0 || nzs < 1 || z0 + nzs > op.nz) return hipErrorInvalidValue;
  ZmArgs<double> z;
  if (zm_setup(op, 2, zm_per_wg(false), 1.0, 0.0, &z) && zm_aligned(X, ldx, 16, 2) && zm_aligned(Yslab, ldy, 16, 2) &&
      zm_aligned(op.field, 0, 16, 2)) {
    z.b = int(b);
    z.z0 = z0;
    z.nzs = nzs;
    z.out_off = int64_t(z0) * op.nx * op.ny;
    z.V = op.field;
    z.src = X;
    z.ld_src = ldx;
    z.out = Yslab;
    z.ld_out = ldy;
    return zm_launch<double, double, 2, ZM_APPLY>(z, op.field_mode != 0, st);
  }
  SepArgs<double> a;
  if (!sep_setup(op, &a)) return hipErrorInvalidValue;
  a.z0 = z0;
  a.nzs = nzs;
  a.out_off = int64_t(z0) * op.nx * op.ny;
  a.src = X;
  a.lds_src = ldx;
  a.out = Yslab;
  a.ld_out = ldy;
  return sep_launch<double, double, SK_APPLY>(a, b, st);
}

// R = A X - B X diag(lam) in one pass (B = NULL: identity).  Class-symmetric only.
hipError_t stencil_residual_f64(const chfsi_operator& A, const chfsi_operator* B, const double* X,
                                int64_t ldx, const double* lam, double* R, int64_t ldr, int64_t b,
                                hipStream_t st) {
  ZmArgs<double> z;
  double cb[4] = {1.0, 0.0, 0.0, 0.0};
  if ((!B || class_symmetric(B->coef, cb)) && zm_setup(A, 2, zm_per_wg(false), 1.0, 0.0, &z) &&
      zm_aligned(X, ldx, 16, 2) && zm_aligned(R, ldr, 16, 2) && zm_aligned(A.field, 0, 16, 2)) {
    for (int k = 0; k < 4; ++k) z.cb[k] = cb[k];
    z.b = int(b);
    z.V = A.field;
    z.src = X;
    z.ld_src = ldx;
    z.out = R;
    z.ld_out = ldr;
    z.colcoef = lam;
    return zm_launch<double, double, 2, ZM_RESID>(z, A.field_mode != 0, st);
  }
  SepArgs<double> a;
  if (!sep_setup(A, &a)) return hipErrorInvalidValue;
  if (B) {
    double cb[4];
    if (!class_symmetric(B->coef, cb)) return hipErrorInvalidValue;
    for (int i = 0; i < 4; ++i) a.cB[i] = cb[i];
    a.b_identity = 0;
  }
  a.src = X;
  a.lds_src = ldx;
  a.out = R;
  a.ld_out = ldr;
  a.colcoef = lam;
  return sep_launch<double, double, SK_RESID>(a, b, st);
}

bool stencil_separable(const chfsi_operator& op) {
  SepArgs<double> a;
  return sep_setup(op, &a);
}

}  // namespace chfsi
