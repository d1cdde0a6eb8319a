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

#include <cmath>

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
    const float av = apply_point<float>(cf, g, x, y, z, [&](int64_t k) { return dinv[k] * col[k]; });
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
                                        [&](int64_t k) { return dinv[k] * bf16_to_f32(col[k]); });
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
  k_apply_f64<<<grid_for(op.n * b), 256, 0, st>>>(make_coefs_d(op), make_grid(op), X, ldx, Y, ldy,
                                                  op.n, b);
  return hipGetLastError();
}

hipError_t stencil_rchfsi_step_f64(const chfsi_operator& op, const double* dinv, const double* RY,
                                   double* RX, const double* Yf, int64_t ldf,
                                   const double* colcoef, StencilStep s, int64_t b,
                                   hipStream_t st) {
  k_rstep_f64<<<grid_for(op.n * b), 256, 0, st>>>(make_coefs_d(op), make_grid(op), dinv, RY, RX,
                                                  Yf, ldf, colcoef, s, op.n, b);
  return hipGetLastError();
}

hipError_t stencil_rchfsi_step_f32(const chfsi_operator& op, const float* dinv, const float* RY,
                                   float* RX, const float* Yf, const float* colcoef,
                                   StencilStep s, int64_t b, hipStream_t st) {
  k_rstep_f32<<<grid_for(op.n * b), 256, 0, st>>>(make_coefs_f(op), make_grid(op), dinv, RY, RX,
                                                  Yf, colcoef, float(s.alpha), float(s.beta),
                                                  float(s.gamma), float(s.delta), op.n, b);
  return hipGetLastError();
}

hipError_t stencil_rchfsi_step_bf16(const chfsi_operator& op, const float* dinv, const void* RY,
                                    void* RX, const void* Yf, const float* colcoef, StencilStep s,
                                    int64_t b, hipStream_t st) {
  k_rstep_bf16<<<grid_for(op.n * b), 256, 0, st>>>(
      make_coefs_f(op), make_grid(op), dinv, static_cast<const uint16_t*>(RY),
      static_cast<uint16_t*>(RX), static_cast<const uint16_t*>(Yf), colcoef, float(s.alpha),
      float(s.beta), float(s.gamma), float(s.delta), op.n, b);
  return hipGetLastError();
}

hipError_t stencil_chfsi_step_f64(const chfsi_operator& op, const double* dinv, const double* src,
                                  int64_t lds, const double* prev, int64_t ldp, double* dst,
                                  StencilStep s, int64_t b, hipStream_t st) {
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

}  // namespace chfsi
