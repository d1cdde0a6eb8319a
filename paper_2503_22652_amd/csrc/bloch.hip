// Bloch-phase (k-point) grid operators (Section 4.3's complex problems on the
// periodic grid), run in a twisted frame.
//
// The Bloch operator at wave vector k multiplies the coefficient of offset o
// by exp(i k.o).  With D = diag(exp(i k.r)) over the grid points r = (x, y, z)
// it equals D^* A_tw D, where A_tw is the real periodic stencil except that a
// neighbour reached through a periodic wrap carries the factor
//   phi = exp(i (s_x k_x n_x + s_y k_y n_y + s_z k_z n_z)),
// s_d = +1 for a wrap past the upper face of dimension d, -1 past the lower
// face, 0 otherwise.  D is unitary and commutes with the diagonal D^{-1} and V,
// so the pencil in the twisted frame has the same eigenvalues, eigenvectors
// D u and residuals D r.  In that frame a complex block is kept planar (n x 2b:
// real parts in columns 0..b-1, imaginary parts in b..2b-1); the real
// z-marching kernels act on both halves unchanged, and the phases enter as a
// correction at the boundary points only:
//   (A_tw - A_per) psi (p) = sum over wrapped offsets o of w(p, o) (phi - 1) psi(q),
// q = p + o (mod grid), w = c(o), plus 1/2 m(o) (V(p) + V(q)) for the
// mass-weighted potential (the diagonal potential has no wrapped term).
//
// The boundary points (n - (nx-2)(ny-2)(nz-2) of them) are enumerated as the
// two z faces, then the y = 0 and y = ny-1 rows of the inner planes, then the
// x = 0 and x = nx-1 points of the inner rows.
#include "internal.h"
#include "stencil_api.h"

#include <cmath>
#include <cstdint>
#include <type_traits>

namespace chfsi {

namespace {

constexpr int kThreads = 256;

inline int64_t grid_for(int64_t total, int64_t cap = 65536) {
  int64_t g = (total + kThreads - 1) / kThreads;
  if (g < 1) g = 1;
  return g > cap ? cap : g;
}

template <typename F>
__device__ __forceinline__ double load_el(F v) {
  return double(v);
}
template <>
__device__ __forceinline__ double load_el<uint16_t>(uint16_t v) {
  return double(__uint_as_float(uint32_t(v) << 16));
}
template <typename F>
__device__ __forceinline__ F store_el(double v) {
  return F(v);
}
template <>
__device__ __forceinline__ uint16_t store_el<uint16_t>(double v) {
  // bfloat16, round to nearest even (hardware conversion)
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(float(v)));
}

// phase angle k.r of grid point i (x fastest)
__device__ __forceinline__ double point_phase(const Twist& tw, int64_t i) {
  const int64_t x = i % tw.nx, r = i / tw.nx;
  const int64_t y = r % tw.ny, z = r / tw.ny;
  return tw.kx * double(x) + tw.ky * double(y) + tw.kz * double(z);
}

// R_Y = scale * D R, R_X = 0, Yc = D R (planar, ld n) from the interleaved
// residual; E (may be null) receives R_Y's x = 0 and x = nx-1 values,
// ((z ny + y) 2 + (x == nx-1)) per column, ld 2 n / nx
template <typename F>
__global__ __launch_bounds__(kThreads) void k_binit(const double* __restrict__ R, int64_t ldr,
                                                    int64_t n, int64_t b, double scale,
                                                    F* __restrict__ RY, F* __restrict__ RX,
                                                    F* __restrict__ Yc, F* __restrict__ E,
                                                    Twist tw) {
  const int64_t total = n * b, lde = 2 * (n / tw.nx);
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    double s, c;
    sincos(point_phase(tw, i), &s, &c);
    const double zr = R[2 * (i + j * ldr)], zi = R[2 * (i + j * ldr) + 1];
    const double re = c * zr - s * zi, im = s * zr + c * zi;
    const int64_t pr = i + j * n, pi = i + (b + j) * n;
    const F yr = store_el<F>(scale * re), yi = store_el<F>(scale * im);
    RY[pr] = yr;
    RY[pi] = yi;
    const int64_t x = i % tw.nx;
    if (E && (x == 0 || x == tw.nx - 1)) {
      const int64_t e = (i / tw.nx) * 2 + (x == 0 ? 0 : 1);   // (z ny + y) 2 + end
      E[e + j * lde] = yr;
      E[e + (b + j) * lde] = yi;
    }
    RX[pr] = store_el<F>(0.0);
    RX[pi] = store_el<F>(0.0);
    Yc[pr] = store_el<F>(re);
    Yc[pi] = store_el<F>(im);
  }
}

// Yp = D^* (D^{-1} R_Y) + X Lambda_Y (interleaved complex, FP64); X is in the
// untwisted frame
template <typename F>
__global__ __launch_bounds__(kThreads) void k_brecon(const F* __restrict__ RY,
                                                     const double* __restrict__ dinv,
                                                     const double* __restrict__ X, int64_t ldx,
                                                     const double* __restrict__ lam, double* Yp,
                                                     int64_t ldy, int64_t n, int64_t b, Twist tw) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    double s, c;
    sincos(point_phase(tw, i), &s, &c);
    const double d = dinv ? dinv[i] : 1.0, l = lam[j];
    const double pr = d * load_el<F>(RY[i + j * n]), pi = d * load_el<F>(RY[i + (b + j) * n]);
    const double xr = X[2 * (i + j * ldx)], xi = X[2 * (i + j * ldx) + 1];
    Yp[2 * (i + j * ldy)] = c * pr + s * pi + xr * l;
    Yp[2 * (i + j * ldy) + 1] = c * pi - s * pr + xi * l;
  }
}

// planar P = D Z (n x 2b, ld n) from interleaved Z (ld ldz), and Z = D^* P
__global__ __launch_bounds__(kThreads) void k_bto_planar(const double* __restrict__ Z, int64_t ldz,
                                                         int64_t n, int64_t b,
                                                         double* __restrict__ P, Twist tw) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    double s, c;
    sincos(point_phase(tw, i), &s, &c);
    const double zr = Z[2 * (i + j * ldz)], zi = Z[2 * (i + j * ldz) + 1];
    P[i + j * n] = c * zr - s * zi;
    P[i + (b + j) * n] = s * zr + c * zi;
  }
}

__global__ __launch_bounds__(kThreads) void k_bfrom_planar(const double* __restrict__ P, int64_t n,
                                                           int64_t b, double* __restrict__ Z,
                                                           int64_t ldz, Twist tw) {
  const int64_t total = n * b;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t j = idx / n, i = idx - j * n;
    double s, c;
    sincos(point_phase(tw, i), &s, &c);
    const double pr = P[i + j * n], pi = P[i + (b + j) * n];
    Z[2 * (i + j * ldz)] = c * pr + s * pi;
    Z[2 * (i + j * ldz) + 1] = c * pi - s * pr;
  }
}

struct FixArgs {
  double c[27];      // stencil coefficient of offset (dx,dy,dz), index (dz+1)*9 + (dy+1)*3 + dx+1
  double hm[27];     // half the mass coefficient (mass-weighted potential), else zero
  double cw[3], sw[3];   // cos, sin of k_d n_d for d = x, y, z
  int nx, ny, nz, field2;
};

// boundary point t (0 <= t < number of boundary points, < 2^31) -> (x, y, z)
__device__ __forceinline__ void boundary_point(int t, int nx, int ny, int nz, int* x, int* y,
                                               int* z) {
  const int face = nx * ny;
  if (t < 2 * face) {
    const int r = t < face ? t : t - face;
    *z = t < face ? 0 : nz - 1;
    *y = r / nx;
    *x = r - *y * nx;
    return;
  }
  t -= 2 * face;
  const int rows = 2 * nx * (nz - 2);
  if (t < rows) {
    const int zz = t / (2 * nx), r = t - zz * 2 * nx;
    *z = 1 + zz;
    *y = r < nx ? 0 : ny - 1;
    *x = r < nx ? r : r - nx;
    return;
  }
  t -= rows;
  const int zz = t / (2 * (ny - 2)), r = t - zz * 2 * (ny - 2);
  *z = 1 + zz;
  *y = 1 + r / 2;
  *x = (r & 1) ? nx - 1 : 0;
}

// Pairs of columns per thread of the correction kernels: the geometry, wrap
// phase and weight of each wrapped offset are computed once and applied to
// kPairs column pairs (independent gathers).
constexpr int kPairs = 16;

// The correction at boundary point t for column pairs (j, b + j), j in
// [j0, j0 + kPairs) (those below b): out(j) = alpha * sum over the wrapped
// offsets o of w(p, o) (phi(o) - 1) (dinv .* src)(p + o), accumulated in C.
// RMW: dst(p) += out (planar block, ld ldd); else corr(t) = out (ld ldd).
// colscale (RMW only; may be null): out(j) is multiplied by colscale[j].
template <typename T, typename C, bool RMW>
__global__ __launch_bounds__(kThreads) void k_bloch(FixArgs a, const double* __restrict__ V,
                                                    const double* __restrict__ dinv, double alpha,
                                                    const double* __restrict__ colscale,
                                                    const T* __restrict__ src, int64_t lds,
                                                    const T* __restrict__ edge,
                                                    void* __restrict__ dstv, int64_t ldd,
                                                    int64_t b, int nbnd) {
  // XCD-aware order: consecutive workgroup ids on one XCD take consecutive
  // point blocks of one pair chunk, so the neighbour rows that nearby
  // boundary points share are hit in that XCD's L2
  const int nblk = gridDim.x, bid = blockIdx.x;
  const int q8 = nblk >> 3, r8 = nblk & 7, xcd = bid & 7, loc = bid >> 3;
  const int lin = xcd < r8 ? xcd * (q8 + 1) + loc : r8 * (q8 + 1) + (xcd - r8) * q8 + loc;
  const int ntb = (nbnd + kThreads - 1) / kThreads;
  const int chunk = lin / ntb;
  const int t = (lin - chunk * ntb) * kThreads + threadIdx.x;
  if (t >= nbnd) return;
  const int64_t j0 = int64_t(chunk) * kPairs;
  const int np = int(b - j0 < kPairs ? b - j0 : kPairs);
  int x, y, z;
  boundary_point(t, a.nx, a.ny, a.nz, &x, &y, &z);
  const int nxy = a.nx * a.ny;
  const int p = x + a.nx * y + nxy * z;
  const double vp = a.field2 ? V[p] : 0.0;
  const T* s0 = src + j0 * lds;
  // x-face points (inner y and z): every wrapped neighbour has x = nx-1 or 0
  // and is read from the compact row-end copy when there is one
  const bool from_edge = edge != nullptr && y > 0 && y < a.ny - 1 && z > 0 && z < a.nz - 1;
  const int64_t lde = int64_t(2) * a.ny * a.nz;
  const T* e0 = from_edge ? edge + j0 * lde : nullptr;
  const int64_t cs = from_edge ? lde : lds;                  // column stride of the gathers
  C accr[kPairs], acci[kPairs];
#pragma unroll
  for (int jj = 0; jj < kPairs; ++jj) accr[jj] = acci[jj] = C(0);
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    int qz = z + dz, wz = 0;
    if (qz < 0) {
      qz += a.nz;
      wz = -1;
    } else if (qz >= a.nz) {
      qz -= a.nz;
      wz = 1;
    }
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      int qy = y + dy, wy = 0;
      if (qy < 0) {
        qy += a.ny;
        wy = -1;
      } else if (qy >= a.ny) {
        qy -= a.ny;
        wy = 1;
      }
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        int qx = x + dx, wx = 0;
        if (qx < 0) {
          qx += a.nx;
          wx = -1;
        } else if (qx >= a.nx) {
          qx -= a.nx;
          wx = 1;
        }
        if ((wx | wy | wz) == 0) continue;
        // phi = prod_d exp(i w_d k_d n_d); g = alpha w (phi - 1) (times dinv(q))
        double fr = 1.0, fi = 0.0;
        if (wx) {
          const double cr = a.cw[0], ci = wx * a.sw[0];
          const double t0 = fr * cr - fi * ci;
          fi = fr * ci + fi * cr;
          fr = t0;
        }
        if (wy) {
          const double cr = a.cw[1], ci = wy * a.sw[1];
          const double t0 = fr * cr - fi * ci;
          fi = fr * ci + fi * cr;
          fr = t0;
        }
        if (wz) {
          const double cr = a.cw[2], ci = wz * a.sw[2];
          const double t0 = fr * cr - fi * ci;
          fi = fr * ci + fi * cr;
          fr = t0;
        }
        const int o = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
        const int q = qx + a.nx * qy + nxy * qz;
        double w = alpha * a.c[o];
        if (a.field2) w += alpha * a.hm[o] * (vp + V[q]);
        if (dinv) w *= dinv[q];
        const C gr = C(w * (fr - 1.0)), gi = C(w * fi);
        const T* sq = from_edge ? e0 + (int64_t(qz) * a.ny + qy) * 2 + (qx == 0 ? 0 : 1) : s0 + q;
        // all gathers first (columns past the last pair re-read the last
        // pair's and are discarded at the store), then the updates
        T ur[kPairs], ui[kPairs];
#pragma unroll
        for (int jj = 0; jj < kPairs; ++jj) {
          const int64_t jc = jj < np ? jj : np - 1;
          ur[jj] = sq[jc * cs];
          ui[jj] = sq[(b + jc) * cs];
        }
#pragma unroll
        for (int jj = 0; jj < kPairs; ++jj) {
          const C vr = C(load_el<T>(ur[jj])), vi = C(load_el<T>(ui[jj]));
          accr[jj] += gr * vr - gi * vi;
          acci[jj] += gr * vi + gi * vr;
        }
      }
    }
  }
  if constexpr (RMW) {
    T* d0 = static_cast<T*>(dstv) + j0 * ldd + p;
    T dr[kPairs], di[kPairs];
#pragma unroll
    for (int jj = 0; jj < kPairs; ++jj) {
      const int64_t jc = jj < np ? jj : np - 1;
      dr[jj] = d0[jc * ldd];
      di[jj] = d0[(b + jc) * ldd];
    }
#pragma unroll
    for (int jj = 0; jj < kPairs; ++jj) {
      if (jj < np) {
        const double sc = colscale ? colscale[j0 + jj] : 1.0;
        d0[jj * ldd] = store_el<T>(load_el<T>(dr[jj]) + sc * double(accr[jj]));
        d0[(b + jj) * ldd] = store_el<T>(load_el<T>(di[jj]) + sc * double(acci[jj]));
      }
    }
  } else {
    C* c0 = static_cast<C*>(dstv) + j0 * ldd + t;
#pragma unroll
    for (int jj = 0; jj < kPairs; ++jj) {
      if (jj < np) {
        c0[jj * ldd] = accr[jj];
        c0[(b + jj) * ldd] = acci[jj];
      }
    }
  }
}

// edge (ld 2 ny nz per column) = the x = 0 and x = nx-1 values of each grid
// row of the planar block src (cols columns, ld lds)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bloch_edges(const T* __restrict__ src, int64_t lds,
                                                          int nx, int64_t nrows, int64_t cols,
                                                          T* __restrict__ edge) {
  const int64_t total = nrows * cols;
  for (int64_t idx = blockIdx.x * int64_t(kThreads) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kThreads) {
    const int64_t c = idx / nrows, r = idx - c * nrows;
    const T* row = src + c * lds + r * nx;
    edge[c * 2 * nrows + 2 * r] = row[0];
    edge[c * 2 * nrows + 2 * r + 1] = row[nx - 1];
  }
}

FixArgs fix_args(const chfsi_operator& op) {
  FixArgs a;
  for (int o = 0; o < 27; ++o) {
    a.c[o] = op.coef[o];
    a.hm[o] = op.field_mode == 2 ? 0.5 * op.coef_mass[o] : 0.0;
  }
  const int nd[3] = {op.nx, op.ny, op.nz};
  for (int d = 0; d < 3; ++d) {
    a.cw[d] = std::cos(op.bloch[d] * nd[d]);
    a.sw[d] = std::sin(op.bloch[d] * nd[d]);
  }
  a.nx = op.nx;
  a.ny = op.ny;
  a.nz = op.nz;
  a.field2 = op.field_mode == 2 ? 1 : 0;
  return a;
}

bool fix_ok(const chfsi_operator& op, int64_t pairs) {
  // 32-bit point indices
  return op.nx >= 3 && op.ny >= 3 && op.nz >= 3 && op.n < (int64_t(1) << 31) && pairs >= 1 &&
         pairs <= 65535 && (op.field_mode != 2 || op.field);
}

}  // namespace

int64_t bloch_boundary_points(int nx, int ny, int nz) {
  return int64_t(nx) * ny * nz - int64_t(nx - 2) * (ny - 2) * (nz - 2);
}

template <typename F>
hipError_t bloch_init(const double* R, int64_t ldr, int64_t n, int64_t b, double scale, F* RY,
                      F* RX, F* Yc, const Twist& tw, hipStream_t st, F* E) {
  k_binit<F><<<grid_for(n * b), kThreads, 0, st>>>(R, ldr, n, b, scale, RY, RX, Yc, E, tw);
  return hipGetLastError();
}

template <typename F>
hipError_t bloch_reconstruct(const F* RY, const double* dinv, const double* X, int64_t ldx,
                             const double* lamY, double* Yp, int64_t ldy, int64_t n, int64_t b,
                             const Twist& tw, hipStream_t st) {
  k_brecon<F><<<grid_for(n * b), kThreads, 0, st>>>(RY, dinv, X, ldx, lamY, Yp, ldy, n, b, tw);
  return hipGetLastError();
}

hipError_t bloch_to_planar(const double* Z, int64_t ldz, int64_t n, int64_t b, double* P,
                           const Twist& tw, hipStream_t st) {
  k_bto_planar<<<grid_for(n * b), kThreads, 0, st>>>(Z, ldz, n, b, P, tw);
  return hipGetLastError();
}

hipError_t bloch_from_planar(const double* P, int64_t n, int64_t b, double* Z, int64_t ldz,
                             const Twist& tw, hipStream_t st) {
  k_bfrom_planar<<<grid_for(n * b), kThreads, 0, st>>>(P, n, b, Z, ldz, tw);
  return hipGetLastError();
}

template <typename F>
hipError_t bloch_fix(const chfsi_operator& op, const double* dinv, double alpha, const F* src,
                     int64_t lds, F* dst, int64_t ldd, int64_t pairs, hipStream_t st,
                     const double* colscale, const F* edge) {
  if (!fix_ok(op, pairs) || lds < op.n || ldd < op.n) return hipErrorInvalidValue;
  const int64_t nb = bloch_boundary_points(op.nx, op.ny, op.nz);
  const dim3 grid(unsigned((nb + kThreads - 1) / kThreads * ((pairs + kPairs - 1) / kPairs)));
  // the correction accumulates in FP64 for FP64 blocks, else FP32
  using C = typename std::conditional<sizeof(F) == 8, double, float>::type;
  k_bloch<F, C, true><<<grid, kThreads, 0, st>>>(fix_args(op), op.field, dinv, alpha, colscale,
                                                 src, lds, edge, dst, ldd, pairs, int(nb));
  return hipGetLastError();
}

template <typename T, typename C>
hipError_t bloch_corr(const chfsi_operator& op, const double* dinv, double alpha, const T* src,
                      int64_t lds, const T* edge, C* corr, int64_t ldc, int64_t pairs,
                      hipStream_t st) {
  const int64_t nb = bloch_boundary_points(op.nx, op.ny, op.nz);
  if (!fix_ok(op, pairs) || lds < op.n || ldc < nb) return hipErrorInvalidValue;
  const dim3 grid(unsigned((nb + kThreads - 1) / kThreads * ((pairs + kPairs - 1) / kPairs)));
  k_bloch<T, C, false><<<grid, kThreads, 0, st>>>(fix_args(op), op.field, dinv, alpha, nullptr,
                                                  src, lds, edge, corr, ldc, pairs, int(nb));
  return hipGetLastError();
}

template hipError_t bloch_init<double>(const double*, int64_t, int64_t, int64_t, double, double*,
                                       double*, double*, const Twist&, hipStream_t, double*);
template hipError_t bloch_init<float>(const double*, int64_t, int64_t, int64_t, double, float*,
                                      float*, float*, const Twist&, hipStream_t, float*);
template hipError_t bloch_init<uint16_t>(const double*, int64_t, int64_t, int64_t, double,
                                         uint16_t*, uint16_t*, uint16_t*, const Twist&,
                                         hipStream_t, uint16_t*);
template hipError_t bloch_reconstruct<double>(const double*, const double*, const double*, int64_t,
                                              const double*, double*, int64_t, int64_t, int64_t,
                                              const Twist&, hipStream_t);
template hipError_t bloch_reconstruct<float>(const float*, const double*, const double*, int64_t,
                                             const double*, double*, int64_t, int64_t, int64_t,
                                             const Twist&, hipStream_t);
template hipError_t bloch_reconstruct<uint16_t>(const uint16_t*, const double*, const double*,
                                                int64_t, const double*, double*, int64_t, int64_t,
                                                int64_t, const Twist&, hipStream_t);
template hipError_t bloch_fix<double>(const chfsi_operator&, const double*, double, const double*,
                                      int64_t, double*, int64_t, int64_t, hipStream_t,
                                      const double*, const double*);
template hipError_t bloch_fix<float>(const chfsi_operator&, const double*, double, const float*,
                                     int64_t, float*, int64_t, int64_t, hipStream_t,
                                     const double*, const float*);
template hipError_t bloch_fix<uint16_t>(const chfsi_operator&, const double*, double,
                                        const uint16_t*, int64_t, uint16_t*, int64_t, int64_t,
                                        hipStream_t, const double*, const uint16_t*);
template <typename T>
hipError_t bloch_edges(const chfsi_operator& op, const T* src, int64_t lds, T* edge, int64_t cols,
                       hipStream_t st) {
  if (op.nx < 3 || lds < op.n || cols < 1) return hipErrorInvalidValue;
  const int64_t nrows = int64_t(op.ny) * op.nz;
  k_bloch_edges<T><<<grid_for(nrows * cols), kThreads, 0, st>>>(src, lds, op.nx, nrows, cols,
                                                                  edge);
  return hipGetLastError();
}

template hipError_t bloch_edges<double>(const chfsi_operator&, const double*, int64_t, double*,
                                        int64_t, hipStream_t);
template hipError_t bloch_corr<double, double>(const chfsi_operator&, const double*, double,
                                               const double*, int64_t, const double*, double*,
                                               int64_t, int64_t, hipStream_t);
template hipError_t bloch_corr<float, float>(const chfsi_operator&, const double*, double,
                                             const float*, int64_t, const float*, float*, int64_t,
                                             int64_t, hipStream_t);
template hipError_t bloch_corr<uint16_t, float>(const chfsi_operator&, const double*, double,
                                                const uint16_t*, int64_t, const uint16_t*, float*,
                                                int64_t, int64_t, hipStream_t);

}  // namespace chfsi
