/*
 * Periodic 27-point grid pencil and the residual-based Chebyshev filter
 * (Algorithm 3) in FP64 on the CPU -- oracle.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/ and by the CPU baseline leg of
 * bench.py.  Plain loops, one column at a time, OpenMP over grid planes.  It
 * shares no code with the HIP library.
 *
 * Grid vectors have n = nx ny nz entries indexed x + nx (y + ny z); offsets
 * (dx, dy, dz) in {-1, 0, 1}^3 wrap periodically; coefficient of an offset:
 * coef[(dz + 1) 9 + (dy + 1) 3 + (dx + 1)].  The pencil is A = S_A + potential
 * term, with field_mode 0 (none), 1 (diag(V) x) or 2 (the mass-weighted
 * 1/2 (diag(V) M + M diag(V)) x, M given by coef_mass).
 *
 * Algorithm 3, per column j (Ritz value lambda_j, residual column y_j):
 *   e = (lmax - lT) / 2, c = (lmax + lT) / 2, sigma = sigma_1 = e / (lmin - c)
 *   R_Y = (sigma_1 / e) y_j, R_X = 0, L_X = 1, L_Y = (sigma_1 / e)(lambda_j - c)
 *   k = 2..p: sigma' = 1 / (2 / sigma_1 - sigma), a = 2 sigma' / e
 *             R_X = a A(D^{-1} R_Y) - a c R_Y - sigma sigma' R_X + a L_Y y_j
 *             L_X = a L_Y lambda_j - a c L_Y - sigma sigma' L_X
 *             swap (R_X, R_Y), swap (L_X, L_Y), sigma = sigma'
 *   out_j = D^{-1} R_Y + L_Y x_j
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int64_t wrap(int64_t i, int64_t n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

/* y = S x for one grid vector */
void o_stencil_apply(const double* coef, int nx, int ny, int nz, const double* x, double* y) {
#pragma omp parallel for collapse(2) schedule(static)
  for (int z = 0; z < nz; ++z)
    for (int yy = 0; yy < ny; ++yy)
      for (int xx = 0; xx < nx; ++xx) {
        double s = 0.0;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const double c = coef[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
              if (c == 0.0) continue;
              const int64_t i = wrap(xx + dx, nx) + (int64_t)nx * (wrap(yy + dy, ny) +
                                                                 (int64_t)ny * wrap(z + dz, nz));
              s += c * x[i];
            }
        y[xx + (int64_t)nx * (yy + (int64_t)ny * z)] = s;
      }
}

/* y = A x (S_A plus the potential term); t1, t2: scratch of n doubles */
void o_pencil_apply(const double* coef_A, const double* coef_mass, const double* V, int field_mode,
                    int nx, int ny, int nz, const double* x, double* y, double* t1, double* t2) {
  const int64_t n = (int64_t)nx * ny * nz;
  o_stencil_apply(coef_A, nx, ny, nz, x, y);
  if (field_mode == 1) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] += V[i] * x[i];
  } else if (field_mode == 2) {
    o_stencil_apply(coef_mass, nx, ny, nz, x, t1);   /* M x */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      t2[i] = V[i] * x[i];
      y[i] += 0.5 * V[i] * t1[i];
    }
    o_stencil_apply(coef_mass, nx, ny, nz, t2, t1);  /* M (V x) */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] += 0.5 * t1[i];
  }
}

/* Algorithm 3 on ncols columns; dinv NULL means D^{-1} = I.  Returns 0, or -1
 * if scratch memory could not be allocated. */
int o_rchfsi_filter(const double* coef_A, const double* coef_mass, const double* V,
                    int field_mode, int nx, int ny, int nz, const double* dinv, int64_t ncols,
                    const double* X, int64_t ldx, const double* ritz, const double* R, int64_t ldr,
                    double* Yp, int64_t ldy, double lmin, double lmax, double lT, int degree) {
  const int64_t n = (int64_t)nx * ny * nz;
  double* RX = (double*)malloc(sizeof(double) * n);
  double* RY = (double*)malloc(sizeof(double) * n);
  double* Z = (double*)malloc(sizeof(double) * n);
  double* AZ = (double*)malloc(sizeof(double) * n);
  double* t1 = (double*)malloc(sizeof(double) * n);
  double* t2 = (double*)malloc(sizeof(double) * n);
  if (!RX || !RY || !Z || !AZ || !t1 || !t2) {
    free(RX); free(RY); free(Z); free(AZ); free(t1); free(t2);
    return -1;
  }
  const double e = (lmax - lT) / 2.0, c = (lmax + lT) / 2.0;
  const double sigma1 = e / (lmin - c);
  for (int64_t j = 0; j < ncols; ++j) {
    const double* y = R + j * ldr;
    const double lam = ritz[j];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      RY[i] = (sigma1 / e) * y[i];
      RX[i] = 0.0;
    }
    double LX = 1.0, LY = (sigma1 / e) * (lam - c), sigma = sigma1;
    for (int k = 2; k <= degree; ++k) {
      const double sigma2 = 1.0 / (2.0 / sigma1 - sigma);
      const double a = 2.0 * sigma2 / e;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) Z[i] = dinv ? dinv[i] * RY[i] : RY[i];
      o_pencil_apply(coef_A, coef_mass, V, field_mode, nx, ny, nz, Z, AZ, t1, t2);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i)
        RX[i] = a * AZ[i] - a * c * RY[i] - sigma * sigma2 * RX[i] + a * LY * y[i];
      const double LN = a * LY * lam - a * c * LY - sigma * sigma2 * LX;
      double* tmp = RX;
      RX = RY;
      RY = tmp;
      LX = LY;
      LY = LN;
      sigma = sigma2;
    }
    double* out = Yp + j * ldy;
    const double* xj = X + j * ldx;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = (dinv ? dinv[i] * RY[i] : RY[i]) + LY * xj[i];
  }
  free(RX); free(RY); free(Z); free(AZ); free(t1); free(t2);
  return 0;
}

/* OpenMP threads a parallel region here uses */
#ifdef _OPENMP
#include <omp.h>
int o_threads(void) { return omp_get_max_threads(); }
#else
int o_threads(void) { return 1; }
#endif
