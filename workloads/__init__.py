"""Seeded synthetic inputs for the Chebyshev-filtered eigensolver workloads.

This module builds *problem inputs only*: matrices with a prescribed
spectrum, mass/stiffness stencil coefficients, a Gaussian-well potential and
random starting blocks.  It holds none of the eigensolver's arithmetic (no
Chebyshev filter, no Rayleigh-Ritz, no residuals), so both the CPU oracle and
the GPU library can consume what it produces without sharing method code.

Every generator draws from ``numpy.random.default_rng(seed)`` in a fixed,
documented order so that a (config, seed) pair always yields the same arrays.

Workload families (sizes are parameters so that tests can shrink them):

* ``dense_standard``   -- A = Q diag(lam) Q^T with Q a product of seeded
  Householder reflectors (the dense standard problem; B = I).
* ``dense_generalized`` -- the same A together with B = D + eps*S, D diagonal
  U[0.5, 2], S = (G + G^T)/2, eps chosen so that ||D^{-1} eps S||_2 equals a
  target (the approximate inverse of B is then D^{-1}).
* ``stencil_problem``  -- a periodic tensor-product Q1 finite-element pencil:
  stiffness/mass 27-point coefficients and a potential made of Gaussian wells.
* ``dense_hermitian`` -- the complex Hermitian counterpart of
  ``dense_generalized`` (complex reflectors, complex Hermitian S, real D).
* ``toy_standard`` / ``toy_generalized`` -- the paper's controlled dense
  experiments (Section 4.1): prescribed spectra, a QR-generated orthogonal
  basis and a unit-norm symmetric perturbation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "householder_vectors", "apply_householder_similarity", "dense_from_spectrum",
    "cfg0_spectrum", "cfg1_spectrum", "dense_standard", "dense_generalized",
    "stencil_coefficients_1d", "tensor_stencil_27", "gaussian_wells",
    "stencil_problem", "random_block", "unit_sym_perturbation",
    "toy_standard", "toy_generalized", "DenseProblem", "StencilProblem",
    "serving_schedule", "complex_householder_vectors", "hermitian_from_spectrum",
    "dense_hermitian", "random_block_complex",
]


# ----------------------------------------------------------------------------
# dense problems with a prescribed spectrum
# ----------------------------------------------------------------------------

def householder_vectors(rng: np.random.Generator, n: int, count: int) -> np.ndarray:
    """Draw ``count`` reflector vectors v_i ~ N(0,1)^n (columns), in order."""
    return np.stack([rng.standard_normal(n) for _ in range(count)], axis=1)


def apply_householder_similarity(M: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Return Q M Q^T with Q = H_1 H_2 ... H_c, H_i = I - 2 v_i v_i^T / (v_i^T v_i).

    Applied reflector by reflector from the innermost one outwards, so the cost
    is O(c n^2) instead of forming Q.  Works in place on a copy of M.
    """
    A = np.array(M, dtype=np.float64, copy=True)
    for i in range(V.shape[1] - 1, -1, -1):
        v = V[:, i]
        beta = 2.0 / float(v @ v)
        # left: H A = A - beta v (v^T A)
        w = v @ A
        A -= beta * np.outer(v, w)
        # right: A H = A - beta (A v) v^T
        u = A @ v
        A -= beta * np.outer(u, v)
    return 0.5 * (A + A.T)


def dense_from_spectrum(lam: np.ndarray, V: np.ndarray) -> np.ndarray:
    return apply_householder_similarity(np.diag(np.asarray(lam, dtype=np.float64)), V)


def cfg0_spectrum(rng: np.random.Generator, n: int, n_low: int = 32,
                  low: tuple = (-1.0, -0.2), high: float = 10.0) -> np.ndarray:
    """n_low eigenvalues evenly spaced in [low0, low1], the rest U[0, high) sorted."""
    j = np.arange(n_low, dtype=np.float64)
    lo = low[0] + (low[1] - low[0]) * j / max(n_low - 1, 1)
    rest = np.sort(rng.uniform(0.0, high, size=n - n_low))
    return np.concatenate([lo, rest])


def cfg1_spectrum(rng: np.random.Generator, n: int, n_low: int = 256) -> np.ndarray:
    return cfg0_spectrum(rng, n, n_low=n_low, low=(-1.0, -0.1))


@dataclass
class DenseProblem:
    """A dense symmetric(-definite) eigenproblem A x = lambda B x."""
    A: np.ndarray
    B: Optional[np.ndarray]          # None: standard problem (B = I)
    dinv: Optional[np.ndarray]       # diagonal approximate inverse of B (None: I)
    lam_A: np.ndarray                # spectrum of A (ascending)
    n_wanted: int
    block: int
    degree: int
    tol: float
    eps: float = 0.0                 # scale of the off-diagonal part of B
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]


def dense_standard(n: int = 1024, n_low: int = 32, block: int = 40, degree: int = 16,
                   tol: float = 1e-10, seed: int = 1000, n_refl: int = 8) -> DenseProblem:
    """Dense standard problem (the N=1024 / 32 wanted / block 40 / degree 16 workload).

    Draw order: the ``n_refl`` reflector vectors, then the n - n_low uniforms.
    """
    rng = np.random.default_rng(seed)
    V = householder_vectors(rng, n, n_refl)
    lam = cfg0_spectrum(rng, n, n_low=n_low)
    A = dense_from_spectrum(lam, V)
    return DenseProblem(A=A, B=None, dinv=None, lam_A=lam, n_wanted=n_low, block=block,
                        degree=degree, tol=tol, meta={"seed": seed, "n_refl": n_refl})


def _sigma_max_power(S: np.ndarray, dinv: np.ndarray, seed: int = 12345) -> float:
    """Largest singular value of diag(dinv) S (Lanczos on M^T M, fixed start vector).

    Used only to scale the generated B; it is part of input construction.
    """
    from scipy.sparse.linalg import LinearOperator, eigsh
    n = S.shape[0]
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(n)

    def mtm(x):
        x = np.asarray(x).reshape(-1)
        y = dinv * (S @ x)
        return S @ (dinv * y)

    op = LinearOperator((n, n), matvec=mtm, dtype=np.float64)
    w = eigsh(op, k=1, which="LA", v0=v0, tol=1e-13, return_eigenvectors=False)
    return float(math.sqrt(w[0]))


def dense_generalized(n: int = 8192, n_low: int = 256, block: int = 320, degree: int = 20,
                      tol: float = 1e-8, seed: int = 1001, n_refl: int = 8,
                      target: float = 0.05, sigma_max: Optional[float] = None) -> DenseProblem:
    """Dense generalized problem (the N=8192 / 256 wanted / block 320 / degree 20 workload).

    Draw order: reflector vectors, the n - n_low uniforms of the spectrum of A,
    the n diagonal entries D ~ U[0.5, 2], then G ~ N(0,1)^{n x n} (row-major).
    S = (G + G^T)/2 and eps = target / sigma_max(D^{-1} S), so that
    ||D^{-1} eps S||_2 = target.  The approximate inverse is D^{-1}.
    """
    rng = np.random.default_rng(seed)
    V = householder_vectors(rng, n, n_refl)
    lam = cfg1_spectrum(rng, n, n_low=n_low)
    d = rng.uniform(0.5, 2.0, size=n)
    G = rng.standard_normal((n, n))
    S = G
    S += G.T.copy()
    S *= 0.5
    dinv = 1.0 / d
    if sigma_max is None:
        sigma_max = _sigma_max_power(S, dinv)
    eps = target / sigma_max
    B = S
    B *= eps
    B[np.diag_indices(n)] += d
    A = dense_from_spectrum(lam, V)
    return DenseProblem(A=A, B=B, dinv=dinv, lam_A=lam, n_wanted=n_low, block=block,
                        degree=degree, tol=tol, eps=eps,
                        meta={"seed": seed, "sigma_max": sigma_max, "target": target,
                              "dmin": float(d.min()), "dmax": float(d.max())})


# ----------------------------------------------------------------------------
# complex Hermitian problems (Section 4.3)
# ----------------------------------------------------------------------------

def complex_householder_vectors(rng: np.random.Generator, n: int, count: int) -> np.ndarray:
    """``count`` complex reflector vectors v_i = a_i + i b_i, a_i, b_i ~ N(0,1)^n,
    drawn in the order a_1, b_1, a_2, b_2, ... (columns)."""
    cols = []
    for _ in range(count):
        a = rng.standard_normal(n)
        b = rng.standard_normal(n)
        cols.append(a + 1j * b)
    return np.stack(cols, axis=1)


def hermitian_from_spectrum(lam: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Q diag(lam) Q^H with Q = H_1 ... H_c, H_i = I - 2 v_i v_i^H / (v_i^H v_i)
    (each H_i is Hermitian and unitary), applied reflector by reflector."""
    A = np.diag(np.asarray(lam, dtype=np.complex128))
    for i in range(V.shape[1] - 1, -1, -1):
        v = V[:, i]
        beta = 2.0 / float(np.real(np.vdot(v, v)))
        w = v.conj() @ A                  # v^H A
        A -= beta * np.outer(v, w)
        u = A @ v                         # A v
        A -= beta * np.outer(u, v.conj())
    return 0.5 * (A + A.conj().T)


def _sigma_max_power_complex(S: np.ndarray, dinv: np.ndarray, seed: int = 12345) -> float:
    """Largest singular value of diag(dinv) S for Hermitian complex S (Lanczos on
    M^H M from a fixed start vector); input construction only."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    n = S.shape[0]
    v0 = np.random.default_rng(seed).standard_normal(n).astype(np.complex128)

    def mhm(x):
        x = np.asarray(x).reshape(-1)
        y = dinv * (S @ x)
        return S @ (dinv * y)

    op = LinearOperator((n, n), matvec=mhm, dtype=np.complex128)
    w = eigsh(op, k=1, which="LA", v0=v0, tol=1e-13, return_eigenvectors=False)
    return float(math.sqrt(abs(w[0])))


def dense_hermitian(n: int = 8192, n_low: int = 256, block: int = 320, degree: int = 20,
                    tol: float = 1e-8, seed: int = 1003, n_refl: int = 8,
                    target: float = 0.05, generalized: bool = True) -> DenseProblem:
    """Complex Hermitian counterpart of ``dense_generalized`` (Section 4.3).

    Draw order: the complex reflector vectors, the n - n_low uniforms of the
    spectrum (as ``cfg1_spectrum``), then (generalized) the n diagonal entries
    D ~ U[0.5, 2] and G = G_r + i G_i with G_r, G_i ~ N(0,1)^{n x n}
    (row-major, G_r first).  A = Q Lambda Q^H; B = D + eps S with
    S = (G + G^H)/2 and eps = target / sigma_max(D^{-1} S), so that
    ||D^{-1} eps S||_2 = target; the approximate inverse is the real D^{-1}.
    With ``generalized=False`` B = I and D^{-1} = I.
    """
    rng = np.random.default_rng(seed)
    V = complex_householder_vectors(rng, n, n_refl)
    lam = cfg1_spectrum(rng, n, n_low=n_low)
    A = hermitian_from_spectrum(lam, V)
    if not generalized:
        return DenseProblem(A=A, B=None, dinv=None, lam_A=lam, n_wanted=n_low, block=block,
                            degree=degree, tol=tol, meta={"seed": seed, "complex": True})
    d = rng.uniform(0.5, 2.0, size=n)
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    S = 0.5 * (G + G.conj().T)
    dinv = 1.0 / d
    sigma_max = _sigma_max_power_complex(S, dinv)
    eps = target / sigma_max
    B = eps * S
    B[np.diag_indices(n)] += d
    return DenseProblem(A=A, B=B, dinv=dinv, lam_A=lam, n_wanted=n_low, block=block,
                        degree=degree, tol=tol, eps=eps,
                        meta={"seed": seed, "sigma_max": sigma_max, "target": target,
                              "dmin": float(d.min()), "dmax": float(d.max()), "complex": True})


def random_block_complex(n: int, b: int, seed: int) -> np.ndarray:
    """Complex start block: real parts N(0,1)^{n x b} then imaginary parts, each
    drawn as in ``random_block``."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((b, n)).T
    im = rng.standard_normal((b, n)).T
    return np.asfortranarray(re + 1j * im)


def random_block(n: int, b: int, seed: int) -> np.ndarray:
    """Starting block X0 ~ N(0,1)^{n x b}, column-major (Fortran order) float64."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((b, n)).T)


def unit_sym_perturbation(rng: np.random.Generator, n: int) -> np.ndarray:
    """E = (F + F^T)/2, F ~ N(0,1)^{n x n}, normalised to ||E||_2 = 1."""
    F = rng.standard_normal((n, n))
    E = 0.5 * (F + F.T)
    w = np.linalg.eigvalsh(E)
    return E / max(abs(w[0]), abs(w[-1]))


# ----------------------------------------------------------------------------
# the paper's controlled dense experiments (Section 4.1)
# ----------------------------------------------------------------------------

def _qr_orthogonal(rng: np.random.Generator, m: int) -> np.ndarray:
    G = rng.standard_normal((m, m))
    Q, R = np.linalg.qr(G)           # Householder QR (LAPACK geqrf/orgqr)
    return Q


def toy_spectrum(m: int = 1000, n: int = 10) -> np.ndarray:
    j = np.arange(1, m + 1, dtype=np.float64)
    lam = np.where(j <= n, 1.0 + 3.0 * (j - 1) / (n - 1), 5.0 + 0.2 * (j - n - 1))
    return lam


def toy_standard(m: int = 1000, n: int = 10, eps: float = 0.0, seed: int = 0,
                 pert_seed: int = 1):
    """Standard toy problem: A = Q diag(lam) Q^T, filter matrix A~ = A + eps E."""
    rng = np.random.default_rng(seed)
    Q = _qr_orthogonal(rng, m)
    lam = toy_spectrum(m, n)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    E = unit_sym_perturbation(np.random.default_rng(pert_seed), m)
    return {"A": A, "A_filter": A + eps * E, "lam": lam, "Q": Q}


def toy_generalized(m: int = 1000, n: int = 10, zeta: float = 0.0, seed: int = 0,
                    pert_seed: int = 1):
    """Generalized toy problem with shared eigenbasis; D^{-1} = B^{-1} + zeta E."""
    rng = np.random.default_rng(seed)
    Q = _qr_orthogonal(rng, m)
    lam = toy_spectrum(m, n)
    bj = 1.0 + 4.0 * np.arange(m, dtype=np.float64) / (m - 1)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    B = (Q * bj) @ Q.T
    B = 0.5 * (B + B.T)
    Binv = (Q / bj) @ Q.T
    Binv = 0.5 * (Binv + Binv.T)
    E = unit_sym_perturbation(np.random.default_rng(pert_seed), m)
    return {"A": A, "B": B, "Binv": Binv, "Dinv": Binv + zeta * E,
            "lam_gen": lam / bj, "Q": Q, "bj": bj}


def toy_diagonal_mass(m: int = 1000, n: int = 10, seed: int = 0, mass_seed: int = 1):
    """Toy spectrum for A (as ``toy_standard``) with a diagonal mass matrix.

    B = diag(b), b ~ U[1, 5] (kappa(B) <= 5, the range of Section 4.1.1), so
    the diagonal D^{-1} = B^{-1} is exact and a reduced-precision filter is
    the only source of filtering error.
    """
    rng = np.random.default_rng(seed)
    Q = _qr_orthogonal(rng, m)
    lam = toy_spectrum(m, n)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    b = np.random.default_rng(mass_seed).uniform(1.0, 5.0, size=m)
    return {"A": A, "B": np.diag(b), "Binv": np.diag(1.0 / b), "dinv": 1.0 / b}


# ----------------------------------------------------------------------------
# periodic Q1 finite-element stencil pencils
# ----------------------------------------------------------------------------

def stencil_coefficients_1d():
    """1D linear-element stiffness and mass stencils at offsets (-1, 0, +1), h = 1."""
    K1 = np.array([-1.0, 2.0, -1.0])
    M1 = np.array([1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0])
    return K1, M1


def tensor_stencil_27(kind: str) -> np.ndarray:
    """27 coefficients c[dz+1, dy+1, dx+1] of the 3D tensor-product operator.

    kind = "mass":      M1 (x) M1 (x) M1
    kind = "stiffness": K1(x)M1(x)M1 + M1(x)K1(x)M1 + M1(x)M1(x)K1
    These describe the problem (its matrices), not the solver.
    """
    K1, M1 = stencil_coefficients_1d()
    if kind == "mass":
        return np.einsum("i,j,k->ijk", M1, M1, M1)
    if kind == "stiffness":
        return (np.einsum("i,j,k->ijk", K1, M1, M1) + np.einsum("i,j,k->ijk", M1, K1, M1)
                + np.einsum("i,j,k->ijk", M1, M1, K1))
    raise ValueError(kind)


def gaussian_wells(shape, n_wells: int, rng: np.random.Generator,
                   depth=(1.0, 5.0), width=(2.0, 4.0)):
    """Potential V(r) = -sum_w d_w exp(-|r - c_w|^2 / (2 s_w^2)) on a periodic grid.

    Draw order per the workload recipe: all centres (n_wells x 3, U[0, n_d)),
    then all depths U[depth], then all widths U[width].  Distances use the
    periodic minimum image; grid points are integer (h = 1).  Returns V with
    shape (nz, ny, nx) and index x + nx*(y + ny*z).
    """
    nz, ny, nx = shape
    centres = rng.uniform(0.0, 1.0, size=(n_wells, 3)) * np.array([nx, ny, nz], dtype=np.float64)
    depths = rng.uniform(depth[0], depth[1], size=n_wells)
    widths = rng.uniform(width[0], width[1], size=n_wells)
    V = np.zeros((nz, ny, nx), dtype=np.float64)
    xs = np.arange(nx, dtype=np.float64)
    ys = np.arange(ny, dtype=np.float64)
    zs = np.arange(nz, dtype=np.float64)

    def mi(a, c, L):
        d = np.abs(a - c)
        return np.minimum(d, L - d)

    for w in range(n_wells):
        cx, cy, cz = centres[w]
        s2 = 2.0 * widths[w] ** 2
        gx = np.exp(-mi(xs, cx, nx) ** 2 / s2)
        gy = np.exp(-mi(ys, cy, ny) ** 2 / s2)
        gz = np.exp(-mi(zs, cz, nz) ** 2 / s2)
        V -= depths[w] * (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
    return V, {"centres": centres, "depths": depths, "widths": widths}


@dataclass
class StencilProblem:
    """Periodic grid pencil A = 0.5 K + P_V, B = M, approximate inverse D^{-1} = I.

    ``coef_A`` are the 27 coefficients of 0.5 K, ``coef_B`` those of M, and the
    potential term is either the lumped diagonal V (field_mode 1, "R1") or the
    mass-weighted 1/2 (diag(V) M + M diag(V)) (field_mode 2, "R2").
    """
    shape: tuple
    coef_A: np.ndarray
    coef_B: np.ndarray
    V: np.ndarray
    field_mode: int
    n_wanted: int
    block: int
    degree: int
    tol: float
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))


def stencil_problem(grid: int = 128, n_wells: int = 64, n_wanted: int = 1000, block: int = 1200,
                    degree: int = 30, tol: float = 1e-8, seed: int = 1002,
                    field_mode: int = 2) -> StencilProblem:
    """The 27-point periodic FE pencil (128^3 / 64 wells, or 160^3 / 200 wells)."""
    rng = np.random.default_rng(seed)
    shape = (grid, grid, grid)
    V, info = gaussian_wells(shape, n_wells, rng)
    return StencilProblem(shape=shape, coef_A=0.5 * tensor_stencil_27("stiffness"),
                          coef_B=tensor_stencil_27("mass"), V=V, field_mode=field_mode,
                          n_wanted=n_wanted, block=block, degree=degree, tol=tol,
                          meta={"seed": seed, "n_wells": n_wells, **info})


# ----------------------------------------------------------------------------
# sparse (CSR) pencils
# ----------------------------------------------------------------------------

def grid_pencil_csr(shape, coef_A: np.ndarray, coef_B: np.ndarray, V: np.ndarray,
                    field_mode: int):
    """The periodic 27-point grid pencil (A, B) assembled as scipy CSR matrices.

    Entry (i, j) of a stencil operator is the coefficient of the offset from
    grid point i to grid point j (periodic wrap; offsets that wrap onto the
    same point on grids of width 1 or 2 add up).  The potential term: field_mode
    1 adds V_i on the diagonal, field_mode 2 adds B_ij (V_i + V_j) / 2."""
    import scipy.sparse as sp
    nz, ny, nx = shape
    n = nx * ny * nz
    idx = np.arange(n).reshape(nz, ny, nx)

    def assemble(coef):
        rows, cols, vals = [], [], []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    c = coef[dz + 1, dy + 1, dx + 1]
                    if c == 0.0:
                        continue
                    nb = np.roll(idx, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
                    rows.append(idx.reshape(-1))
                    cols.append(nb.reshape(-1))
                    vals.append(np.full(n, c))
        M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(n, n)).tocsr()
        M.sum_duplicates()
        return M

    A, B = assemble(coef_A), assemble(coef_B)
    v = np.asarray(V, dtype=np.float64).reshape(-1)
    if field_mode == 1:
        A = A + sp.diags(v)
    elif field_mode == 2:
        A = A + 0.5 * (sp.diags(v) @ B + B @ sp.diags(v))
    A, B = A.tocsr(), B.tocsr()
    A.sort_indices()
    B.sort_indices()
    return A, B


def random_sparse_pencil(n: int, per_row: int, long_rows: int, long_len: int, seed: int):
    """A random symmetric sparse A (about per_row entries per row plus `long_rows`
    rows and columns of `long_len` entries, values N(0,1), diagonal N(0,1) + 2)
    and an SPD diagonally dominant sparse B = I + 0.05 S (S symmetric, random
    pattern); CSR, sorted indices.  D^{-1} = 1 / diag(B)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    r = rng.integers(0, n, n * per_row // 2)
    c = rng.integers(0, n, n * per_row // 2)
    lr = rng.choice(n, long_rows, replace=False)
    r = np.concatenate([r, np.repeat(lr, long_len)])
    c = np.concatenate([c, rng.integers(0, n, long_rows * long_len)])
    G = sp.coo_matrix((rng.standard_normal(r.size), (r, c)), shape=(n, n)).tocsr()
    A = (0.5 * (G + G.T) + sp.diags(rng.standard_normal(n) + 2.0)).tocsr()
    r2 = rng.integers(0, n, 2 * n)
    c2 = rng.integers(0, n, 2 * n)
    H = sp.coo_matrix((rng.uniform(-1.0, 1.0, r2.size), (r2, c2)), shape=(n, n)).tocsr()
    S = 0.5 * (H + H.T)
    rowsum = np.asarray(abs(S).sum(axis=1)).reshape(-1)
    B = (sp.eye(n) + 0.05 * (S + sp.diags(rowsum))).tocsr()
    A.sort_indices()
    B.sort_indices()
    return A, B, 1.0 / B.diagonal()


# ----------------------------------------------------------------------------
# serving workload
# ----------------------------------------------------------------------------

def serving_schedule(n_requests: int = 512, n_seq: int = 64, rate: float = 200.0,
                     sizes=(512, 1024, 2048, 4096, 8192), seed: int = 5000):
    """Poisson arrival times and per-sequence sizes of the serving stream.

    Request i belongs to sequence i mod n_seq and is its step i // n_seq.
    Returns (arrival_seconds[n_requests], size_per_sequence[n_seq]).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes_seq = rng.choice(np.asarray(sizes), size=n_seq)
    return arrivals, sizes_seq
