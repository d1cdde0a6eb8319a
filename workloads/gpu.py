"""Seeded GPU-side input construction for large / many-matrix workloads.

Same recipes as ``workloads/__init__.py`` (input construction only: no
eigensolver arithmetic), built with torch on the device so that streams of
thousands-square matrices (the serving workload) can be produced in
milliseconds.  Randomness comes from a seeded ``torch.Generator`` on the
device, so a (seed, size) pair reproduces the same matrices on the same
software stack.

* ``dense_problem``: A = Q diag(lam) Q^T with Q a product of 8 Householder
  reflectors (lowest k eigenvalues evenly in [-1, -0.1], the rest U[0, 10)),
  B = D + eps S with D = diag(U[0.5, 2]), S = (G + G^T)/2 and eps chosen so
  that ||D^{-1} eps S||_2 ~= 0.05 (largest singular value by power iteration).
* ``hermitian_problem``: the complex Hermitian counterpart of ``dense_problem``
  (complex reflectors v = a + i b, S = (G + G^H)/2 with complex Gaussian G,
  real D), as ``workloads.dense_hermitian`` builds on the host.
* ``unit_perturbation``: E = (F + F^T)/2 scaled to ||E||_2 ~= 1 (power iteration).
"""
from __future__ import annotations

import torch


def _gen(seed: int, device="cuda"):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _colmajor(M: torch.Tensor) -> torch.Tensor:
    """Column-major (Fortran-order) view with the same values."""
    return M.t().contiguous().t()


def _sym_norm2(M: torch.Tensor, g, iters: int = 40) -> float:
    x = torch.randn(M.shape[0], 1, dtype=M.dtype, device=M.device, generator=g)
    x /= torch.linalg.vector_norm(x)
    s = 0.0
    for _ in range(iters):
        y = M @ x
        s = float(torch.linalg.vector_norm(y))
        x = y / s
    return s


def dense_problem(n: int, k: int, seed: int, target: float = 0.05, device="cuda"):
    """Returns (A, B, dinv, lam_A) as float64 device tensors (A, B column-major)."""
    g = _gen(seed, device)
    dt = torch.float64
    V = torch.randn(n, 8, dtype=dt, device=device, generator=g)
    lo = -1.0 + 0.9 * torch.arange(k, dtype=dt, device=device) / max(k - 1, 1)
    hi, _ = torch.sort(torch.rand(n - k, dtype=dt, device=device, generator=g) * 10.0)
    lam = torch.cat([lo, hi])
    A = torch.diag(lam)
    for i in range(7, -1, -1):
        v = V[:, i:i + 1]
        beta = 2.0 / float((v * v).sum())
        A -= beta * v @ (v.t() @ A)
        A -= beta * (A @ v) @ v.t()
    A = 0.5 * (A + A.t())
    d = torch.rand(n, dtype=dt, device=device, generator=g) * 1.5 + 0.5
    G = torch.randn(n, n, dtype=dt, device=device, generator=g)
    S = 0.5 * (G + G.t())
    del G
    dinv = 1.0 / d
    # largest singular value of D^{-1} S: power iteration on S D^{-2} S
    x = torch.randn(n, 1, dtype=dt, device=device, generator=g)
    x /= torch.linalg.vector_norm(x)
    s2 = 0.0
    for _ in range(60):
        y = S @ (dinv[:, None] ** 2 * (S @ x))
        s2 = float(torch.linalg.vector_norm(y))
        x = y / s2
    eps = target / (s2 ** 0.5)
    B = S.mul_(eps)
    B.diagonal().add_(d)
    return _colmajor(A), _colmajor(B), dinv.contiguous(), lam


def hermitian_problem(n: int, k: int, seed: int, target: float = 0.05, device="cuda"):
    """Returns (A, B, dinv, lam_A): A, B complex128 column-major, dinv float64."""
    g = _gen(seed, device)
    dt, ct = torch.float64, torch.complex128
    V = torch.complex(torch.randn(n, 8, dtype=dt, device=device, generator=g),
                      torch.randn(n, 8, dtype=dt, device=device, generator=g))
    lo = -1.0 + 0.9 * torch.arange(k, dtype=dt, device=device) / max(k - 1, 1)
    hi, _ = torch.sort(torch.rand(n - k, dtype=dt, device=device, generator=g) * 10.0)
    lam = torch.cat([lo, hi])
    A = torch.diag(lam).to(ct)
    for i in range(7, -1, -1):
        v = V[:, i:i + 1]
        beta = 2.0 / float((v.conj() * v).real.sum())
        A -= beta * v @ (v.conj().t() @ A)
        A -= beta * (A @ v) @ v.conj().t()
    A = 0.5 * (A + A.conj().t())
    d = torch.rand(n, dtype=dt, device=device, generator=g) * 1.5 + 0.5
    G = torch.complex(torch.randn(n, n, dtype=dt, device=device, generator=g),
                      torch.randn(n, n, dtype=dt, device=device, generator=g))
    S = 0.5 * (G + G.conj().t())
    del G
    dinv = 1.0 / d
    x = torch.randn(n, 1, dtype=dt, device=device, generator=g).to(ct)
    x /= torch.linalg.vector_norm(x)
    s2 = 0.0
    for _ in range(60):
        y = S @ ((dinv[:, None] ** 2) * (S @ x))
        s2 = float(torch.linalg.vector_norm(y))
        x = y / s2
    eps = target / (s2 ** 0.5)
    B = S.mul_(eps)
    B.diagonal().add_(d)
    return _colmajor(A), _colmajor(B), dinv.contiguous(), lam


def unit_perturbation(n: int, seed: int, device="cuda", dtype=torch.float64) -> torch.Tensor:
    g = _gen(seed, device)
    F = torch.randn(n, n, dtype=dtype, device=device, generator=g)
    E = 0.5 * (F + F.t())
    del F
    E /= _sym_norm2(E, g)
    return E
