"""Per-column parity bounds for the filter tests (test helper, not a test module).

Every filtered column is compared with the oracle's column against its own
scale, never one Frobenius norm over the block: filtered columns differ in
size by orders of magnitude, and a wrong small column would hide in a block
norm.

The scale of column j is
  * the residual part ||D^{-1} R_Y,j|| of the oracle's result for the
    reduced-precision residual filters (Algorithm 3): its rounding touches only
    that part, and Theorem 3.4 bounds the filtering error by a multiple of the
    residual it carries;
  * the oracle column's own norm for FP64 filters and for the plain filter
    (Algorithm 2), whose rounding touches the whole column.

The bound on |Y_gpu,j - Y_oracle,j| / scale_j is G u sqrt(K p):
  u  unit roundoff of the rounding that dominates: 2^-53 (FP64), 2^-24 (FP32
     blocks and products), 2^-8 (bfloat16 storage or bfloat16 product inputs);
  p  the degree (p steps, each adding fresh rounding; independent errors add
     in quadrature);
  K  terms summed per element of one operator product in FP32/FP64 (the
     standard sqrt(K) growth of random rounding errors in a dot product):
     n for a dense operator, 81 for a grid operator (three 27-point sums with
     the mass-weighted potential).  For bfloat16 the rounding of stored or
     rounded inputs dominates and is not summed in a dot product's order, so
     K = 1;
  G  growth factor: 1 for FP32, 8 for FP64, 3 for bfloat16.
Calibration (tests/test_parity_bounds.py, FP32/bfloat16 arithmetic emulated
on the CPU): the measured ratio err / (u sqrt(K p)) is 0.2 for FP32 and at most
1.5 for bfloat16 over the dense and grid test shapes, so G leaves a margin of
about 5x (FP32) and 2x-8x (bfloat16).  A coefficient of one step wrong by
1e-3 (relative) moves the result by 7e-5 to 7e-4 of the residual part, well
above the FP32 and FP64 bounds at every test size.
"""
import math

import numpy as np

U = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16": 2.0 ** -8}
G = {"fp64": 8.0, "fp32": 1.0, "bf16": 3.0}
GRID_TERMS = 81


def bound(prec: str, degree: int, terms: int) -> float:
    """G u sqrt(K p) for precision 'fp64' | 'fp32' | 'bf16'."""
    k = 1 if prec == "bf16" else max(int(terms), 1)
    return G[prec] * U[prec] * math.sqrt(k * max(int(degree), 1))


def column_errors(got, ref, scale):
    """Per-column |got_j - ref_j| / scale_j (complex columns by their modulus)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    if got.ndim == 1:
        got, ref = got[:, None], ref[:, None]
    err = np.linalg.norm(got - ref, axis=0)
    scale = np.maximum(np.asarray(scale, dtype=np.float64).reshape(-1), 1e-300)
    return err / scale


def assert_columns(got, ref, scale, prec: str, degree: int, terms: int, label: str = "",
                   fp64_floor: bool = False):
    """Assert every column's error is within bound(prec, degree, terms) of its scale.

    fp64_floor: also allow the FP64 bound on the column's own norm (for blocks
    whose residual part is itself at FP64 rounding level, e.g. b = N)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    tol = bound(prec, degree, terms)
    if fp64_floor:
        if got.ndim == 1:
            got, ref = got[:, None], ref[:, None]
        scale = np.asarray(scale, dtype=np.float64).reshape(-1)
        scale = scale + bound("fp64", degree, terms) / tol * np.linalg.norm(ref, axis=0)
    r = column_errors(got, ref, scale)
    print(f"{label} {prec} p={degree} K={terms}: max column err/scale {r.max():.3e} "
          f"(bound {tol:.3e}, ratio {r.max() / tol:.3f})", flush=True)
    assert np.all(np.isfinite(r)), label
    assert np.all(r <= tol), (label, float(r.max()), tol, int(np.argmax(r)))
    return r


def residual_part(RYp, dinv=None):
    """Per-column norm of D^{-1} R_Y (the reduced-precision part of Algorithm 3's result)."""
    R = np.asarray(RYp)
    if dinv is not None:
        R = np.asarray(dinv)[:, None] * R
    return np.linalg.norm(R, axis=0)


def prec_name(code: int) -> str:
    return {0: "fp64", 1: "fp32", 2: "bf16"}[int(code)]
