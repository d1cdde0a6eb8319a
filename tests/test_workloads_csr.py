"""The CSR grid pencil of the input generator equals the oracle's stencil
operators (every field_mode, ragged grids and the smallest grid), is
symmetric, and the random sparse pencil has an SPD B and rows longer than the
LDS-staged kernel's limit (so both CSR kernels are exercised)."""
import numpy as np
import pytest

import workloads as wl
from oracle import stencil


@pytest.mark.parametrize("shape", [(5, 6, 7), (3, 3, 3), (4, 9, 10)])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_grid_pencil_csr_equals_stencil(shape, mode):
    rng = np.random.default_rng(3)
    V, _ = wl.gaussian_wells(shape, 2, rng)
    cA = 0.5 * wl.tensor_stencil_27("stiffness")
    cB = wl.tensor_stencil_27("mass")
    A, B = wl.grid_pencil_csr(shape, cA, cB, V, mode)
    aA, aB = stencil.make_ops(cA, cB, V, shape, mode)
    n = int(np.prod(shape))
    X = rng.standard_normal((n, 4))
    assert np.abs(A @ X - aA(X)).max() < 1e-13
    assert np.abs(B @ X - aB(X)).max() < 1e-13
    assert abs(A - A.T).max() == 0.0 and abs(B - B.T).max() == 0.0


def test_random_sparse_pencil():
    A, B, dinv = wl.random_sparse_pencil(400, 8, 3, 120, 5)
    assert abs(A - A.T).max() == 0.0 and abs(B - B.T).max() == 0.0
    assert np.diff(A.indptr).max() > 80
    assert np.linalg.eigvalsh(B.toarray()).min() > 0.5
    np.testing.assert_allclose(dinv, 1.0 / B.diagonal())
