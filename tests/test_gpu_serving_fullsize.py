"""The serving stream's requests at their own sizes, through the server,
against LAPACK.

Each request is built as the Poisson serving workload builds it: a dense
generalized pencil with N from the stream's size set, k = 5% of N wanted
pairs, block ceil(1.25 k / 16) * 16, degree 20, FP32 residual filter with the
FP64 Rayleigh-Ritz, residual tolerance 1e-8.  Two steps of one sequence run:
a cold start, then A + 1e-3 ||A|| E (E a unit-norm symmetric perturbation)
warm-started from the first step's subspace.  The k lowest eigenvalues of
both steps must match LAPACK's (scipy.linalg.eigh on the host copies), and
the warm start must not take more iterations than the cold one.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2503_22652_amd as P  # noqa: E402
from workloads import gpu as wg  # noqa: E402


def _request(A, B, dinv, k, b, lmax, seq, seed):
    req = P.chfsi_request()
    req.A = P.dense_operator(A)
    req.B = P.dense_operator(B)
    req.d_inv = dinv.data_ptr()
    req.params = P.make_params(k, b, 20, max_iter=60, tol=1e-8, method=P.METHOD_RCHFSI,
                               filter_prec=P.PREC_FP32, lambda_max=lmax, seed=seed)
    req.seq_id = seq
    return req


@pytest.mark.parametrize("n", [1024, 4096, 8192])
def test_serving_sequence_at_stream_sizes(n):
    k = int(math.ceil(0.05 * n))
    b = int(math.ceil(1.25 * k / 16) * 16)
    A, B, dinv, lam = wg.dense_problem(n, k, 3000 + n)
    lmax = 10.0 / (0.95 * float(1.0 / dinv.max())) + 0.1
    normA = float(lam.abs().max())
    Bh = B.cpu().numpy()
    srv = P.Server(slots=2)
    its = []
    for t in range(2):
        if t > 0:
            E = wg.unit_perturbation(n, 4000 + n)
            A = (A + 1e-3 * normA * E).t().contiguous().t()
            del E
        torch.cuda.synchronize()
        print("serving request n", n, "k", k, "b", b, "step", t, flush=True)
        r = srv.wait(srv.submit(_request(A, B, dinv, k, b, lmax, 11, 5000 + t), keep=(A, B, dinv)))
        assert r["status"] == P.OK
        assert r["max_residual"] <= 1e-8
        w = sla.eigh(A.cpu().numpy(), Bh, eigvals_only=True, subset_by_index=[0, k - 1])
        got = np.asarray(r["evals"][:k])
        err = np.max(np.abs(got - w)) / np.max(np.abs(w))
        print("  iterations", r["iterations"], "max eigenvalue error / max |lambda|", err,
              flush=True)
        assert err <= 1e-10
        its.append(r["iterations"])
    srv.close()
    assert its[1] <= its[0]
