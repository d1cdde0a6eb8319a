"""Continuous-batching server on the GPU.

* A request's result is bitwise identical whether it runs alone or mixed with
  other requests on other streams (same kernels, same launch shapes).
* A sequence of perturbed matrices is warm-started from the previous Ritz
  vectors and needs fewer iterations than a cold start.
* Pending requests can be cancelled; requests that can never fit the
  device-memory budget are refused at submission.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2503_22652_amd as P  # noqa: E402


def _request(prob, lmax, seq_id=-1, X0=None, tol=1e-9, max_iter=60, prec=P.PREC_FP32):
    A = P.to_colmajor(prob.A)
    B = P.to_colmajor(prob.B)
    d = torch.from_numpy(prob.dinv).cuda()
    req = P.chfsi_request()
    req.A = P.dense_operator(A)
    req.B = P.dense_operator(B)
    req.d_inv = d.data_ptr()
    req.params = P.make_params(prob.n_wanted, prob.block, prob.degree, max_iter=max_iter, tol=tol,
                               method=P.METHOD_RCHFSI, filter_prec=prec, lambda_max=lmax)
    req.seq_id = seq_id
    keep = [A, B, d]
    if X0 is not None:
        Xd = P.to_colmajor(X0)
        req.X0 = Xd.data_ptr()
        keep.append(Xd)
    return req, keep


def _problems():
    out = []
    for i, n in enumerate((384, 512, 640)):
        p = wl.dense_generalized(n=n, n_low=12 + 4 * i, block=16 + 4 * i, degree=12, seed=40 + i)
        w = sla.eigvalsh(p.A, p.B)
        out.append((p, float(w[-1]) + 0.5, w))
    return out


def test_alone_equals_mixed_bitwise():
    probs = _problems()
    X0s = [wl.random_block(p.n, p.block, 90 + i) for i, (p, _, _) in enumerate(probs)]
    # alone: one slot, one request at a time
    alone = []
    srv = P.Server(slots=1)
    for (p, lmax, w), X0 in zip(probs, X0s):
        req, keep = _request(p, lmax, X0=X0)
        t = srv.submit(req, keep)
        alone.append(srv.wait(t))
    srv.close()
    # mixed: three slots, all submitted at once (plus extra load)
    srv = P.Server(slots=3)
    tickets = []
    for (p, lmax, w), X0 in zip(probs, X0s):
        req, keep = _request(p, lmax, X0=X0)
        tickets.append(srv.submit(req, keep))
    extra = []
    for (p, lmax, w), X0 in zip(probs, X0s):
        req, keep = _request(p, lmax, X0=X0[:, ::-1].copy())
        extra.append(srv.submit(req, keep))
    mixed = [srv.wait(t) for t in tickets]
    for t in extra:
        srv.wait(t)
    srv.close()
    for (p, lmax, w), a, m in zip(probs, alone, mixed):
        assert a["status"] == P.OK and m["status"] == P.OK
        assert a["evals"] == m["evals"]            # bitwise
        assert a["iterations"] == m["iterations"]
        rel = np.abs(np.asarray(m["evals"][: p.n_wanted]) - w[: p.n_wanted]) / np.maximum(
            np.abs(w[: p.n_wanted]), 1e-3 * abs(w[-1]))
        assert rel.max() < 1e-10


def test_warm_started_sequence():
    p = wl.dense_generalized(n=512, n_low=16, block=20, degree=12, seed=60)
    rng = np.random.default_rng(61)
    normA = np.abs(p.lam_A).max()
    srv = P.Server(slots=2)
    its = []
    A_t = p.A.copy()
    for t in range(3):
        if t > 0:
            A_t = A_t + 1e-3 * normA * wl.unit_sym_perturbation(rng, p.n)
        q = wl.DenseProblem(A=A_t, B=p.B, dinv=p.dinv, lam_A=p.lam_A, n_wanted=16, block=20,
                            degree=12, tol=1e-9)
        w = sla.eigvalsh(A_t, p.B)
        req, keep = _request(q, float(w[-1]) + 0.5, seq_id=7,
                             X0=wl.random_block(p.n, 20, 62) if t == 0 else None)
        r = srv.wait(srv.submit(req, keep))
        assert r["status"] == P.OK
        rel = np.abs(np.asarray(r["evals"][:16]) - w[:16]) / np.maximum(np.abs(w[:16]),
                                                                         1e-3 * abs(w[-1]))
        assert rel.max() < 1e-10
        its.append(r["iterations"])
    srv.close()
    assert its[1] < its[0] and its[2] < its[0]


def test_cancel_and_admission():
    p, lmax, w = _problems()[1]
    srv = P.Server(slots=1)
    req, keep = _request(p, lmax, X0=wl.random_block(p.n, p.block, 1))
    t1 = srv.submit(req, keep)
    req2, keep2 = _request(p, lmax, X0=wl.random_block(p.n, p.block, 2))
    t2 = srv.submit(req2, keep2)
    srv.cancel(t2)
    r2 = srv.wait(t2)
    r1 = srv.wait(t1)
    assert r1["status"] == P.OK
    assert r2["status"] in (P.ERR_CANCELLED, P.OK)   # it may have started before the cancel
    srv.close()
    tiny = P.Server(slots=1, memory_budget=1024)
    req3, keep3 = _request(p, lmax)
    with pytest.raises(P.ChfsiError) as e:
        tiny.submit(req3, keep3)
    assert e.value.status == P.ERR_NOMEM
    tiny.close()


def test_complex_requests_through_the_server():
    """Complex requests (a Bloch grid pencil and a dense Hermitian pencil) carry
    interleaved complex blocks: the server's start block, warm-start copy and
    X_out hold n x b complex values.  Results match LAPACK on the assembled
    pencils, and the warm-started second request of the grid sequence needs
    fewer iterations."""
    from oracle import stencil
    shape, k = (6, 8, 10), (0.3, -0.7, 1.1)
    V, _ = wl.gaussian_wells(shape, 1, np.random.default_rng(5))
    cA, cB = 0.5 * wl.tensor_stencil_27("stiffness"), wl.tensor_stencil_27("mass")
    apply_A, apply_B = stencil.make_ops_bloch(cA, cB, V, shape, 2, k)
    n = int(np.prod(shape))
    Ad, Bd = apply_A(np.eye(n)), apply_B(np.eye(n))
    w_grid = sla.eigh(Ad, Bd, eigvals_only=True, subset_by_index=(0, 5))
    Vd = torch.from_numpy(np.ascontiguousarray(V).reshape(-1)).cuda()
    hp = wl.dense_hermitian(n=517, n_low=20, block=28, degree=12, seed=83)
    w_herm = sla.eigh(hp.A, hp.B, eigvals_only=True, subset_by_index=(0, 19))
    Ah, Bh = P.to_colmajor_complex(hp.A), P.to_colmajor_complex(hp.B)
    dh = torch.from_numpy(hp.dinv).cuda()

    def grid_request(X0=None, X_out=None):
        req = P.chfsi_request()
        req.A = P.stencil_operator(shape, cA, coef_mass=cB, field=Vd, field_mode=2, bloch=k)
        req.B = P.stencil_operator(shape, cB, bloch=k)
        req.params = P.make_params(6, 12, 16, max_iter=100, tol=1e-10, method=P.METHOD_RCHFSI,
                                   filter_prec=P.PREC_BF16, lambda_max=18.5)
        req.seq_id = 7
        req.X0 = 0 if X0 is None else X0.data_ptr()
        req.X_out = 0 if X_out is None else X_out.data_ptr()
        return req

    herm = P.chfsi_request()
    herm.A = P.hermitian_operator(Ah)
    herm.B = P.hermitian_operator(Bh)
    herm.d_inv = dh.data_ptr()
    herm.params = P.make_params(20, 28, 12, max_iter=60, tol=1e-10, method=P.METHOD_RCHFSI,
                                filter_prec=P.PREC_FP32,
                                lambda_max=10.0 / (0.95 * hp.meta["dmin"]) + 0.1)
    herm.seq_id = -1
    herm.X0 = 0
    herm.X_out = 0

    X0 = P.to_colmajor_complex(wl.random_block_complex(n, 12, 9))
    Xo1, Xo2 = P.colmajor_empty_complex(n, 12), P.colmajor_empty_complex(n, 12)
    srv = P.Server(slots=2)
    t1 = srv.submit(grid_request(X0, Xo1), (Vd, X0, Xo1))
    th = srv.submit(herm, (Ah, Bh, dh))
    r1 = srv.wait(t1)
    t2 = srv.submit(grid_request(None, Xo2), (Vd, Xo2))     # warm start from the sequence
    r2 = srv.wait(t2)
    rh = srv.wait(th)
    srv.close()
    print("grid cold", r1["iterations"], "warm", r2["iterations"], "hermitian", rh["iterations"])
    for r in (r1, r2):
        assert r["status"] == P.OK
        assert np.max(np.abs(np.array(r["evals"][:6]) - w_grid)) <= 1e-10 * np.max(np.abs(w_grid))
    assert r2["iterations"] < r1["iterations"]
    assert rh["status"] == P.OK
    assert np.max(np.abs(np.array(rh["evals"][:20]) - w_herm)) <= 1e-10 * np.max(np.abs(w_herm))
    for Xo, r in ((Xo1, r1), (Xo2, r2)):
        X = Xo.cpu().numpy()[:, :6]
        lam = np.array(r["evals"][:6])
        assert np.linalg.norm(X.conj().T @ Bd @ X - np.eye(6)) <= 1e-9
        assert np.max(np.linalg.norm(Ad @ X - Bd @ X * lam[None, :], axis=0)) < 1e-9


def test_budget_accounting_and_steady_state_pools():
    """The budget charges each running request its workspace and block, and each
    sequence its warm-start block for as long as the sequence holds it.  With a
    budget that fits one running request plus both sequences' blocks, the two
    sequences' first requests run one after the other and the charge left when
    the server is idle is exactly the two warm-start blocks.  Later requests of
    the same sizes draw everything from the pools: no new chunk is allocated."""
    p = wl.dense_generalized(n=512, n_low=16, block=20, degree=12, seed=60)
    w = sla.eigvalsh(p.A, p.B)
    lmax = float(w[-1]) + 0.5
    req0, keep0 = _request(p, lmax, seq_id=1)
    ws = P.chfsi_workspace_bytes(req0.A, req0.B, req0.params)
    blk = p.n * p.block * 8
    budget = ws + blk + 2 * blk + 4096
    srv = P.Server(slots=2, memory_budget=budget)
    rs = []
    for sid in (1, 2):
        req, keep = _request(p, lmax, seq_id=sid, X0=wl.random_block(p.n, p.block, 70 + sid))
        rs.append(srv.submit(req, keep))
    out = [srv.wait(t) for t in rs]
    assert all(o["status"] == P.OK for o in out)
    # one after the other: the second starts when the first has finished
    assert out[1]["start_ms"] >= out[0]["finish_ms"] or out[0]["start_ms"] >= out[1]["finish_ms"]
    st = srv.stats()
    assert st["used"] == 2 * blk and st["sequence_bytes"] == 2 * blk
    chunks = (st["device_pool_chunks"], st["host_pool_chunks"])
    for t in range(3):                       # warm-started requests of both sequences
        ts = [srv.submit(*_request(p, lmax, seq_id=sid)) for sid in (1, 2)]
        for tk in ts:
            assert srv.wait(tk)["status"] == P.OK
    st2 = srv.stats()
    assert st2["used"] == 2 * blk
    assert (st2["device_pool_chunks"], st2["host_pool_chunks"]) == chunks
    srv.close()
