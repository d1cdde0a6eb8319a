"""The C-ABI library loads on a machine without a GPU and exports every
function that include/chfsi.h declares (no compute calls are made here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chfsi.h")
LIB = os.path.join(ROOT, "paper_2503_22652_amd", "libchfsi.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(chfsi_[a-z_]+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2503_22652_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("chfsi_create", "chfsi_filter", "chfsi_solve", "chfsi_submit",
                     "chfsi_rayleigh_ritz", "chfsi_wait", "chfsi_cancel", "chfsi_destroy",
                     "chfsi_workspace_bytes", "chfsi_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_exports_are_c_linkage():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (chfsi_[a-z_]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_version_and_error_strings_without_gpu(lib):
    lib.chfsi_version.restype = ctypes.c_char_p
    lib.chfsi_last_error.restype = ctypes.c_char_p
    assert b"gfx950" in lib.chfsi_version()
    assert isinstance(lib.chfsi_last_error(), bytes)


def test_workspace_bytes_rejects_bad_params_without_gpu():
    import paper_2503_22652_amd as P
    op = P.identity_operator(100)
    op.kind = P.OP_DENSE          # dense without a pointer: invalid
    prm = P.make_params(10, 20, 8, lambda_max=5.0)
    assert P.chfsi_workspace_bytes(op, None, prm) == 0
    st = P.stencil_operator((8, 8, 8), [0.0] * 27)
    assert P.chfsi_workspace_bytes(st, None, P.make_params(10, 20, 8, lambda_max=5.0)) > 0
    assert P.chfsi_workspace_bytes(st, None, P.make_params(30, 20, 8, lambda_max=5.0)) == 0


def test_bloch_operator_checks_without_gpu():
    """Host-side checks of the Bloch-phase grid kind (complex contexts)."""
    import paper_2503_22652_amd as P
    k = (0.3, -0.7, 1.1)
    coef = [0.0] * 27
    A = P.stencil_operator((8, 8, 8), coef, bloch=k)
    assert A.kind == P.OP_STENCIL27_BLOCH and tuple(A.bloch) == k

    def ws(B, **kw):
        kw.setdefault("method", P.METHOD_RCHFSI)
        return P.chfsi_workspace_bytes(A, B, P.make_params(10, 20, 8, lambda_max=5.0, **kw))

    f64, f32, bf16 = (ws(None, filter_prec=p) for p in (P.PREC_FP64, P.PREC_FP32, P.PREC_BF16))
    assert f64 > f32 > bf16 > 0          # planar filter blocks in the filter precision
    assert ws(P.stencil_operator((8, 8, 8), coef, bloch=k)) > f64    # B Y block
    # B on another wave vector, a real B, B on another grid, plain ChFSI, slab mode
    assert ws(P.stencil_operator((8, 8, 8), coef, bloch=(0.3, 0.0, 0.0))) == 0
    assert ws(P.stencil_operator((8, 8, 8), coef)) == 0
    assert ws(P.stencil_operator((8, 8, 4), coef, bloch=k)) == 0
    assert ws(None, method=P.METHOD_CHFSI) == 0
    assert ws(None, memory_mode=1) == 0
    nan = P.stencil_operator((8, 8, 8), coef, bloch=(float("nan"), 0.0, 0.0))
    assert P.chfsi_workspace_bytes(nan, None, P.make_params(10, 20, 8, lambda_max=5.0)) == 0
    nofield = P.stencil_operator((8, 8, 8), coef, field_mode=2, bloch=k)   # mode 2 without V
    assert P.chfsi_workspace_bytes(nofield, None, P.make_params(10, 20, 8, lambda_max=5.0)) == 0


def test_exact_inverse_parameter_checks_without_gpu():
    """binv_exact needs dense A and B, the plain filter and FP64."""
    import paper_2503_22652_amd as P
    A = P.identity_operator(64)
    A.kind, A.dense, A.ld = P.OP_DENSE, 0x1000, 64     # never dereferenced by the size query
    B = P.identity_operator(64)
    B.kind, B.dense, B.ld = P.OP_DENSE, 0x2000, 64

    def ws(B_, **kw):
        return P.chfsi_workspace_bytes(A, B_, P.make_params(8, 16, 8, lambda_max=5.0, **kw))

    plain = ws(B, method=P.METHOD_CHFSI, filter_prec=P.PREC_FP64)
    exact = ws(B, method=P.METHOD_CHFSI, filter_prec=P.PREC_FP64, binv_exact=1)
    assert exact >= plain + 64 * 64 * 8 > 0
    assert ws(None, method=P.METHOD_CHFSI, filter_prec=P.PREC_FP64, binv_exact=1) == 0
    assert ws(B, method=P.METHOD_RCHFSI, filter_prec=P.PREC_FP64, binv_exact=1) == 0
    assert ws(B, method=P.METHOD_CHFSI, filter_prec=P.PREC_FP32, binv_exact=1) == 0
    assert ws(B, method=P.METHOD_CHFSI, filter_prec=P.PREC_FP64, binv_exact=2) == 0


def test_leading_dimension_of_blocks_without_gpu():
    """The binding passes a block's column stride as its leading dimension.
    A single column's stride is arbitrary (numpy reports any value for a size-1
    dimension), so its leading dimension is its length; a row-major block is
    refused rather than read with the wrong layout."""
    import numpy as np
    torch = pytest.importorskip("torch")
    import paper_2503_22652_amd as P
    one = torch.from_numpy(np.ascontiguousarray(np.zeros((37, 1)).T)).t()
    assert P._ld(one) == 37
    assert P._ld(torch.empty((5, 40), dtype=torch.float64).t()) == 40
    assert P._ld(torch.empty((5, 48), dtype=torch.float64).t()[:40]) == 48
    with pytest.raises(ValueError):
        P._ld(torch.empty((40, 5), dtype=torch.float64))
    with pytest.raises(ValueError):
        P._ld(torch.empty((80, 1), dtype=torch.float64)[::2])
