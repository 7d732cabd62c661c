"""The C-ABI library loads and exports every entry point include/oqr.h declares (CPU only).

Calls here stop at host-side argument validation, before any HIP call, so the
suite runs without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oqr.h")

oqr = pytest.importorskip("paper_1401_5171_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(oqr_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(oqr.LIB_PATH):
        from paper_1401_5171_amd import build
        build.build(verbose=False)
    return oqr.lib()


def test_header_declares_the_paper_algorithms():
    names = declared_functions()
    for f in ("oqr_cholqr", "oqr_cholqr2", "oqr_chol_a", "oqr_eig_a", "oqr_gs", "oqr_cholqr2_batched",
              "oqr_workspace_bytes", "oqr_status_string", "oqr_check"):
        assert f in names


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 12
    for f in names:
        assert hasattr(L, f), f
    assert set(oqr.EXPORTS) <= set(names)


def test_status_strings(L):
    for code in range(7):
        assert oqr.status_string(code).startswith("OQR_")
    assert "unknown" in oqr.status_string(99)
    assert L.oqr_version() >= 100


def test_default_opts(L):
    o = oqr._Opts()
    L.oqr_default_opts(ctypes.byref(o))
    assert (o.pass1, o.pass2, o.shift_c, o.max_retries, o.gs_variant) == (0, 0, 1.0, 3, 0)


def _dense_op(m):
    op = oqr._Op()
    op.kind, op.dtype, op.a, op.lda = oqr.OQR_OP_DENSE, oqr.OQR_F64, 0x1000, m
    return op


@pytest.mark.parametrize("fn", ["oqr_cholqr", "oqr_cholqr2", "oqr_chol_a", "oqr_eig_a", "oqr_gs"])
def test_argument_errors_before_any_launch(L, fn):
    f = getattr(L, fn)
    op = _dense_op(10)
    fake = 0x10000
    # m < n
    assert f(ctypes.byref(op), fake, 10, 4, 5, fake * 2, 10, fake * 3, 5, None, fake * 4, 1 << 20, fake * 5, None) \
        == oqr.OQR_E_ARG
    # ldz < m
    assert f(ctypes.byref(op), fake, 5, 10, 4, fake * 2, 10, fake * 3, 4, None, fake * 4, 1 << 20, fake * 5, None) \
        == oqr.OQR_E_ARG
    # null info
    assert f(ctypes.byref(op), fake, 10, 10, 4, fake * 2, 10, fake * 3, 4, None, fake * 4, 1 << 20, None, None) \
        == oqr.OQR_E_ARG
    # n beyond the kernels' limit
    op2 = _dense_op(1000)
    assert f(ctypes.byref(op2), fake, 1000, 1000, 300, fake * 2, 1000, fake * 3, 300, None, fake * 4, 1 << 20,
             fake * 5, None) == oqr.OQR_E_UNSUPPORTED
    # overlapping Q and Z that are not the same matrix
    assert f(ctypes.byref(op), fake, 10, 10, 4, fake + 8, 10, fake * 3, 4, None, fake * 4, 1 << 20, fake * 5,
             None) == oqr.OQR_E_ARG


def test_noalloc_host_checks_before_any_launch(L):
    """oqr_cholqr2_noalloc: argument errors, and a request beyond its fixed scratch, are refused on the
    host before the scratch is looked up or anything is enqueued."""
    f = L.oqr_cholqr2_noalloc
    fake = 0x10000
    op = _dense_op(10)
    assert f(ctypes.byref(op), fake, 10, 4, 5, fake * 2, 10, fake * 3, 5, None, fake * 5, None) == oqr.OQR_E_ARG
    assert f(ctypes.byref(op), fake, 10, 10, 4, fake * 2, 10, fake * 3, 4, None, None, None) == oqr.OQR_E_ARG
    m, n = 30000, 256                      # W and A W of this shape alone exceed the scratch
    op2 = _dense_op(m)
    assert 2 * 8 * m * n > L.oqr_noalloc_scratch_bytes() == 64 << 20
    big = 1 << 40
    assert f(ctypes.byref(op2), big, m, m, n, 2 * big, m, 3 * big, n, None, 4 * big, None) == oqr.OQR_E_SCRATCH


def test_offset_reach_limits(L):
    """Leading dimensions or m beyond what 32-bit tile offsets reach over min(n, 256) columns (dense
    operator) or min(n, 64) (others), m + 32 included, are refused with OQR_E_UNSUPPORTED before any
    launch; the largest accepted values pass validation (they stop at the workspace check).  The fake
    operands lie 2^40 bytes apart, so that they do not overlap at these leading dimensions."""
    fake = 1 << 40
    op = _dense_op(1000)
    for n, ldz, rc in ((256, 1048575, oqr.OQR_E_WORKSPACE), (256, 1048576, oqr.OQR_E_UNSUPPORTED),
                       (8, 33554431, oqr.OQR_E_WORKSPACE), (8, 33554432, oqr.OQR_E_UNSUPPORTED)):
        assert L.oqr_cholqr2(ctypes.byref(op), fake, ldz, 1000, n, fake * 2, ldz, fake * 3, n, None, fake * 4, 0,
                             fake * 5, None) == rc, (n, ldz)
    st = oqr._Op()
    st.kind, st.nx, st.ny, st.nz, st.center, st.off = oqr.OQR_OP_STENCIL7, 2048, 2048, 1, 6.001, -1.0
    m = 2048 * 2048                      # n = 64: m + 32 beyond 4194303
    assert L.oqr_cholqr(ctypes.byref(st), fake, m, m, 64, fake * 2, m, fake * 3, 64, None, fake * 4, 0, fake * 5,
                        None) == oqr.OQR_E_UNSUPPORTED
    assert L.oqr_cholqr(ctypes.byref(st), fake, m, m, 8, fake * 2, m, fake * 3, 8, None, fake * 4, 0, fake * 5,
                        None) == oqr.OQR_E_WORKSPACE
    st.nx = 2047
    m = 2047 * 2048
    assert L.oqr_cholqr(ctypes.byref(st), fake, m, m, 64, fake * 2, m, fake * 3, 64, None, fake * 4, 0, fake * 5,
                        None) == oqr.OQR_E_WORKSPACE


def test_bad_options_rejected(L):
    op = _dense_op(10)
    o = oqr.make_opts()
    o.pass1 = 7
    assert L.oqr_cholqr(ctypes.byref(op), 0x10000, 10, 10, 4, 0x20000, 10, 0x30000, 4, ctypes.byref(o), 0x40000,
                        1 << 20, 0x50000, None) == oqr.OQR_E_ARG
    o = oqr.make_opts(shift_c=-1.0)
    assert L.oqr_cholqr(ctypes.byref(op), 0x10000, 10, 10, 4, 0x20000, 10, 0x30000, 4, ctypes.byref(o), 0x40000,
                        1 << 20, 0x50000, None) == oqr.OQR_E_ARG


def test_workspace_query(L):
    op = _dense_op(1000)
    for alg in ("cholqr", "cholqr2"):
        nb = L.oqr_workspace_bytes(oqr.ALG[alg], ctypes.byref(op), 1000, 64, None)
        assert nb >= 1000 * 64 * 8
    o = oqr.make_opts(pass1="bf16x3")
    assert L.oqr_workspace_bytes(oqr.ALG["cholqr2"], ctypes.byref(op), 1000, 64, ctypes.byref(o)) > \
        L.oqr_workspace_bytes(oqr.ALG["cholqr2"], ctypes.byref(op), 1000, 64, None)
    assert L.oqr_workspace_bytes(oqr.ALG["cholqr"], ctypes.byref(op), 10, 64, None) == 0   # m < n
    st = oqr._Op()
    st.kind, st.nx, st.ny, st.nz, st.center, st.off = oqr.OQR_OP_STENCIL7, 8, 8, 8, 6.001, -1.0
    assert L.oqr_workspace_bytes(oqr.ALG["cholqr2"], ctypes.byref(st), 512, 16, None) > 0
    assert L.oqr_workspace_bytes(oqr.ALG["cholqr2"], ctypes.byref(st), 500, 16, None) == 0   # m != nx ny nz


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        oqr.make_op(torch.eye(4, dtype=torch.float64))
