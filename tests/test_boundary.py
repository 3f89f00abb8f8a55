"""The C-ABI library: builds, loads, exports every declared symbol, and rejects
bad arguments on the host before any device work (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qrx.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1912_05508_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1912_05508_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qrx_[a-z_A-Z0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("qrx_create", "qrx_destroy", "qrx_qr_factor", "qrx_lls_solve",
                 "qrx_lls_solve_with_R", "qrx_qr_workspace_size", "qrx_lls_workspace_size"):
        assert want in names


def test_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_1912_05508_amd import _lib
    assert set(_lib._SIGS) == set(declared_functions())


@pytest.fixture()
def host_handle(lib):
    h = C.c_void_p()
    assert lib.qrx_create(C.byref(h), -1) == 0     # host-only handle: validation / sizes
    yield h
    assert lib.qrx_destroy(h) == 0


def test_status_strings(lib):
    from paper_1912_05508_amd import _lib
    for code in (0, -1, -2, -3, 1, 2, 3):
        assert lib.qrx_status_string(code).decode().startswith("QRX_")
    assert _lib.status_string(99) == "unknown qrx status"


def test_null_handle_and_outputs(lib):
    from paper_1912_05508_amd import _lib
    sz = C.c_size_t()
    assert lib.qrx_create(None, 0) == _lib.QRX_EINVAL
    assert lib.qrx_destroy(None) == _lib.QRX_EINVAL
    assert lib.qrx_qr_workspace_size(None, 10, 5, None, C.byref(sz)) == _lib.QRX_EINVAL


FAKE = C.c_void_p(0x1000)   # never dereferenced: validation fails or the handle has no device


@pytest.mark.parametrize("m,n,lda,ldr", [(4, 5, 5, 5), (5, 0, 5, 1), (10, 3, 9, 3), (10, 3, 10, 2),
                                         (-1, 1, 1, 1)])
def test_qr_bad_sizes(lib, host_handle, m, n, lda, ldr):
    from paper_1912_05508_amd import _lib
    rc = lib.qrx_qr_factor(host_handle, m, n, FAKE, lda, FAKE, ldr, None, 0, None, None, None)
    assert rc == _lib.QRX_EINVAL


def test_qr_bad_pointers_and_options(lib, host_handle):
    from paper_1912_05508_amd import _lib
    L = _lib
    assert lib.qrx_qr_factor(host_handle, 10, 3, None, 10, FAKE, 3, None, 0, None, None, None) == L.QRX_EINVAL
    assert lib.qrx_qr_factor(host_handle, 10, 3, FAKE, 10, None, 3, None, 0, None, None, None) == L.QRX_EINVAL
    for field, val, panel in (("gemm_prec", 4, "gram"), ("gemm_prec", -1, "gram"),
                              ("panel_width", 129, "gram"), ("panel_width", 33, "tsqr"),
                              ("cutoff", -4, "gram"), ("block_rows", 128, "gram"),
                              ("no_col_scaling", 2, "gram"), ("panel_alg", 2, "gram"),
                              ("gemm_tiles", 2, "gram"), ("split_target", 8, "gram"),
                              ("split_target", 9000, "gram"), ("q_reorth", 2, "gram"),
                              ("q_reorth", -1, "gram")):
        o = L.qr_opts(panel=panel)
        setattr(o, field, val)
        assert lib.qrx_qr_factor(host_handle, 10, 3, FAKE, 10, FAKE, 3, None, 0, C.byref(o),
                                 None, None) == L.QRX_EINVAL, field
    # a valid call reaches the device stage and fails there on a host-only handle
    assert lib.qrx_qr_factor(host_handle, 10, 3, FAKE, 10, FAKE, 3, None, 0, None, None, None) == L.QRX_EHIP


def test_short_workspace(lib, host_handle):
    from paper_1912_05508_amd import _lib
    sz = C.c_size_t()
    assert lib.qrx_qr_workspace_size(host_handle, 1000, 100, None, C.byref(sz)) == 0
    assert sz.value > 0
    rc = lib.qrx_qr_factor(host_handle, 1000, 100, FAKE, 1000, FAKE, 100, FAKE, sz.value - 1,
                           None, None, None)
    assert rc == _lib.QRX_EINVAL
    rc = lib.qrx_qr_factor(host_handle, 1000, 100, FAKE, 1000, FAKE, 100, FAKE, sz.value,
                           None, None, None)
    assert rc == _lib.QRX_EHIP


def test_lls_bad_arguments(lib, host_handle):
    from paper_1912_05508_amd import _lib as L
    info = L.qrx_lls_info()
    call = lambda o, b=FAKE, x=FAKE, inf=C.byref(info): lib.qrx_lls_solve(
        host_handle, 50, 10, FAKE, 50, b, x, None, 0, o, inf, None)
    for field, val in (("tol", -1.0), ("tol", float("nan")), ("max_iter", -1), ("method", 2),
                       ("use_x0", 5)):
        o = L.lls_opts()
        setattr(o, field, val)
        assert call(C.byref(o)) == L.QRX_EINVAL, field
    o = L.lls_opts()
    assert call(C.byref(o), b=None) == L.QRX_EINVAL
    assert call(C.byref(o), x=None) == L.QRX_EINVAL
    assert call(C.byref(o), inf=None) == L.QRX_EINVAL
    assert call(C.byref(o)) == L.QRX_EHIP
    assert lib.qrx_lls_solve_with_R(host_handle, 50, 10, FAKE, 50, FAKE, 9, FAKE, FAKE, None, 0,
                                    C.byref(o), C.byref(info), None) == L.QRX_EINVAL
    sz = C.c_size_t()
    assert lib.qrx_lls_workspace_size(host_handle, 50, 10, C.byref(o), C.byref(sz)) == 0
    assert sz.value > 50 * 10 * 4


def test_timing_api_on_host_handle(lib, host_handle):
    from paper_1912_05508_amd import _lib as L
    assert lib.qrx_timing_enable(host_handle, 1) == 0
    arr = (L.qrx_kernel_stat * 4)()
    cnt = C.c_int()
    assert lib.qrx_timing_get(host_handle, arr, 4, C.byref(cnt)) == 0 and cnt.value == 0
    assert lib.qrx_timing_reset(host_handle) == 0


def test_product_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_1912_05508_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", txt).lower() or f == "build.py", f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith(".py"):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1912_05508_amd" not in txt and "synth" not in txt, f


def _i64(*v):
    return (C.c_int64 * len(v))(*v)


def test_batched_plan_validation(lib, host_handle):
    # a batch plan checks sizes and options on the host before any device work
    # (a host-only handle then stops at the device stage with QRX_EHIP)
    from paper_1912_05508_amd import _lib
    EINVAL, EHIP = _lib.QRX_EINVAL, _lib.QRX_EHIP
    m, n = _i64(100, 64, 300), _i64(40, 64, 256)
    plan = C.c_void_p()
    lo = _lib.lls_opts("bf16")
    assert lib.qrx_batch_plan_create(host_handle, 3, m, n, None, None, C.byref(lo), 1,
                                     C.byref(plan)) == EHIP
    assert lib.qrx_batch_plan_create(host_handle, 3, m, n, None, None, None, 0,
                                     C.byref(plan)) == EHIP
    for bad_m, bad_n in (((10,), (11,)), ((300,), (257,)), ((5,), (0,))):
        assert lib.qrx_batch_plan_create(host_handle, 1, _i64(*bad_m), _i64(*bad_n), None, None,
                                         None, 0, C.byref(plan)) == EINVAL
    assert lib.qrx_batch_plan_create(host_handle, 0, m, n, None, None, None, 0,
                                     C.byref(plan)) == EINVAL
    assert lib.qrx_batch_plan_create(host_handle, 3, m, n, None, None, None, 2,
                                     C.byref(plan)) == EINVAL
    for field, val in (("gemm_prec", 1), ("gemm_prec", 3), ("panel_alg", 1), ("panel_width", 16),
                       ("panel_single_pass", 1), ("node_reorth", 1), ("q_reorth", 1),
                       ("gemm_tiles", 2), ("split_target", 256)):
        o = _lib.lls_opts("fp32")
        setattr(o.qr, field, val)
        assert lib.qrx_batch_plan_create(host_handle, 3, m, n, None, None, C.byref(o), 0,
                                         C.byref(plan)) == EINVAL, field
    for field, val in (("method", 1), ("use_x0", 1), ("tol", -1.0)):
        o = _lib.lls_opts("bf16")
        setattr(o, field, val)
        assert lib.qrx_batch_plan_create(host_handle, 3, m, n, None, None, C.byref(o), 1,
                                         C.byref(plan)) == EINVAL, field
    # per-problem cutoffs and tiles
    assert lib.qrx_batch_plan_create(host_handle, 3, m, n, (C.c_int * 3)(64, 0, 32), None,
                                     None, 0, C.byref(plan)) == EINVAL
    assert lib.qrx_batch_plan_create(host_handle, 3, m, n, None, (C.c_int * 3)(0, 2, 1),
                                     None, 0, C.byref(plan)) == EINVAL
    assert lib.qrx_batch_plan_create(host_handle, 3, m, n, (C.c_int * 3)(64, 128, 32),
                                     (C.c_int * 3)(0, 1, 1), None, 0, C.byref(plan)) == EHIP
    sz = C.c_size_t()
    assert lib.qrx_batch_plan_workspace_size(None, C.byref(sz)) == EINVAL
    assert lib.qrx_batch_plan_destroy(None) == EINVAL
    ptrs = C.c_void_p(0x1000)
    assert lib.qrx_lls_solve_batched(host_handle, None, ptrs, ptrs, ptrs, ptrs, None, 0, ptrs,
                                     None) == EINVAL
    assert lib.qrx_qr_factor_batched(host_handle, None, ptrs, ptrs, ptrs, ptrs, None, 0, ptrs,
                                     None) == EINVAL


def test_binding_checks_fire_before_the_library():
    # the Python helpers validate dtype, device, size and layout of every buffer
    # before any library call: a wrong dtype would make the library read or write
    # past the end of the buffer
    import torch
    import paper_1912_05508_amd as P

    class NoLib:
        def __getattr__(self, name):
            raise AssertionError(f"library called: {name}")

    h = P.Handle.__new__(P.Handle)
    h.h = C.c_void_p(1)
    h.lib = NoLib()
    A = torch.zeros((8, 3), dtype=torch.float32).t().contiguous().t()
    b = torch.zeros(8, dtype=torch.float64)
    x = torch.zeros(3, dtype=torch.float64)
    info = torch.zeros(C.sizeof(P.qrx_lls_info), dtype=torch.uint8)
    for args in ((A, b, x, info), (A, b.float(), x, info), (A, b, x.float(), info),
                 (A, b[:5], x, info), (A.double(), b, x, info)):
        with pytest.raises(P.QrxArgumentError):
            h.lstsq_async(*args)
    with pytest.raises(P.QrxArgumentError):
        h.qr_out(A, A.clone(), torch.zeros((3, 3)), torch.zeros(1, dtype=torch.int32))
    with pytest.raises(P.QrxArgumentError):
        P._check_vec("b", torch.zeros(4, dtype=torch.float64), 5, torch.float64)
    h.h = None
