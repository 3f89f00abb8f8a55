"""The autotuner's cache and argument checks on the host (no GPU needed):
the key of a size class, the JSON cache round trip, and validation."""
import ctypes as C
import json
import os

import pytest

from paper_1912_05508_amd import _lib as L

FAKE = C.c_void_p(0x1000)   # never dereferenced


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_1912_05508_amd import build
        build.build()
    return L.load()


@pytest.fixture()
def host_handle(lib):
    h = C.c_void_p()
    assert lib.qrx_create(C.byref(h), -1) == 0
    yield h
    assert lib.qrx_destroy(h) == 0


def test_key_is_the_size_class(lib):
    assert L.tune_key("gfx950", 32768, 4096, "fp16") == "gfx950/fp16/gram/m15/n12"
    # ceil(log2): one more row moves to the next class, a power of two stays
    assert L.tune_key("gfx950", 32769, 4096, "fp16") == "gfx950/fp16/gram/m16/n12"
    assert L.tune_key("gfx950", 65536, 8192, "fp16x3", "tsqr") == "gfx950/fp16x3/tsqr/m16/n13"
    assert L.tune_key("gfx950", 4096, 256, "bf16", "batched") == "gfx950/bf16/batched/m12/n8"
    buf = C.create_string_buffer(8)
    assert lib.qrx_tune_key(b"gfx950", 10, 5, 1, 0, buf, 8) == L.QRX_EINVAL      # too short
    assert lib.qrx_tune_key(b"gfx950", 10, 5, 7, 0, buf, 8) == L.QRX_EINVAL      # precision
    assert lib.qrx_tune_key(b'gf"x', 10, 5, 1, 0, C.create_string_buffer(64), 64) == L.QRX_EINVAL


def test_cache_round_trip(lib, tmp_path):
    path = str(tmp_path / "tune.json")
    k1 = L.tune_key("gfx950", 32768, 4096, "fp16")
    k2 = L.tune_key("gfx950", 4096, 256, "bf16", "batched")
    assert L.tune_cache_get(path, k1) is None               # no file yet
    L.tune_cache_put(path, k1, 64, 128, 0, 256, 13.25)
    L.tune_cache_put(path, k2, 32, 64, 0, 0, 42.5)
    r = L.tune_cache_get(path, k1)
    assert (r["panel_width"], r["cutoff"], r["gemm_tiles"], r["split_target"]) == (64, 128, 0, 256)
    assert r["ms"] == pytest.approx(13.25) and r["from_cache"] == 1 and r["trials"] == 0
    # replacing an entry keeps the others
    L.tune_cache_put(path, k1, 32, 256, 1, 512, 12.0)
    r = L.tune_cache_get(path, k1)
    assert (r["panel_width"], r["cutoff"], r["gemm_tiles"], r["split_target"]) == (32, 256, 1, 512)
    assert L.tune_cache_get(path, k2)["cutoff"] == 64
    assert L.tune_cache_get(path, "gfx950/fp32/gram/m1/n1") is None
    # the file is JSON
    doc = json.load(open(path))
    assert sorted(e["key"] for e in doc["qrx_tune"]) == sorted([k1, k2])
    assert not os.path.exists(path + ".tmp")


def test_cache_refuses_foreign_files(lib, tmp_path):
    path = tmp_path / "other.json"
    path.write_text('{"something": 1}\n')
    r = L.qrx_tune_result()
    assert lib.qrx_tune_cache_get(str(path).encode(), b"k", C.byref(r)) == L.QRX_EINVAL
    assert lib.qrx_tune_cache_put(str(path).encode(), b"k", C.byref(r)) == L.QRX_EINVAL
    assert path.read_text() == '{"something": 1}\n'            # left as it was
    good = tmp_path / "c.json"
    assert lib.qrx_tune_cache_put(str(good).encode(), b'bad"key', C.byref(r)) == L.QRX_EINVAL
    assert lib.qrx_tune_cache_get(None, b"k", C.byref(r)) == L.QRX_EINVAL


def test_tune_validates_before_device_work(lib, host_handle):
    r = L.qrx_tune_result()
    o = L.qr_opts("fp16")
    assert lib.qrx_tune(None, 100, 10, FAKE, 100, C.byref(o), 3, None, C.byref(r), None) == L.QRX_EINVAL
    assert lib.qrx_tune(host_handle, 100, 10, FAKE, 99, C.byref(o), 3, None, C.byref(r), None) == L.QRX_EINVAL
    assert lib.qrx_tune(host_handle, 100, 10, FAKE, 100, C.byref(o), 0, None, C.byref(r), None) == L.QRX_EINVAL
    assert lib.qrx_tune(host_handle, 100, 10, FAKE, 100, C.byref(o), 21, None, C.byref(r), None) == L.QRX_EINVAL
    bad = L.qr_opts("fp16")
    bad.gemm_tiles = 3
    assert lib.qrx_tune(host_handle, 100, 10, FAKE, 100, C.byref(bad), 3, None, C.byref(r), None) == L.QRX_EINVAL
    # valid arguments reach the device stage: a host-only handle has none
    assert lib.qrx_tune(host_handle, 100, 10, FAKE, 100, C.byref(o), 3, None, C.byref(r), None) == L.QRX_EHIP
    m = (C.c_int64 * 2)(100, 60)
    n = (C.c_int64 * 2)(10, 20)
    lda = (C.c_int64 * 2)(100, 60)
    A = (C.c_void_p * 2)(0x1000, 0x2000)
    ob = L.qr_opts("bf16")
    cut, til = (C.c_int * 2)(), (C.c_int * 2)()
    assert lib.qrx_tune_batched(host_handle, 2, m, n, A, lda, C.byref(ob), 3, None, cut, til,
                                C.byref(r), None) == L.QRX_EHIP
    assert lib.qrx_tune_batched(host_handle, 2, m, n, A, lda, C.byref(ob), 3, None, None, til,
                                C.byref(r), None) == L.QRX_EINVAL
    ob.split_target = 256                     # not a batched option
    assert lib.qrx_tune_batched(host_handle, 2, m, n, A, lda, C.byref(ob), 3, None, cut, til,
                                C.byref(r), None) == L.QRX_EINVAL
