"""The autotuner on the GPU: it returns parameters from its candidate sets,
stores them in the JSON cache, reads them back without measuring, and the
tuned factorisation keeps the accuracy of its precision."""
import json

import numpy as np
import pytest

import synth
from oracle import metrics as M

from gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qrx():
    import torch
    assert torch.cuda.is_available()
    import paper_1912_05508_amd as P
    h = P.Handle()
    yield h
    h.close()


def test_tune_qr_and_cache(qrx, tmp_path):
    import torch
    p = synth.scaled_config("c2", 4096, 1024, seed=2)
    A = dev(p.A)
    before = A.clone()
    cache = str(tmp_path / "tune.json")
    r = qrx.tune(A, prec="fp16", cache=cache, reps=2)
    print(r)
    assert torch.equal(A, before)                      # the input is not modified
    assert r["from_cache"] == 0 and r["trials"] >= 5 and r["ms"] > 0
    assert r["panel_width"] in (32, 64) and r["cutoff"] in (64, 128, 256, 512)
    assert r["gemm_tiles"] in (0, 1) and r["split_target"] in (0, 128, 256, 512, 1024)
    doc = json.load(open(cache))
    assert len(doc["qrx_tune"]) == 1 and doc["qrx_tune"][0]["key"].endswith("/fp16/gram/m12/n10")
    r2 = qrx.tune(A, prec="fp16", cache=cache, reps=2)
    assert r2["from_cache"] == 1 and r2["trials"] == 0
    for k in ("panel_width", "cutoff", "gemm_tiles", "split_target"):
        assert r2[k] == r[k]
    kw = {k: r[k] for k in ("panel_width", "cutoff", "gemm_tiles", "split_target")}
    Q, R, st = qrx.qr(A, prec="fp16", **kw)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert M.qr_backward_error(p.A, host(Q), host(R)) < 4e-3


def test_tune_batched(qrx, tmp_path):
    # per size class (ceil log2 m, ceil log2 n): a cutoff and a product tile for
    # each class, cached per class; the tuned batch keeps the BF16 accuracy
    import torch
    g = np.random.default_rng(3)
    mats = []
    for i in range(24):
        n = int(8 * g.integers(4, 17))
        m = int(n * g.integers(4, 9))
        mats.append(dev(g.standard_normal((m, n)).astype(np.float32)))
    copies = [a.clone() for a in mats]
    cache = str(tmp_path / "tune.json")
    r = qrx.tune_batched(mats, prec="bf16", cache=cache, reps=2)
    print(r)
    assert all(torch.equal(a, b) for a, b in zip(mats, copies))
    assert all(c in (32, 64, 128, 256) for c in r["cutoff"]) and len(r["cutoff"]) == 24
    assert all(t in (0, 1) for t in r["tiles"]) and r["trials"] >= 2 and r["from_cache"] == 0
    classes = {(int(np.ceil(np.log2(a.shape[0]))), int(np.ceil(np.log2(a.shape[1])))) for a in mats}
    doc = json.load(open(cache))
    assert len(doc["qrx_tune"]) == len(classes)
    # problems of one class share their values
    by_class = {}
    for a, c, t in zip(mats, r["cutoff"], r["tiles"]):
        key = (int(np.ceil(np.log2(a.shape[0]))), int(np.ceil(np.log2(a.shape[1]))))
        assert by_class.setdefault(key, (c, t)) == (c, t)
    r2 = qrx.tune_batched(mats, prec="bf16", cache=cache, reps=2)
    assert r2["from_cache"] == 1 and r2["trials"] == 0
    assert r2["cutoff"] == r["cutoff"] and r2["tiles"] == r["tiles"]
    Qs, Rs, st = qrx.qr_batched(mats, prec="bf16", cutoff=r["cutoff"], tiles=r["tiles"])
    torch.cuda.synchronize()
    assert st == [0] * len(mats)
    for A0, Q, R in zip(copies, Qs, Rs):
        assert M.qr_backward_error(host(A0), host(Q), host(R)) < 3e-2
