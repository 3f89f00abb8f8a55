"""GPU parity of the batched path (one persistent launch, one workgroup per
problem at a time off a device work queue) against the oracle, through the C
ABI: QR factors of uneven problems (FP32 and BF16 products, both product
tiles), per-problem statuses (including bad device descriptors), least-squares
solutions certified to eta_F <= 1e-10, and the batch recorded into a HIP graph."""
import numpy as np
import pytest

import synth
from oracle import householder as H
from oracle import lls as L
from oracle import metrics as M

from gpu_util import dev, dev64, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qrx():
    import torch
    assert torch.cuda.is_available()
    import paper_1912_05508_amd as P
    h = P.Handle()
    yield h
    h.close()


def _mixed_shapes():
    # ragged n (multiples of 8 and not), m = n, tall, the 256-column maximum,
    # and more rows than one 128-row update tile or one 64-row Gram chunk
    return [(1, 1), (8, 8), (17, 5), (40, 40), (100, 33), (130, 64), (300, 96), (257, 128),
            (1000, 129), (640, 160), (2048, 200), (256, 256), (3000, 256), (4096, 248)]


def _matrix(g, m, n, scale=True):
    A = g.standard_normal((m, n))
    if scale:
        A = A * 10.0 ** g.uniform(-2, 2, n)
    return np.asfortranarray(A.astype(np.float32))


@pytest.mark.parametrize("prec,be_bound,tiles", [("fp32", 2e-6, 0), ("bf16", 4e-3, 0),
                                                 ("bf16", 4e-3, 1)])
def test_batched_qr_matches_oracle(qrx, prec, be_bound, tiles):
    import torch
    g = np.random.default_rng(11)
    shapes = _mixed_shapes()
    mats = [_matrix(g, m, n) for m, n in shapes]
    Qs, Rs, st = qrx.qr_batched([dev(A) for A in mats], prec=prec, tiles=tiles)
    torch.cuda.synchronize()
    assert st == [0] * len(mats)
    u = 2.0 ** -24 if prec == "fp32" else 2.0 ** -8
    for A, Q, R in zip(mats, Qs, Rs):
        Qh, Rh = host(Q), host(R)
        n = A.shape[1]
        assert M.upper_triangular_ok(Rh)
        assert np.all(np.diag(Rh) > 0)
        be = M.qr_backward_error(A, Qh, Rh)
        assert be < be_bound, (A.shape, be)
        # R against the oracle's sign-normalised Householder R, column by column
        # (column scaling 10^[-2,2] makes a global norm meaningless); kappa of the
        # column-equilibrated matrix, which Gram-Schmidt does not see
        _, Ro = H.qr(A.astype(np.float64))
        cerr = np.linalg.norm(Rh - Ro, axis=0) / np.linalg.norm(Ro, axis=0)
        kappa = np.linalg.cond(A.astype(np.float64) / np.linalg.norm(A, axis=0))
        assert cerr.max() < max(1e-5, 50 * kappa * (6e-8 if prec == "fp32" else 4e-3)), A.shape
        if n > 1:
            # loss of orthogonality within 10 kappa u of the product precision
            # (Sec. 3.2.1), where that bound is below one
            orth = M.orthogonality(Qh)
            bound = max(1e-5, 10 * kappa * u)
            if bound < 1.0:
                assert orth < bound, (A.shape, orth, bound)


def test_batched_bad_descriptor_is_local(qrx):
    # a problem whose device descriptor is invalid (lda < m) reports QRX_EINVAL
    # and the others are solved
    import torch
    import paper_1912_05508_amd as P
    g = np.random.default_rng(14)
    mats = [_matrix(g, m, n, scale=False) for m, n in ((200, 40), (150, 30), (300, 64))]
    rhs = [g.standard_normal(A.shape[0]) for A in mats]
    At = [dev(A) for A in mats]
    bt = [dev64(b) for b in rhs]
    xs = [torch.zeros(A.shape[1], dtype=torch.float64, device="cuda") for A in mats]
    plan = qrx.plan_batched([A.shape for A in mats], prec="bf16", lls=True, tol=1e-10)
    try:
        info = P.info_tensor(3, device="cuda")
        lda = torch.tensor([200, 149, 300], dtype=torch.int64, device="cuda")   # 149 < m
        qrx.lstsq_batched_async(plan, qrx._ptrs(At, "cuda"), lda, qrx._ptrs(bt, "cuda"),
                                qrx._ptrs(xs, "cuda"), info)
        infos = P.read_info(info, 3)
    finally:
        plan.close()
    assert [i["status"] for i in infos] == [0, -1, 0]
    for k in (0, 2):
        assert M.eta_F(mats[k], rhs[k], host(xs[k])) <= 1.05e-10


def test_batched_lls_graph_replay_matches_eager(qrx):
    # the whole batch (fill of the queue head + one persistent kernel) records
    # into a HIP graph; replays give the eager x and info bit for bit
    import torch
    import paper_1912_05508_amd as P
    probs = synth.batched_problems(64, seed=5, nmin_j=4, nmax_j=32, kmin=2, kmax=8)
    At = [dev(p.A) for p in probs]
    bt = [dev64(p.b) for p in probs]
    xs = [torch.zeros(p.A.shape[1], dtype=torch.float64, device="cuda") for p in probs]
    plan = qrx.plan_batched([p.A.shape for p in probs], prec="bf16", lls=True, tol=1e-10,
                            max_iter=400)
    try:
        work = torch.empty(plan.work_bytes, dtype=torch.uint8, device="cuda")
        info = P.info_tensor(len(probs), device="cuda")
        Ap, bp, xp = (qrx._ptrs(v, "cuda") for v in (At, bt, xs))
        lda = torch.tensor([p.A.shape[0] for p in probs], dtype=torch.int64, device="cuda")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            qrx.lstsq_batched_async(plan, Ap, lda, bp, xp, info, work=work)
            torch.cuda.synchronize()
            xe = [x.clone() for x in xs]
            ie = info.clone()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                qrx.lstsq_batched_async(plan, Ap, lda, bp, xp, info, work=work)
        torch.cuda.synchronize()
        assert all(i["status"] == 0 for i in P.read_info(ie, len(probs)))
        for rep in range(3):
            for x in xs:
                x.zero_()
            info.zero_()
            g.replay()
            torch.cuda.synchronize()
            assert all(torch.equal(a, b) for a, b in zip(xs, xe)), f"replay {rep}"
            assert torch.equal(info, ie)
            # eager work between replays
            qrx.lstsq_batched(At[:8], bt[:8], prec="fp32")
            torch.cuda.synchronize()
        del g
    finally:
        plan.close()


def test_batched_status_per_problem(qrx):
    import torch
    g = np.random.default_rng(12)
    good = _matrix(g, 200, 48)
    nan = _matrix(g, 150, 40)
    nan[17, 3] = np.nan
    zero = _matrix(g, 120, 24)
    zero[:, 5] = 0.0
    mats = [good, nan, zero, good.copy()]
    Qs, Rs, st = qrx.qr_batched([dev(A) for A in mats], prec="bf16")
    torch.cuda.synchronize()
    assert st == [0, 2, 1, 0]                # OK, QRX_ENONFINITE, QRX_ESINGULAR, OK
    assert M.qr_backward_error(good, host(Qs[0]), host(Rs[0])) < 4e-3


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_batched_lls_reaches_1e10(qrx, prec):
    import torch
    probs = synth.batched_problems(48, seed=3, nmin_j=1, nmax_j=32, kmin=2, kmax=16)
    xs, infos = qrx.lstsq_batched([dev(p.A) for p in probs], [dev64(p.b) for p in probs],
                                  prec=prec, tol=1e-10, max_iter=400)
    torch.cuda.synchronize()
    worst = 0.0
    for p, x, info in zip(probs, xs, infos):
        xh = host(x)
        assert info["status"] == 0, (p.A.shape, info)
        eta = M.eta_F(p.A, p.b, xh)
        worst = max(worst, eta)
        assert eta <= 1.05e-10, (p.A.shape, eta, info)
        assert abs(info["eta_F"] - eta) <= 0.05 * eta + 1e-13
        xo, _, _ = L.lls_direct(p.A, p.b)
        # a 1e-10 backward error bounds the forward error by cond * 1e-10 (columns
        # scaled by up to 1e4 relative to each other)
        kappa = np.linalg.cond(p.A.astype(np.float64))
        assert M.forward_error(xh, xo) <= max(1e-8, 10 * kappa * 1e-10), p.A.shape
    print(f"{prec}: worst eta_F {worst:.2e}, iters {[i['iters'] for i in infos[:8]]}")


def test_batched_lls_deterministic_and_ragged(qrx):
    import torch
    g = np.random.default_rng(13)
    mats, rhs = [], []
    for m, n in ((33, 33), (65, 7), (700, 250), (129, 64)):
        A = _matrix(g, m, n, scale=False)
        _, b = synth.lls_problem(g, A, "rel1e-6")
        mats.append(A)
        rhs.append(b)
    r1 = qrx.lstsq_batched([dev(A) for A in mats], [dev64(b) for b in rhs], prec="bf16")
    r2 = qrx.lstsq_batched([dev(A) for A in mats], [dev64(b) for b in rhs], prec="bf16")
    torch.cuda.synchronize()
    for A, b, x1, x2, info in zip(mats, rhs, r1[0], r2[0], r1[1]):
        assert np.array_equal(host(x1), host(x2))
        assert info["status"] == 0
        xh = host(x1)
        if A.shape[0] > A.shape[1]:
            assert M.eta_F(A, b, xh) <= 1.05e-10
        else:
            # square: a compatible system, certified by ||r|| / (||A||_F ||x|| + ||b||)
            _, nr = M.eta(A, b, xh)
            assert nr / (M.fro(A) * np.linalg.norm(xh) + np.linalg.norm(b)) <= 1.05e-10


@pytest.mark.slow
def test_c4_full_batch(qrx):
    """The full 4096-problem batch (n = 8 U{4..32}, m = n U{4..16}) in one batched
    call with BF16 products: every problem certified; a sample of 32 problems
    checked against the oracle's eta_F and least-squares solution."""
    import torch
    mats, rhs = synth.batched_problems_device(4096, seed=0, device="cuda")
    xs, infos = qrx.lstsq_batched(mats, rhs, prec="bf16", tol=1e-10, max_iter=400)
    torch.cuda.synchronize()
    assert all(i["status"] == 0 for i in infos)
    assert max(i["eta_F"] for i in infos) <= 1e-10
    pick = np.random.default_rng(1).choice(len(mats), 32, replace=False)
    for k in pick:
        A, b, x = host(mats[k]).astype(np.float32), host(rhs[k]), host(xs[k])
        eta = M.eta_F(A, b, x)
        xo, _, _ = L.lls_direct(A, b)
        fe = M.forward_error(x, xo)
        kappa = np.linalg.cond(A.astype(np.float64))
        assert eta <= 1.05e-10, (k, eta)
        assert abs(eta - infos[k]["eta_F"]) <= 0.05 * eta + 1e-14
        # the forward error of a backward-stable least-squares solution: O(kappa eta)
        assert fe <= 1e3 * kappa * 1e-10 + 1e-12, (k, fe, kappa)
