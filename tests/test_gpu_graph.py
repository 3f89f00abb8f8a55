"""The QR call records into a HIP graph: it enqueues only kernels on the given
stream (flags are cleared by a kernel, the workspace comes from the handle's
pool, no host synchronisation), so a captured factorisation replays to the
same bits as the eager call. Every replay is checked, with eager work and
synchronisations of the program in between."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,nb", [("fp16", 0), ("fp16x3", 0), ("fp32", 128)])
def test_qr_graph_replay_matches_eager(prec, nb):
    import torch
    import paper_1912_05508_amd as P
    h = P.Handle()
    try:
        p = synth.scaled_config("c2", 2048, 512, seed=5)
        A = torch.empty((512, 2048), dtype=torch.float32, device="cuda").t()
        A.copy_(torch.from_numpy(p.A))
        other = torch.empty_like(A)
        other.copy_(torch.from_numpy(synth.scaled_config("c2", 2048, 512, seed=6).A))
        m, n = A.shape
        Q = torch.empty((n, m), dtype=torch.float32, device="cuda").t()
        R = torch.empty((n, n), dtype=torch.float32, device="cuda").t()
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        Q2, R2, st2 = torch.empty_like(Q), torch.empty_like(R), torch.zeros_like(st)
        kw = dict(prec=prec, cutoff=128, panel_width=nb)

        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            h.qr_out(A, Q, R, st, **kw)          # eager (also sizes the handle's pool)
            torch.cuda.synchronize()
            Qe, Re = Q.clone(), R.clone()
            assert int(st.item()) == 0
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                h.qr_out(A, Q, R, st, **kw)
        torch.cuda.synchronize()
        for rep in range(3):
            Q.zero_()
            R.zero_()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(Q, Qe) and torch.equal(R, Re), f"replay {rep}"
            assert int(st.item()) == 0
            # the program's own eager work between replays (another factorisation)
            h.qr_out(other, Q2, R2, st2, **kw)
            torch.cuda.synchronize()
        del g
    finally:
        h.close()


@pytest.mark.parametrize("prec,method", [("fp16", "lsqr"), ("fp32", "cgls")])
def test_lls_graph_replay_matches_eager(prec, method):
    """The whole least-squares solve (scan, QR, R^-1, the persistent Krylov
    kernel with its device-side stopping test, certification and restarts)
    records into a HIP graph: no host round trip per iteration. Replays give
    the eager x and info bit for bit, with eager work between them; a larger
    eager solve in between makes the handle grow its workspace, which must not
    invalidate the recorded one."""
    import torch
    import paper_1912_05508_amd as P
    h = P.Handle()
    try:
        g0 = synth.rng(3)
        An = synth.svd_matrix(g0, 2048, 256, synth.spectrum("loguniform", 256, 1e4, g0))
        _, bn = synth.lls_problem(synth.rng(4), An, "rel1e-6")
        A = P.colmajor(torch.from_numpy(An).cuda())
        b = torch.as_tensor(bn, device="cuda")
        Ab = P.colmajor(torch.from_numpy(synth.scaled_config("c1", 4096, 512, seed=7).A).cuda())
        bb = torch.randn(4096, dtype=torch.float64, device="cuda")
        x = torch.zeros(256, dtype=torch.float64, device="cuda")
        info = P.info_tensor(device="cuda")
        kw = dict(prec=prec, method=1 if method == "cgls" else 0, tol=1e-10, max_iter=2000,
                  cutoff=64)

        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            h.lstsq_async(A, b, x, info, **kw)    # eager (also sizes the handle's pool)
            torch.cuda.synchronize()
            xe, ie = x.clone(), info.clone()
            e = P.read_info(ie)[0]
            assert e["status"] == 0 and e["iters"] > 0, e
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                h.lstsq_async(A, b, x, info, **kw)
        torch.cuda.synchronize()
        for rep in range(3):
            x.zero_()
            info.zero_()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(x, xe) and torch.equal(info, ie), f"replay {rep}"
            # eager work between replays: a larger solve (grows the workspace)
            xb, ib = h.lstsq(Ab, bb, prec="fp32", tol=1e-10)
            torch.cuda.synchronize()
            assert ib["status"] == 0
        del g
    finally:
        h.close()
