"""The no-allocation QR entry point (workspace in a static device array) gives
the results of qrx_qr_factor (same kernels, workspace elsewhere), through the
C ABI, on two calls in a row (the second smaller), and rejects a problem whose
workspace exceeds the array before enqueueing anything."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _call(lib, h, fn, A, R, st, o):
    import torch
    m, n = A.shape
    args = [h.h, m, n, C.c_void_p(A.data_ptr()), A.stride(1), C.c_void_p(R.data_ptr()),
            R.stride(1)]
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if fn == "qrx_qr_factor":
        args += [None, 0]
    return getattr(lib, fn)(*args, C.byref(o), C.c_void_p(st.data_ptr()), s)


def test_noalloc_matches_qr_factor():
    import torch
    import paper_1912_05508_amd as P
    from paper_1912_05508_amd import _lib as L
    h = P.Handle()
    lib = h.lib
    try:
        cases = [(4096, 512, "fp16", 1), (1000, 200, "fp32", 2)]   # the second is smaller
        inputs, ref = [], []
        for (m, n, prec, seed) in cases:
            p = synth.scaled_config("c2", m, n, seed=seed)
            o = L.qr_opts(prec, cutoff=128)
            sz = C.c_size_t()
            assert lib.qrx_qr_workspace_size(h.h, m, n, C.byref(o), C.byref(sz)) == 0
            assert sz.value <= L.QRX_NOALLOC_SCRATCH_BYTES
            inputs.append((p.A, o))
            A = P.colmajor(torch.from_numpy(p.A).cuda())
            R = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda").t()
            st = torch.full((1,), -7, dtype=torch.int32, device="cuda")
            assert _call(lib, h, "qrx_qr_factor", A, R, st, o) == 0
            torch.cuda.synchronize()
            assert int(st.item()) == 0
            ref.append((A.cpu().numpy(), R.cpu().numpy()))
        # two no-allocation calls in a row, the second on a smaller problem
        outs = []
        for (An, o) in inputs:
            m, n = An.shape
            A = P.colmajor(torch.from_numpy(An).cuda())
            R = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda").t()
            st = torch.full((1,), -7, dtype=torch.int32, device="cuda")
            assert _call(lib, h, "qrx_qr_factor_noalloc", A, R, st, o) == 0
            outs.append((A, R, st))
        torch.cuda.synchronize()
        for (A, R, st), (Q1, R1) in zip(outs, ref):
            assert int(st.item()) == 0
            Q2, R2 = A.cpu().numpy(), R.cpu().numpy()
            print(f"{Q2.shape}: max |dQ| {np.abs(Q1 - Q2).max()}, max |dR| {np.abs(R1 - R2).max()}")
            assert np.array_equal(Q1, Q2) and np.array_equal(R1, R2)
        # a problem whose workspace exceeds the static array is rejected up front
        m, n = 65536, 4096
        o = L.qr_opts("fp16", cutoff=128)
        sz = C.c_size_t()
        assert lib.qrx_qr_workspace_size(h.h, m, n, C.byref(o), C.byref(sz)) == 0
        assert sz.value > L.QRX_NOALLOC_SCRATCH_BYTES
        dummy = torch.zeros(1, dtype=torch.float32, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        rc = lib.qrx_qr_factor_noalloc(h.h, m, n, C.c_void_p(dummy.data_ptr()), m,
                                       C.c_void_p(dummy.data_ptr()), n, C.byref(o),
                                       C.c_void_p(st.data_ptr()), None)
        assert rc == L.QRX_EINVAL
    finally:
        h.close()
