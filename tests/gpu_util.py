"""Helpers shared by the GPU tests (device transfer, column-major layout)."""
import numpy as np


def dev(A, ld=None):
    """numpy (m, n) -> column-major float32 cuda tensor (leading dim ld >= m)."""
    import torch
    A = np.asarray(A, dtype=np.float32)
    m, n = A.shape
    ld = ld or m
    buf = torch.zeros((n, ld), dtype=torch.float32, device="cuda")
    t = buf.t()[:m, :]
    t.copy_(torch.from_numpy(np.ascontiguousarray(A)))
    return t


def dev64(v):
    import torch
    return torch.as_tensor(np.asarray(v, dtype=np.float64), device="cuda").contiguous()


def host(t):
    return t.detach().cpu().numpy()
