"""Seeded synthetic inputs for the least-squares workloads.

This module is shared by the tests, the benchmark and the smoke check. It holds
no arithmetic of the factorisation or of the Krylov solvers: it only draws
random numbers (numpy PCG64, ``default_rng(seed)``, draws taken in the order
each function lists) and builds matrices with a prescribed singular spectrum.
Orthogonal factors U, V come from a *library* QR (LAPACK via numpy, or
torch.linalg.qr on a GPU for the large shapes) of Gaussian matrices, sign
normalised so that the factor is unique.

Matrix families follow the paper's experimental section (Sec. 4.2: uniform on
(0,1) and (-1,1), standard normal, and SVD-constructed matrices with
geometric, arithmetic or clustered singular values of a given condition
number). The paper generated them with MAGMA, which is not available; the
U diag(s) V^T construction below stands in for it.

Every matrix is returned as float32 in column-major (Fortran) order, because
the problem instance is the stored FP32 array; right-hand sides are float64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "rng", "gaussian", "orthonormal", "spectrum", "svd_matrix",
    "paper_family", "PAPER_TYPES", "lls_problem", "config_problem", "batched_problems",
    "CONFIGS", "scaled_config",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def gaussian(g: np.random.Generator, m: int, n: int) -> np.ndarray:
    """N(0,1) draws filled in column-major order (one column after another)."""
    return g.standard_normal((n, m)).T  # Fortran-ordered view, column-major fill


def _sign_fix(Q, R):
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def orthonormal(G, device: str = "cpu"):
    """Sign-normalised thin Q of a library QR of G (float64)."""
    if device == "cpu":
        Q, R = np.linalg.qr(np.asarray(G, dtype=np.float64))
        return np.asfortranarray(_sign_fix(Q, R))
    import torch
    Gt = torch.as_tensor(np.ascontiguousarray(np.asarray(G, dtype=np.float64).T),
                         device=device).t()
    Q, R = torch.linalg.qr(Gt)
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    return Q * d


def spectrum(kind: str, n: int, cond: float, g: np.random.Generator | None = None):
    """Singular values s_1 >= ... >= s_n with s_1 = 1, s_n = 1/cond.

    geometric: log s evenly spaced; arithmetic: s evenly spaced on [1/cond, 1];
    cluster: (1, ..., 1, 1/cond); loguniform: s_i = cond**(-t_i), t_i ~ U[0,1]
    i.i.d., sorted, with t_1 = 0 and t_n = 1 pinned so cond is exact.
    """
    if n == 1:
        return np.ones(1)
    if kind == "geometric":
        return cond ** (-np.arange(n) / (n - 1))
    if kind == "arithmetic":
        return np.linspace(1.0, 1.0 / cond, n)
    if kind == "cluster":
        s = np.ones(n)
        s[-1] = 1.0 / cond
        return s
    if kind == "loguniform":
        t = np.sort(g.random(n))
        t[0], t[-1] = 0.0, 1.0
        return cond ** (-t)
    raise ValueError(kind)


def svd_matrix(g, m, n, s, col_scale=None, device: str = "cpu"):
    """A = U diag(s) V^T (D), built in float64 and rounded once to float32.

    Draw order: U's Gaussian (m x n), then V's Gaussian (n x n).
    """
    G1 = gaussian(g, m, n)
    G2 = gaussian(g, n, n)
    U = orthonormal(G1, device)
    V = orthonormal(G2, device)
    if device == "cpu":
        A = (U * s) @ V.T
        if col_scale is not None:
            A = A * col_scale
        return np.asfortranarray(A.astype(np.float32))
    import torch
    st = torch.as_tensor(s, device=device, dtype=torch.float64)
    A = (U * st) @ V.t()
    if col_scale is not None:
        A = A * torch.as_tensor(col_scale, device=device, dtype=torch.float64)
    A32 = A.to(torch.float32)
    out = torch.empty((n, m), dtype=torch.float32, device=device).t()
    out.copy_(A32)
    return out


def paper_family(g, kind: str, m: int, n: int, cond: float = 1e3, device: str = "cpu"):
    """The paper's eight matrix types (Sec. 4.2, Fig. 3). With a device, the
    matrix is returned there (column-major float32 tensor); the draws are the
    same as on the CPU."""
    if kind in ("uniform01", "uniform11", "normal"):
        if kind == "uniform01":
            A = np.asfortranarray(g.random((n, m)).T.astype(np.float32))
        elif kind == "uniform11":
            A = np.asfortranarray((2.0 * g.random((n, m)).T - 1.0).astype(np.float32))
        else:
            A = np.asfortranarray(gaussian(g, m, n).astype(np.float32))
        if device == "cpu":
            return A
        import torch
        out = torch.empty((n, m), dtype=torch.float32, device=device).t()
        out.copy_(torch.from_numpy(A))
        return out
    return svd_matrix(g, m, n, spectrum(kind, n, cond, g), device=device)


# The eight types of the paper's sweep (Sec. 4.2): (kind, condition number)
PAPER_TYPES = (("uniform01", None), ("uniform11", None), ("normal", None),
               ("geometric", 1e3), ("arithmetic", 1e5), ("arithmetic", 1e6),
               ("cluster", 1e5), ("cluster", 1e6))


@dataclass
class Problem:
    A: object                 # float32 (m, n) column-major (numpy F-order or torch col-major)
    b: object = None          # float64 (m,)
    x_star: object = None     # float64 (n,)
    s: np.ndarray | None = None
    cond: float | None = None
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return tuple(self.A.shape)


def _rhs(A32, x, noise, g_m):
    """b = A x + noise * g using the stored FP32 A (exactly upcast)."""
    if isinstance(A32, np.ndarray):
        return A32.astype(np.float64) @ x + noise * g_m
    import torch
    dev = A32.device
    xt = torch.as_tensor(x, device=dev)
    gt = torch.as_tensor(g_m, device=dev)
    return (A32.double() @ xt + noise * gt)


def lls_problem(g, A32, noise: str | float = "rel1e-6"):
    """x* ~ N(0,1)^n, then g ~ N(0,1)^m, b = A x* + noise.

    ``noise`` is an absolute factor (b = A x* + noise*g) or "relXXX" for
    noise * (||A x*|| / sqrt(m)) * g, the reading used where a workload does
    not state the right-hand side.
    """
    m, n = A32.shape
    x = g.standard_normal(n)
    gm = g.standard_normal(m)
    if isinstance(noise, str) and noise.startswith("rel"):
        fac = float(noise[3:])
        Ax = _rhs(A32, x, 0.0, np.zeros(m))
        nrm = float(np.linalg.norm(Ax)) if isinstance(Ax, np.ndarray) else float(Ax.norm())
        b = _rhs(A32, x, fac * nrm / math.sqrt(m), gm)
    else:
        b = _rhs(A32, x, float(noise), gm)
    return x, b


# ---------------------------------------------------------------------------
# The five workloads (full sizes) and scaled-down analogues for fast tests.
# ---------------------------------------------------------------------------
CONFIGS = {
    # Plain method, FP32 throughout, Gaussian 1024 x 256, b = A x* + 1e-6 g.
    "c1": dict(m=1024, n=256, kind="gaussian", noise=1e-6),
    # Single mixed-precision QR: U diag(s) V^T, s geometric 1 .. 1e-3.
    "c2": dict(m=32768, n=4096, kind="geometric", cond=1e3, noise=None),
    # Mixed-precision LLS: s log-uniform on [1e-6, 1], b = A x* + 1e-8 g.
    "c3": dict(m=65536, n=8192, kind="loguniform", cond=1e6, noise=1e-8),
    # Very tall-skinny: geometric cond 1e5, columns scaled by 10^U[-4,4].
    "c5": dict(m=262144, n=1024, kind="geometric", cond=1e5, noise="rel1e-6",
               colscale=4.0),
}


def config_problem(name: str, seed: int = 0, device: str = "cpu", m=None, n=None):
    """Build workload ``name`` at its full size, or at (m, n) if given.

    Draw order: Gaussian A (c1) or U's and V's Gaussians (SVD kinds); then the
    log-uniform t (c3 kind); then column exponents u (c5 kind); then x*; then g.
    """
    cfg = dict(CONFIGS[name])
    m = m or cfg["m"]
    n = n or cfg["n"]
    g = rng(seed)
    s = None
    if cfg["kind"] == "gaussian":
        A = gaussian(g, m, n).astype(np.float32)
        A = np.asfortranarray(A)
        if device != "cpu":
            import torch
            At = torch.empty((n, m), dtype=torch.float32, device=device).t()
            At.copy_(torch.from_numpy(A))
            A = At
    else:
        G1 = gaussian(g, m, n)
        G2 = gaussian(g, n, n)
        s = spectrum(cfg["kind"], n, cfg["cond"], g)
        colscale = None
        if "colscale" in cfg:
            colscale = 10.0 ** g.uniform(-cfg["colscale"], cfg["colscale"], n)
        U = orthonormal(G1, device)
        V = orthonormal(G2, device)
        del G1, G2
        if device == "cpu":
            A = (U * s) @ V.T
            if colscale is not None:
                A = A * colscale
            A = np.asfortranarray(A.astype(np.float32))
        else:
            import torch
            A64 = (U * torch.as_tensor(s, device=device)) @ V.t()
            del U, V
            if colscale is not None:
                A64 *= torch.as_tensor(colscale, device=device)
            A = torch.empty((n, m), dtype=torch.float32, device=device).t()
            A.copy_(A64)
            del A64
    p = Problem(A=A, s=s, cond=cfg.get("cond"), meta=dict(name=name, seed=seed, m=m, n=n))
    if cfg["noise"] is not None:
        p.x_star, p.b = lls_problem(g, A, cfg["noise"])
    return p


def scaled_config(name: str, m: int, n: int, seed: int = 0):
    """The same recipe as ``name`` at a reduced (m, n) (CPU, numpy)."""
    return config_problem(name, seed=seed, device="cpu", m=m, n=n)


def batched_problems(count: int = 4096, seed: int = 0, nmin_j: int = 4,
                     nmax_j: int = 32, kmin: int = 4, kmax: int = 16):
    """Uneven batch: n = 8 j, j ~ U{nmin_j..nmax_j}; m = n k, k ~ U{kmin..kmax}.

    Per problem, in order: j, k, A ~ N(0,1)^(m x n), u ~ U[-2,2]^n (column
    scales 10^u), x* ~ N(0,1)^n, g ~ N(0,1)^m, b = A x* + 1e-6 (||A x*||/sqrt(m)) g.
    """
    g = rng(seed)
    out = []
    for _ in range(count):
        j = int(g.integers(nmin_j, nmax_j + 1))
        k = int(g.integers(kmin, kmax + 1))
        n = 8 * j
        m = n * k
        A = gaussian(g, m, n) * (10.0 ** g.uniform(-2.0, 2.0, n))
        A = np.asfortranarray(A.astype(np.float32))
        x, b = lls_problem(g, A, "rel1e-6")
        out.append(Problem(A=A, b=b, x_star=x, meta=dict(m=m, n=n)))
    return out


def batched_sizes(count: int = 4096, seed: int = 0, nmin_j: int = 4, nmax_j: int = 32,
                  kmin: int = 4, kmax: int = 16):
    """The (m, n) list of the uneven batch: n = 8 j, j ~ U{nmin_j..nmax_j}, m = n k,
    k ~ U{kmin..kmax} (drawn in that order per problem)."""
    g = rng(seed)
    out = []
    for _ in range(count):
        j = int(g.integers(nmin_j, nmax_j + 1))
        k = int(g.integers(kmin, kmax + 1))
        out.append((8 * j * k, 8 * j))
    return out


def batched_problems_device(count: int = 4096, seed: int = 0, device: str = "cuda", **kw):
    """The batched recipe drawn on the device (torch's seeded generator) for the
    full-size workload: sizes from ``batched_sizes``; A ~ N(0,1) with columns
    scaled by 10^U[-2,2] (column-major FP32); x* ~ N(0,1); b = A x* + 1e-6
    (||A x*|| / sqrt(m)) g in FP64. Returns (list of A, list of b)."""
    import torch
    sizes = batched_sizes(count, seed, **kw)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    mats, rhs = [], []
    for m, n in sizes:
        A = torch.randn((n, m), generator=gen, device=device, dtype=torch.float32).t()
        A.mul_(10.0 ** (torch.rand(n, generator=gen, device=device, dtype=torch.float32) * 4 - 2))
        x = torch.randn(n, generator=gen, device=device, dtype=torch.float64)
        g = torch.randn(m, generator=gen, device=device, dtype=torch.float64)
        Ax = A.double() @ x
        b = Ax + 1e-6 * (Ax.norm() / math.sqrt(m)) * g
        mats.append(A)
        rhs.append(b.contiguous())
    return mats, rhs
