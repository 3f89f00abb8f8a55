"""CPU FP64 oracle for the mixed-precision QR / least-squares path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything here; only the tests, the
smoke check and the CPU-baseline leg of the benchmark use it. It shares no
code with the GPU path: plain numpy in float64 (np.longdouble where extended
precision is stated), slow and written to be checked against the paper by eye.

Contents (paper = Zhang & Wu, "High Accuracy Low Precision QR Factorization
and Least Square Solver on GPU with TensorCore"):

* ``householder``  -- the thin QR A = QR (Sec. 2.2: Q m x n orthonormal,
  R n x n upper triangular), computed by textbook Householder QR, the method
  behind Alg. 1's xGEQRF; unblocked and compact-WY blocked (Sec. 3.1.2 cites
  the storage-efficient WY form), sign-normalised so R_kk > 0.
* ``lls``          -- the least-squares solution x = argmin ||Ax - b||
  (Sec. 2.2, eq. opt:lls), by Alg. 1 (x = R^{-1} Q^T b) plus correction steps
  with extended-precision residuals.
* ``krylov``       -- LSQR (Paige & Saunders, cited in Sec. 5) and CG on the
  normal equations of A R^{-1} (the mathematics behind Alg. 5's CGLS), both
  optionally right-preconditioned by an upper-triangular R (Sec. 3.2.3).
* ``metrics``      -- ||A - QR||/||A||, ||I - Q^T Q|| (Sec. 3.2.1) and the
  normal-equation backward error ||A^T r|| / (||A||_F ||r||) (Sec. 3.2.2,
  normalised).
* ``rmgs``         -- Alg. 2 (recursive MGS) with Alg. 4 MGS panels in numpy,
  with the trailing products optionally rounded to FP16/BF16 at the points the
  GPU path rounds them: an error-model emulator used to calibrate the per-
  precision QR error bounds (not the definition of the result).

Parity status: every function above is pinned by ``tests/test_oracle_*.py``
against closed forms, exact rational brute force, independent library
routines or hand-derived fixtures (the metrics by closed-form values in
tests/golden/metrics_*.json). In ``rmgs`` the operand rounding (FP16,
BF16, split FP16) and the float32 sums are pinned to their definitions; that
it rounds at the same points as the GPU path (its calibration role) is
"parity unpinned" beyond its FP64 mode.
"""
from . import householder, lls, krylov, metrics, rmgs  # noqa: F401

__all__ = ["householder", "lls", "krylov", "metrics", "rmgs"]
