"""Cyclic Jacobi eigensolver in FP64 (test infrastructure only).

An independent route to the eigenpairs of the block Gram matrix, used to
cross-check LAPACK's ``eigh`` in the oracle's pins.  Row-cyclic ordering,
rotation angle chosen to zero the (p, q) entry (Golub & Van Loan, "Matrix
Computations", the symmetric Schur decomposition and cyclic Jacobi, which the
paper cites for the SVD and for orthonormalisation, Sec. 2.3).
"""
from __future__ import annotations

import math

import numpy as np


def sym_schur2(app: float, aqq: float, apq: float):
    """(c, s) with [c s; -s c]^T [[app apq]; [apq aqq]] [c s; -s c] diagonal."""
    if apq == 0.0:
        return 1.0, 0.0
    tau = (aqq - app) / (2.0 * apq)
    if tau >= 0:
        t = 1.0 / (tau + math.sqrt(1.0 + tau * tau))
    else:
        t = -1.0 / (-tau + math.sqrt(1.0 + tau * tau))
    c = 1.0 / math.sqrt(1.0 + t * t)
    return c, t * c


def cyclic_jacobi(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Eigenvalues and eigenvectors (columns) of symmetric A, unsorted."""
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    V = np.eye(n)
    for _ in range(max_sweeps):
        off = math.sqrt(max(0.0, np.sum(A * A) - np.sum(np.diag(A) ** 2)))
        if off <= tol * math.sqrt(np.sum(A * A)):
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                c, s = sym_schur2(A[p, p], A[q, q], A[p, q])
                if s == 0.0:
                    continue
                J = np.eye(n)
                J[p, p] = c
                J[p, q] = s
                J[q, p] = -s
                J[q, q] = c
                A = J.T @ A @ J
                V = V @ J
    return np.diag(A).copy(), V
