"""Dense references for the shifted equations — TEST INFRASTRUCTURE ONLY.

* ``dense_solve``: the plain definition of the result, x = (z S - H)^{-1} b
  (Sec. 3, Eq. 2), by LU.
* ``green_eig``: the eigen-expansion of the Green's function through the
  generalized eigenproblem H y = lambda S y (Sec. 2, Eq. 1) with
  S-orthonormal eigenvectors, G_ij(z) = sum_k y_ik y_jk / (z - lambda_k).
* ``true_residual``: ||b - (z S - H) x|| / ||b||.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _dense(A):
    return A.toarray() if hasattr(A, "toarray") else np.asarray(A)


def dense_solve(H, S, z, b):
    Hd = _dense(H)
    Sd = np.eye(Hd.shape[0]) if S is None else _dense(S)
    return sla.solve(z * Sd - Hd, np.asarray(b, dtype=np.complex128))


def green_eig(H, S, z, i, j):
    """G_ij(z) for every z in ``z`` from the eigenpairs of (H, S)."""
    Hd = _dense(H)
    if S is None:
        lam, Y = np.linalg.eigh(Hd)
    else:
        lam, Y = sla.eigh(Hd, _dense(S))     # Y^T S Y = I
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    w = Y[i, :] * Y[j, :]
    return (w[None, :] / (z[:, None] - lam[None, :])).sum(axis=1)


def true_residual(H, S, z, b, x):
    Sx = x if S is None else S @ x
    return np.linalg.norm(b - (z * Sx - H @ x)) / np.linalg.norm(b)
