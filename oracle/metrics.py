"""Accuracy measures of a computed CSD (oracle, test infrastructure).

Sec. 6 reports the scaled residual ||A_hat - A||_2 / d(A) and the scaled
orthogonality ||U^T U - I||_2 / u; d(A) is the distance to the nearest partial
isometry, eq. (dAeqn) in Sec. 2.1: d(A) = max_i min(sigma_i, |1 - sigma_i|).
"""
from __future__ import annotations

import numpy as np

U_DOUBLE = 2.0 ** -53


def reconstruct(U1, U2, V1, theta):
    """A_hat = diag(U1, U2) [C; S] V1^T with C = cos(theta), S = sin(theta)."""
    c = np.cos(theta)
    s = np.sin(theta)
    return np.vstack([(U1 * c) @ V1.T, (U2 * s) @ V1.T])


def d_partial_isometry(A):
    """Eq. (dAeqn): max over singular values of min(sigma, |1 - sigma|)."""
    sig = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    return float(np.max(np.minimum(sig, np.abs(1.0 - sig))))


def residual(A1, A2, U1, U2, V1, theta, ord=2):
    A = np.vstack([A1, A2])
    return float(np.linalg.norm(reconstruct(U1, U2, V1, theta) - A, ord))


def orthogonality(U, ord=2):
    U = np.asarray(U, dtype=np.float64)
    return float(np.linalg.norm(U.T @ U - np.eye(U.shape[1]), ord))
