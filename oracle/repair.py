"""Algorithm 2 of Sec. 5.1: repair of the polar factor of an ill-conditioned A_i
(oracle, test infrastructure: only tests, the smoke check and the CPU baseline
use it; the product path never imports it).

When A_i is full rank but sigma_min(A_i) is below the floor eps of the
Zolo-pd lower bound, the computed W~_i is not orthonormal while
H~_i = sym(W~_i^T A_i) is still a good symmetric factor.  With the QR
factorisations A_i = Q_i R_i and H~_i = Q~_i R~_i, both with diag(R) >= 0
(which makes them unique for nonsingular factors), the two R factors agree in
exact arithmetic (A = W H, H = Q~ R~ gives A = (W Q~) R~), and
W_i = Q_i Q~_i^T is orthonormal by construction.  Its residual is
W_i H~_i - A_i = Q_i (R~_i - R_i), so ||R~_i - R_i|| measures the backward
error; the paper accepts the repair when that error is O(n u ||A_i||).

The steps follow Sec. 5.1 in order, with numpy's Householder QR
(LAPACK geqrf/orgqr) as the factorisation primitive.
"""
from __future__ import annotations

import numpy as np


def qr_pos(A):
    """QR with diag(R) >= 0: A = Q R (numpy's QR, then column/row signs flipped)."""
    Q, R = np.linalg.qr(np.asarray(A, dtype=np.float64))
    d = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    return Q * d, R * d[:, None]


def polar_repair(A, Ht):
    """Algorithm 2: W = Q Q~^T from A = Q R and H~ = Q~ R~.

    Returns (W, rel) with rel = ||R~ - R||_F / ||R||_F, the relative backward
    error of W H~ as a factorisation of A (Frobenius norm).
    """
    Q, R = qr_pos(A)
    Qt, Rt = qr_pos(Ht)
    W = Q @ Qt.T
    rel = float(np.linalg.norm(Rt - R) / np.linalg.norm(R))
    return W, rel


def repair_accepted(rel, n, u=2.0 ** -53):
    """The acceptance test of Sec. 5.1 with the constant this library uses: rel <= 100 n u."""
    return rel <= 100.0 * n * u
