"""Complete 2 x 2 CS decomposition (oracle, test infrastructure: only tests, the
smoke check and the CPU baseline use it; the product path never imports it).

Remark (viii) of Sec. 3: an orthogonal A = [A1 A3; A2 A4] (2n x 2n, n x n blocks)
has A = diag(U1, U2) [C -S; S C] diag(V1, V2)^T.  Algorithm 1 applied to the
first block column gives U1, U2, V1, C, S; then X = -A3^T U1 S + A4^T U2 C,
whose QR factor (diag(R) >= 0) is V2 (X itself is orthogonal when A is).
"""
from __future__ import annotations

import numpy as np

from . import csd as O
from .repair import qr_pos


def csd2x2(A):
    """Returns dict U1, U2, V1, V2, theta (ascending) of an orthogonal 2n x 2n A."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    if A.shape != (m, m) or m % 2:
        raise ValueError("A must be 2n x 2n")
    n = m // 2
    A1, A2, A3, A4 = A[:n, :n], A[n:, :n], A[:n, n:], A[n:, n:]
    r = O.csd(A1, A2, rank_mode="full")
    U1, U2, V1, th = r["U1"], r["U2"], r["V1"], r["theta"]
    X = -A3.T @ (U1 * np.sin(th)) + A4.T @ (U2 * np.cos(th))
    V2, _ = qr_pos(X)
    return {"U1": U1, "U2": U2, "V1": V1, "V2": V2, "theta": th, "X": X}


def reconstruct2x2(U1, U2, V1, V2, theta):
    """diag(U1, U2) [C -S; S C] diag(V1, V2)^T."""
    c, s = np.cos(theta), np.sin(theta)
    top = np.hstack([(U1 * c) @ V1.T, -(U1 * s) @ V2.T])
    bot = np.hstack([(U2 * s) @ V1.T, (U2 * c) @ V2.T])
    return np.vstack([top, bot])
