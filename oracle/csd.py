"""CS decomposition by Algorithm 1 / Algorithm 3 (oracle, test infrastructure).

The CSD has a plain definition (Sec. 1; Theorem 2.1 for partial isometries):
A1 = U1 C V1^T, A2 = U2 S V1^T with orthonormal U1, U2, V1, C = diag(cos theta),
S = diag(sin theta), 0 <= theta_1 <= ... <= theta_n <= pi/2.  Zolo-csd is one
backward-stable way to reach it.  This oracle reaches the same decomposition
through the classical backward-stable route the paper names in Remark (v) and
Sec. 5.1: polar decompositions through the SVD and a LAPACK symmetric
eigensolver, with the steps of Algorithm 1 in the paper's order:

  polar   W_i H_i = A_i                     (via SVD: W = P Q^T, H = Q Sigma Q^T)
  rank    mu = 0 if rank(A) = n else 2      (rank from ||A||_F^2, Remark (vi))
  B       B = H2 - H1 + mu (I - A^T A)
  eig     V1 Lambda V1^T = B                (numpy.linalg.eigh)
          rank-deficient: keep the eigenpairs with Lambda in [-1, 1] (Alg. 3, Remark (vii))
  U       U_i = W_i V1
  C, S    C = diag(V1^T H1 V1), S = diag(V1^T H2 V1)
  angles  theta = arctan(S_ii / C_ii), C = cos theta, S = sin theta (Remark (iii)),
          columns ordered by ascending theta (Sec. 1).
          With theta_from="lambda" C and S come instead from the cheaper route of
          Remark (iv): Lambda_ii = sin theta_i - cos theta_i = sqrt(2) sin(theta_i - pi/4),
          so theta_i = pi/4 + arcsin(Lambda_ii / sqrt(2)).

Readings taken where the paper is silent: H and B are symmetrised by
(X + X^T)/2; arctan(S/C) is evaluated as atan2(S, C) and clamped to [0, pi/2].
"""
from __future__ import annotations

import numpy as np


def polar_svd(A):
    """Polar decomposition A = W H through the SVD (Sec. 2: W = P Q^T, H = Q Sigma Q^T)."""
    A = np.asarray(A, dtype=np.float64)
    P, sig, Qt = np.linalg.svd(A, full_matrices=False)
    W = P @ Qt
    H = (Qt.T * sig) @ Qt
    return W, 0.5 * (H + H.T)


def eps_rank(A1, A2):
    """Remark (vi): ||A||_F ~ sqrt(rank(A)) when A is close to a partial isometry."""
    f2 = float(np.sum(A1 * A1) + np.sum(A2 * A2))
    return int(np.floor(f2 + 0.5))


def csd(A1, A2, rank_mode="auto", mu=2.0, b_choice="H2-H1", theta_from="diag"):
    """Algorithm 1 (full rank) / Algorithm 3 (rank deficient) in FP64.

    rank_mode: "auto" (Remark (vi)), "full" or "deficient".
    b_choice : "H2-H1" (the paper's choice).  "H1" is accepted only so the
               tests can reproduce the unstable variant of the worked example
               in Sec. 3; it is never the default.
    theta_from: "diag" (C, S = diag(V1^T H_i V1), the default) or "lambda" (Remark (iv)).
    Returns a dict with U1, U2, V1, theta (economical in the rank-deficient
    case) and the intermediates W1, W2, H1, H2, B, Lambda, rank, mu.
    """
    A1 = np.asarray(A1, dtype=np.float64)
    A2 = np.asarray(A2, dtype=np.float64)
    n = A1.shape[1]
    if A2.shape[1] != n:
        raise ValueError("A1 and A2 must have the same number of columns")
    W1, H1 = polar_svd(A1)
    W2, H2 = polar_svd(A2)
    r_A = eps_rank(A1, A2)
    if rank_mode == "full":
        deficient = False
    elif rank_mode == "deficient":
        deficient = True
    else:
        deficient = r_A < n
    mu_used = mu if deficient else 0.0
    I = np.eye(n)
    if b_choice == "H2-H1":
        B = H2 - H1
        if mu_used != 0.0:
            AtA = A1.T @ A1 + A2.T @ A2
            B = B + mu_used * (I - AtA)
    elif b_choice == "H1":
        B = H1.copy()
    else:
        raise ValueError("unknown b_choice")
    B = 0.5 * (B + B.T)
    lam, V = np.linalg.eigh(B)
    if deficient:
        # Algorithm 3: the eigenvectors whose eigenvalues lie in [-1, 1];
        # the n - r others sit at mu.  eigh sorts ascending, so they are the
        # r_A smallest (r_A from Remark (vi) unless the caller forced the mode).
        keep = int(np.sum(lam <= 0.5 * (1.0 + mu_used)))
        V = V[:, :keep]
        lam = lam[:keep]
    U1 = W1 @ V
    U2 = W2 @ V
    c = np.einsum("ij,ij->j", V, H1 @ V)
    s = np.einsum("ij,ij->j", V, H2 @ V)
    if theta_from == "diag":
        theta = np.clip(np.arctan2(s, c), 0.0, np.pi / 2)
    elif theta_from == "lambda":
        x = np.clip(lam, -1.0, 1.0)
        theta = np.clip(np.pi / 4 + np.arcsin(x / np.sqrt(2.0)), 0.0, np.pi / 2)
    else:
        raise ValueError("unknown theta_from")
    order = np.argsort(theta, kind="stable")
    return {
        "U1": U1[:, order], "U2": U2[:, order], "V1": V[:, order],
        "theta": theta[order], "c_raw": c[order], "s_raw": s[order],
        "Lambda": lam[order], "W1": W1, "W2": W2, "H1": H1, "H2": H2, "B": B,
        "rank": V.shape[1], "mu": mu_used,
    }
