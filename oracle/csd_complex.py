"""CS decomposition of a complex partial isometry (oracle, test infrastructure).

The paper's setting is complex: A = [A1; A2] in C^{(m1+m2) x n} with
orthonormal columns (Sec. 1), or a partial isometry (Theorem 2.1), and
    A1 = U1 C V1^*,  A2 = U2 S V1^*,
U1, U2, V1 unitary, C = diag(cos theta), S = diag(sin theta),
0 <= theta_1 <= ... <= theta_n <= pi/2.  This oracle takes Algorithm 1 /
Algorithm 3 in complex arithmetic, through the classical route the paper
names (polar via the SVD, Hermitian eigensolver), in the paper's order:

  polar   W_i H_i = A_i        W = P Q^*, H = Q Sigma Q^* from A_i = P Sigma Q^*
  rank    mu = 0 if rank(A) = n else 2 (rank = round(||A||_F^2), Remark (vi))
  B       B = H2 - H1 + mu (I - A^* A), made Hermitian by (B + B^*) / 2
  eig     V1 Lambda V1^* = B   (numpy.linalg.eigh); rank deficient: keep the
          eigenpairs with Lambda <= (1 + mu) / 2 (Alg. 3, Remark (vii))
  U       U_i = W_i V1
  C, S    C_ii = Re(v_i^* H1 v_i), S_ii = Re(v_i^* H2 v_i) (real: H_i Hermitian)
  angles  theta = atan2(S_ii, C_ii) clamped to [0, pi/2] (Remark (iii)),
          columns ordered by ascending theta.
Shares no code with the real oracle or the device path.
"""
from __future__ import annotations

import numpy as np


def polar_svd(A):
    """W H = A with W = P Q^*, H = Q Sigma Q^* (Hermitian) from the SVD."""
    A = np.asarray(A, dtype=np.complex128)
    P, sig, Qh = np.linalg.svd(A, full_matrices=False)
    W = P @ Qh
    H = (Qh.conj().T * sig) @ Qh
    return W, 0.5 * (H + H.conj().T)


def csd(A1, A2, rank_mode="auto", mu=2.0):
    """Algorithm 1 / 3 in complex arithmetic; returns U1, U2, V1, theta and rank
    (economical in the rank-deficient case)."""
    A1 = np.asarray(A1, dtype=np.complex128)
    A2 = np.asarray(A2, dtype=np.complex128)
    n = A1.shape[1]
    f2 = float(np.sum(np.abs(A1) ** 2) + np.sum(np.abs(A2) ** 2))
    r = int(np.floor(f2 + 0.5))
    if rank_mode == "full":
        deficient = False
    elif rank_mode == "deficient":
        deficient = True
    else:
        deficient = r < n
    m = mu if deficient else 0.0
    W1, H1 = polar_svd(A1)
    W2, H2 = polar_svd(A2)
    B = H2 - H1
    if m != 0.0:
        B = B + m * (np.eye(n) - A1.conj().T @ A1 - A2.conj().T @ A2)
    B = 0.5 * (B + B.conj().T)
    lam, V = np.linalg.eigh(B)
    if deficient:
        keep = lam <= 0.5 * (1.0 + m)
        V = V[:, keep]
        lam = lam[keep]
    U1 = W1 @ V
    U2 = W2 @ V
    c = np.real(np.einsum("ij,ij->j", V.conj(), H1 @ V))
    s = np.real(np.einsum("ij,ij->j", V.conj(), H2 @ V))
    theta = np.clip(np.arctan2(s, c), 0.0, np.pi / 2)
    order = np.argsort(theta, kind="stable")
    return {"U1": U1[:, order], "U2": U2[:, order], "V1": V[:, order], "theta": theta[order],
            "rank": int(V.shape[1]), "W1": W1, "W2": W2, "H1": H1, "H2": H2, "Lambda": lam[order]}
