"""Zolo-pd as the rational matrix function it defines (oracle, test infrastructure).

Sec. 5: every iterate keeps the singular vectors of A, X_k = P r_k(Sigma) Q^T,
and one iteration applies the Zolotarev function of ``oracle.zolotarev``:

    X_{k+1} = M X_k prod_j (X_k^T X_k + c_{2j} I)(X_k^T X_k + c_{2j-1} I)^{-1}
            = M (X_k + sum_j a_j X_k (X_k^T X_k + c_{2j-1} I)^{-1}).

Two such iterations (the second on [l_1, 1]) give W; H = sym(W^T A).
``zolo_pd`` writes the partial-fraction form out with dense solves in FP64,
no QR or Cholesky restructuring (accurate while X^T X + c I is well
conditioned); ``zolo_pd_svd_form`` applies the scalar function to the singular
values.  The two agree where both are accurate (pinned in the tests); the SVD
form is the reference for the GPU iterates X_1, X_2, W and H when both sides
are given the same l and r.
"""
from __future__ import annotations

import numpy as np

from .zolotarev import two_step


def zolo_step(X, step):
    """One Zolotarev iteration X -> M (X + sum_j a_j X (X^T X + c_{2j-1} I)^{-1})."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[1]
    G = X.T @ X
    acc = X.copy()
    I = np.eye(n)
    for j in range(step.r):
        # X (G + c I)^{-1} = ((G + c I)^{-1} X^T)^T since G + c I is symmetric
        acc += step.a[j] * np.linalg.solve(G + step.c_odd[j] * I, X.T).T
    return step.M * acc


def zolo_pd(A, ell, r, alpha=1.0):
    """Two Zolo-pd iterations on A/alpha with lower bound ell and r terms.

    Returns dict with X1, X2 (= W), H = sym(W^T A), and the two steps.
    """
    A = np.asarray(A, dtype=np.float64)
    s1, s2, resid = two_step(ell, r)
    X0 = A / alpha
    X1 = zolo_step(X0, s1)
    X2 = zolo_step(X1, s2)
    WtA = X2.T @ A
    H = 0.5 * (WtA + WtA.T)
    return {"X1": X1, "X2": X2, "W": X2, "H": H, "step1": s1, "step2": s2,
            "resid": float(resid)}


def zolo_pd_svd_form(A, ell, r, alpha=1.0):
    """The same iterates through the SVD: X_k = P diag(Z_k(...Z_1(sigma))) Q^T.

    This is the iterate as Sec. 5 defines it (same singular vectors as A, the
    scalar Zolotarev function applied to each singular value), exact up to the
    rounding of the SVD for any conditioning, including the modified Zolo-pd
    on [eps, 1] of Sec. 5.1 where the dense-solve form above loses accuracy.
    """
    A = np.asarray(A, dtype=np.float64)
    s1, s2, _ = two_step(ell, r)
    P, sig, Qt = np.linalg.svd(A / alpha, full_matrices=False)
    z1 = np.array([s1(x) for x in sig])
    z2 = np.array([s2(x) for x in z1])
    X2 = (P * z2) @ Qt
    WtA = X2.T @ A
    return {"X1": (P * z1) @ Qt, "X2": X2, "W": X2, "H": 0.5 * (WtA + WtA.T),
            "sigma": sig, "z1": z1, "z2": z2, "step1": s1, "step2": s2}
