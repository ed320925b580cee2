"""Seeded synthetic inputs for the CSD (shared by tests, bench and smoke).

This module only draws random matrices and angle sets and assembles
A = [U1 C V1^T; U2 S V1^T]; it holds none of the decomposition's arithmetic.
Every generator takes a ``numpy.random.Generator`` (PCG64 via
``numpy.random.default_rng(seed)``) and returns FP64 numpy arrays.

Recipes (the paper's test classes of Sec. 6, real analogues):

* ``stiefel``      Haar-distributed 2n x n matrix with orthonormal columns
                   (test class 1): Q of a Gaussian 2n x n, columns sign-normalised.
* ``haar``         Haar orthogonal n x n (same construction).
* ``angles_*``     angle sets: uniform in [0, pi/2]; clustered near 0 and pi/2
                   with offsets 10^-U[8, 12]; the cumulative-sum clustered class
                   of Sec. 6 (test class 2).
* ``from_angles``  A1 = U1 diag(cos t) V1^T, A2 = U2 diag(sin t) V1^T, optionally
                   with C_ii = S_ii = 0 on a set of indices (rank-deficient
                   partial isometry, test class 4).
* ``paper_test_class``  the eight test classes of Sec. 6 (1-4 and the noisy
                   1'-4'), real analogues.
* ``complex_pair`` complex blocks A1 = U1 diag(cos t) V1^H, A2 = U2 diag(sin t) V1^H
                   with Haar unitary factors (Q of a complex Gaussian, phases of
                   diag(R) divided out): uniform or clustered angles, repeated
                   angles of a given multiplicity, zeroed pairs (rank deficient),
                   or a Haar 2n x n matrix with orthonormal columns.
"""
from __future__ import annotations

import numpy as np


def haar(n, rng):
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def stiefel(m, n, rng):
    G = rng.standard_normal((m, n))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def angles_uniform(n, rng):
    return np.sort(rng.uniform(0.0, np.pi / 2, n))


def angles_clustered_ends(n, rng, n_low=None, n_high=None, lo_exp=8.0, hi_exp=12.0):
    """Half uniform in [0, pi/2], a quarter at 10^-U[lo,hi] and a quarter at pi/2 minus that."""
    if n_low is None:
        n_low = n // 4
    if n_high is None:
        n_high = n // 4
    n_mid = n - n_low - n_high
    mid = rng.uniform(0.0, np.pi / 2, n_mid)
    low = 10.0 ** (-rng.uniform(lo_exp, hi_exp, n_low))
    high = np.pi / 2 - 10.0 ** (-rng.uniform(lo_exp, hi_exp, n_high))
    return np.sort(np.concatenate([low, mid, high]))


def angles_cumsum_clustered(n, rng, spread=18.0):
    """Test class 2 of Sec. 6: delta = 10^(-18 U), theta = (pi/2) cumsum(delta)/sum(delta)."""
    delta = 10.0 ** (-spread * rng.uniform(0.0, 1.0, n + 1))
    return (np.pi / 2) * np.cumsum(delta[:n]) / np.sum(delta)


def from_angles(theta, rng, zero_idx=None, U1=None, U2=None, V1=None):
    """A = diag(U1, U2) [C; S] V1^T with Haar factors; C_ii = S_ii = 0 on zero_idx."""
    n = theta.shape[0]
    U1 = haar(n, rng) if U1 is None else U1
    U2 = haar(n, rng) if U2 is None else U2
    V1 = haar(n, rng) if V1 is None else V1
    c = np.cos(theta)
    s = np.sin(theta)
    if zero_idx is not None and len(zero_idx):
        c = c.copy()
        s = s.copy()
        c[zero_idx] = 0.0
        s[zero_idx] = 0.0
    A1 = (U1 * c) @ V1.T
    A2 = (U2 * s) @ V1.T
    return A1, A2, {"U1": U1, "U2": U2, "V1": V1, "theta": theta, "zero_idx": zero_idx}


def rect_pair(m1, m2, n, seed, rank_deficient=0):
    """Rectangular blocks (m1, m2 >= n): A1 = U1 C V1^T (m1 x n), A2 = U2 S V1^T
    (m2 x n) with U_i of orthonormal columns (Stiefel), Haar V1, uniform angles;
    rank_deficient = k zeroes k random (C_ii, S_ii) pairs (rank n - k)."""
    rng = np.random.default_rng(seed)
    theta = angles_uniform(n, rng)
    U1 = stiefel(m1, n, rng)
    U2 = stiefel(m2, n, rng)
    zero_idx = np.sort(rng.choice(n, size=rank_deficient, replace=False)) if rank_deficient else None
    return from_angles(theta, rng, zero_idx=zero_idx, U1=U1, U2=U2)


# ---- named workloads -----------------------------------------------------

def haar_stiefel_pair(n, seed):
    """2n x n Haar matrix split into A1 (top n rows) and A2 (bottom n rows)."""
    rng = np.random.default_rng(seed)
    A = stiefel(2 * n, n, rng)
    return np.ascontiguousarray(A[:n]), np.ascontiguousarray(A[n:]), {}


def clustered_pair(n, seed, rank_deficient=0):
    """Angles: n/2 uniform, n/4 within 1e-8..1e-12 of 0, n/4 within that of pi/2.

    rank_deficient > 0 zeroes C_ii = S_ii on that many random indices (rank n - k).
    """
    rng = np.random.default_rng(seed)
    theta = angles_clustered_ends(n, rng)
    zero_idx = None
    if rank_deficient:
        zero_idx = np.sort(rng.choice(n, size=rank_deficient, replace=False))
    A1, A2, meta = from_angles(theta, rng, zero_idx=zero_idx)
    return A1, A2, meta


def uniform_pair(n, seed):
    rng = np.random.default_rng(seed)
    theta = angles_uniform(n, rng)
    return from_angles(theta, rng)


def haar_unitary(m, n, rng):
    """m x n (m >= n) with orthonormal complex columns, Haar distributed."""
    G = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    Q, R = np.linalg.qr(G)
    d = np.diag(R)
    ph = np.where(np.abs(d) > 0, d / np.where(np.abs(d) > 0, np.abs(d), 1.0), 1.0)
    return Q * ph


def complex_pair(n, seed, kind="uniform", rank_deficient=0, mult=1):
    """Complex128 blocks (A1, A2, meta).  kind: "uniform" (angles uniform in
    [0, pi/2]), "clustered" (as clustered_pair), "repeated" (n / mult distinct
    uniform angles, each `mult` times), "exact_ends" (n // 8 angles exactly 0
    and n // 8 exactly pi/2, the rest uniform), "haar" (a Haar 2n x n matrix
    with orthonormal columns split into its halves).  rank_deficient = k
    zeroes k random (C_ii, S_ii) pairs."""
    rng = np.random.default_rng(seed)
    if kind == "haar":
        A = haar_unitary(2 * n, n, rng)
        return np.ascontiguousarray(A[:n]), np.ascontiguousarray(A[n:]), {}
    if kind == "uniform":
        theta = angles_uniform(n, rng)
    elif kind == "clustered":
        theta = angles_clustered_ends(n, rng)
    elif kind == "exact_ends":
        e = n // 8
        theta = np.concatenate([np.zeros(e), np.sort(rng.uniform(0.0, np.pi / 2, n - 2 * e)),
                                np.full(e, np.pi / 2)])
    elif kind == "repeated":
        if n % mult:
            raise ValueError("complex_pair: n must be a multiple of mult")
        theta = np.sort(np.repeat(rng.uniform(0.0, np.pi / 2, n // mult), mult))
    else:
        raise ValueError(f"unknown kind {kind!r}")
    zero_idx = np.sort(rng.choice(n, size=rank_deficient, replace=False)) if rank_deficient else None
    U1, U2, V1 = (haar_unitary(n, n, rng) for _ in range(3))
    c, s = np.cos(theta), np.sin(theta)
    if zero_idx is not None:
        c[zero_idx] = 0.0
        s[zero_idx] = 0.0
    Vh = V1.conj().T
    A1 = (U1 * c) @ Vh
    A2 = (U2 * s) @ Vh
    return A1, A2, {"U1": U1, "U2": U2, "V1": V1, "theta": theta, "zero_idx": zero_idx}


def complex_rect_pair(m1, m2, n, seed, rank_deficient=0):
    """Rectangular complex blocks (m1, m2 >= n): A1 = U1 C V1^H (m1 x n),
    A2 = U2 S V1^H (m2 x n) with U_i of orthonormal columns (Haar, m_i x n),
    Haar unitary V1 and uniform angles; rank_deficient = k zeroes k random
    (C_ii, S_ii) pairs."""
    rng = np.random.default_rng(seed)
    theta = angles_uniform(n, rng)
    U1, U2 = haar_unitary(m1, n, rng), haar_unitary(m2, n, rng)
    V1 = haar_unitary(n, n, rng)
    zero_idx = np.sort(rng.choice(n, size=rank_deficient, replace=False)) if rank_deficient else None
    c, s = np.cos(theta), np.sin(theta)
    if zero_idx is not None:
        c[zero_idx] = 0.0
        s[zero_idx] = 0.0
    Vh = V1.conj().T
    return (U1 * c) @ Vh, (U2 * s) @ Vh, {"theta": theta, "zero_idx": zero_idx}


PAPER_CLASSES = ("1", "2", "3", "4", "1'", "2'", "3'", "4'")


def paper_test_class(cls, n, rng):
    """Test classes of Sec. 6 (real analogue), split into A1 (top n rows) and A2.

    1 Haar 2n x n with orthonormal columns; 2 clustered angles (cumulative-sum
    recipe) with Haar factors; 3 rank r = nint(3n/4), A = X Y^T with X, Y Haar
    with orthonormal columns (2n x r, n x r); 4 class 2 with C_ii = S_ii = 0 on
    n - r random indices; a trailing prime adds 1e-10 N(0, 1) entries.
    """
    if cls not in PAPER_CLASSES:
        raise ValueError(f"unknown test class {cls!r}")
    c = int(cls[0])
    r = int(np.rint(3 * n / 4))
    if c == 1:
        A = stiefel(2 * n, n, rng)
    elif c == 2:
        A1, A2, _ = from_angles(angles_cumsum_clustered(n, rng), rng)
        A = np.vstack([A1, A2])
    elif c == 3:
        A = stiefel(2 * n, r, rng) @ stiefel(n, r, rng).T
    else:
        theta = angles_cumsum_clustered(n, rng)
        zero_idx = np.sort(rng.choice(n, size=n - r, replace=False))
        A1, A2, _ = from_angles(theta, rng, zero_idx=zero_idx)
        A = np.vstack([A1, A2])
    if cls.endswith("'"):
        A = A + 1e-10 * rng.standard_normal(A.shape)
    return np.ascontiguousarray(A[:n]), np.ascontiguousarray(A[n:])


def paper_sizes(jmax=9):
    """n = nint(30 * 2^(j/2)), j = 0..jmax (Sec. 6)."""
    return [int(np.rint(30 * 2.0 ** (j / 2))) for j in range(jmax + 1)]


def batched_sizes(count, seed, lo=8, hi=256):
    """Sizes drawn log-uniform in [lo, hi] and rounded."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)
