"""Pins of the CSD oracle (CPU).

The oracle (``oracle.csd``) is checked against facts fixed by the paper and by
the mathematics, never against a retyped copy of itself:

* the worked example of Sec. 3 (tests/golden/worked_example_sec3.json);
* inputs built from known factors: the angles are known exactly;
* LAPACK's CS decomposition (``scipy.linalg.cossin``, ?orcsd), a different
  algorithm (the paper's comparison system, Sec. 6);
* invariants: C^2 + S^2 = I, orthogonality, backward error (Theorem 4.1),
  the swap symmetry of Remark (i) (theta -> pi/2 - theta), the closed forms
  f(Lambda) = cos(theta), g(Lambda) = sin(theta) of Sec. 4;
* special cases with a textbook answer: n = 1, diagonal inputs;
* rank-deficient partial isometries (Theorem 2.1, Algorithm 3).
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import csd as O
from oracle import metrics as Mt
from paper_1804_09002_amd import workloads as WL

HERE = os.path.dirname(os.path.abspath(__file__))
U = 2.0 ** -53


def _golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def test_worked_example_sec3():
    g = _golden("worked_example_sec3.json")
    theta = np.array(g["theta"])
    V1 = np.array(g["V1_times_3"], dtype=float) / 3.0
    H1 = V1 @ np.diag(np.cos(theta)) @ V1.T
    H2 = V1 @ np.diag(np.sin(theta)) @ V1.T
    # A1 = H1, A2 = H2 is itself a 6 x 3 matrix with orthonormal columns (H1^2 + H2^2 = I)
    good = O.csd(H1, H2)
    S = good["V1"].T @ H2 @ good["V1"]
    off_good = np.max(np.abs(S - np.diag(np.diag(S))))
    assert off_good < 1e-15                           # paper: 1.7806e-17, "a small multiple of u"
    bad = O.csd(H1, H2, b_choice="H1")
    S = bad["V1"].T @ H2 @ bad["V1"]
    off_bad = np.max(np.abs(S - np.diag(np.diag(S))))
    assert g["paper_offdiag_eig_H1"] / 10 < off_bad < g["paper_offdiag_eig_H1"] * 10
    # the stable variant recovers the tiny angles to absolute accuracy O(u)
    assert np.max(np.abs(good["theta"] - theta)) < 4 * U


@pytest.mark.parametrize("n,seed", [(16, 11), (64, 12), (200, 13)])
def test_known_angles_uniform(n, seed):
    A1, A2, meta = WL.uniform_pair(n, seed)
    out = O.csd(A1, A2)
    assert out["rank"] == n and out["mu"] == 0.0
    assert np.max(np.abs(out["theta"] - np.sort(meta["theta"]))) <= 10 * n * U


@pytest.mark.parametrize("n,seed", [(32, 21), (128, 22)])
def test_known_angles_clustered(n, seed):
    A1, A2, meta = WL.clustered_pair(n, seed)
    out = O.csd(A1, A2)
    assert np.max(np.abs(out["theta"] - np.sort(meta["theta"]))) <= 10 * n * U
    R = Mt.residual(A1, A2, out["U1"], out["U2"], out["V1"], out["theta"], ord="fro")
    assert R <= 1e-13 * np.sqrt(n)


@pytest.mark.parametrize("n,seed", [(8, 1), (64, 1), (100, 3)])
def test_against_lapack_cossin(n, seed):
    A1, A2, _ = WL.haar_stiefel_pair(n, seed)
    out = O.csd(A1, A2)
    X = np.vstack([A1, A2])
    # full 2n x 2n orthogonal completion for LAPACK's 2x2 CSD
    Qf, _ = np.linalg.qr(X, mode="complete")
    Qf = np.hstack([X, Qf[:, n:]])
    _, cs, _ = scipy.linalg.cossin(Qf, p=n, q=n, separate=True)
    th_lapack = np.sort(np.asarray(cs))
    assert np.max(np.abs(out["theta"] - th_lapack)) <= 50 * n * U


@pytest.mark.parametrize("n,seed", [(16, 31), (80, 32)])
def test_invariants_and_backward_error(n, seed):
    A1, A2, _ = WL.haar_stiefel_pair(n, seed)
    out = O.csd(A1, A2)
    c, s = np.cos(out["theta"]), np.sin(out["theta"])
    assert np.max(np.abs(c * c + s * s - 1)) < 4 * U
    for k in ("U1", "U2", "V1"):
        assert Mt.orthogonality(out[k]) <= 100 * U * n
    A = np.vstack([A1, A2])
    res = Mt.residual(A1, A2, out["U1"], out["U2"], out["V1"], out["theta"], ord="fro")
    assert res / np.linalg.norm(A) <= 1e-13
    assert np.all(np.diff(out["theta"]) >= 0)
    assert out["theta"][0] >= 0 and out["theta"][-1] <= np.pi / 2


@pytest.mark.parametrize("n,seed", [(12, 41), (60, 42)])
def test_swap_symmetry_remark_i(n, seed):
    """Remark (i): swapping A1 and A2 negates B; theta -> pi/2 - theta (the text's pi/4 is a typo)."""
    A1, A2, _ = WL.haar_stiefel_pair(n, seed)
    a = O.csd(A1, A2)
    b = O.csd(A2, A1)
    assert np.max(np.abs(b["theta"][::-1] - (np.pi / 2 - a["theta"]))) <= 10 * n * U
    assert np.allclose(b["B"], -a["B"], atol=0, rtol=0) or np.max(np.abs(b["B"] + a["B"])) < 8 * U


@pytest.mark.parametrize("n,seed", [(10, 51), (50, 52)])
def test_closed_form_f_g_sec4(n, seed):
    """Sec. 4: cos(theta) = f(Lambda), sin(theta) = g(Lambda), f, g = (-z +- ... ) / 2 with sqrt(2 - z^2)."""
    A1, A2, _ = WL.haar_stiefel_pair(n, seed)
    out = O.csd(A1, A2)
    z = out["Lambda"]
    f = 0.5 * (-z + np.sqrt(2 - z * z))
    g = 0.5 * (z + np.sqrt(2 - z * z))
    assert np.max(np.abs(f - np.cos(out["theta"]))) < 1e-14
    assert np.max(np.abs(g - np.sin(out["theta"]))) < 1e-14
    assert np.max(np.abs(z - (np.sin(out["theta"]) - np.cos(out["theta"])))) < 1e-14


def test_n_equals_one():
    for a1, a2 in [(0.6, 0.8), (-0.6, 0.8), (1.0, 0.0), (0.0, -1.0), (np.cos(0.3), -np.sin(0.3))]:
        out = O.csd(np.array([[a1]]), np.array([[a2]]))
        assert abs(out["theta"][0] - np.arctan2(abs(a2), abs(a1))) < 4 * U
        assert abs(abs(out["U1"][0, 0]) - 1) < 4 * U and abs(abs(out["V1"][0, 0]) - 1) < 4 * U


def test_diagonal_input_gives_permutation_factors():
    rng = np.random.default_rng(5)
    n = 9
    theta = rng.uniform(0.05, 1.5, n)
    perm = rng.permutation(n)
    A1 = np.diag(np.cos(theta))[:, perm]
    A2 = np.diag(np.sin(theta))[:, perm]
    out = O.csd(A1, A2)
    assert np.max(np.abs(out["theta"] - np.sort(theta))) < 8 * U
    P = np.abs(out["V1"])
    assert np.allclose(P @ P.T, np.eye(n), atol=1e-14)
    assert np.allclose(np.sort(P.max(axis=0)), 1.0, atol=1e-14)


@pytest.mark.parametrize("n,k,seed", [(24, 6, 61), (64, 16, 62)])
def test_rank_deficient_algorithm3(n, k, seed):
    A1, A2, meta = WL.clustered_pair(n, seed, rank_deficient=k)
    out = O.csd(A1, A2)
    r = n - k
    assert out["rank"] == r and out["mu"] == 2.0
    keep = np.setdiff1d(np.arange(n), meta["zero_idx"])
    th_true = np.sort(meta["theta"][keep])
    assert np.max(np.abs(out["theta"] - th_true)) <= 10 * n * U
    for key in ("U1", "U2", "V1"):
        assert out[key].shape == (n, r)
        assert Mt.orthogonality(out[key]) <= 100 * n * U
    res = Mt.residual(A1, A2, out["U1"], out["U2"], out["V1"], out["theta"], ord="fro")
    assert res <= 1e-13 * np.sqrt(r)
    # Theorem 2.1: C^2 + S^2 = diag(I_r, 0) -- the economical form keeps the I_r part
    assert np.max(np.abs(np.cos(out["theta"]) ** 2 + np.sin(out["theta"]) ** 2 - 1)) < 4 * U


def test_rank_deficient_haar_class3():
    """Test class 3 of Sec. 6: A = X Y^T with Haar X (2n x r), Y (n x r)."""
    rng = np.random.default_rng(71)
    n, r = 40, 30
    X = WL.stiefel(2 * n, r, rng)
    Y = WL.stiefel(n, r, rng)
    A = X @ Y.T
    out = O.csd(A[:n], A[n:])
    assert out["rank"] == r
    res = Mt.residual(A[:n], A[n:], out["U1"], out["U2"], out["V1"], out["theta"], ord="fro")
    assert res <= 1e-13 * np.sqrt(r)


def test_d_of_A_formula():
    """Eq. (dAeqn) on a matrix with known singular values."""
    rng = np.random.default_rng(3)
    P = WL.stiefel(10, 4, rng)
    Q = WL.haar(4, rng)
    sig = np.array([1.0 + 1e-9, 0.7, 1e-10, 1 - 3e-9])
    A = (P * sig) @ Q.T
    # min(sigma, |1 - sigma|): 1e-9, 0.3, 1e-10, 3e-9 -> max = 0.3
    assert abs(Mt.d_partial_isometry(A) - 0.3) < 1e-14


def test_noise_class_backward_error_scales_with_dA():
    """Test class 1' of Sec. 6: residual / d(A) of order one (Table 1 reports 1.1 - 1.3)."""
    rng = np.random.default_rng(81)
    n = 30
    A = WL.stiefel(2 * n, n, rng) + 1e-10 * rng.standard_normal((2 * n, n))
    out = O.csd(A[:n], A[n:])
    ratio = Mt.residual(A[:n], A[n:], out["U1"], out["U2"], out["V1"], out["theta"]) / Mt.d_partial_isometry(A)
    assert 0.5 < ratio < 3.0


@pytest.mark.parametrize("m1,m2,n,k,seed", [(30, 45, 20, 0, 71), (90, 60, 40, 7, 72), (25, 25, 10, 0, 73)])
def test_rectangular_blocks_known_factors(m1, m2, n, k, seed):
    """Algorithm 1 / 3 with m1, m2 >= n (the setting of Sec. 2): blocks built
    from known factors (U_i with orthonormal columns, Haar V1, known angles,
    k zeroed pairs) give back the known angles, the rank n - k, orthonormal
    factors and the blocks."""
    A1, A2, meta = WL.rect_pair(m1, m2, n, seed, rank_deficient=k)
    r = O.csd(A1, A2)
    rank = n - k
    assert r["rank"] == rank
    keep = np.setdiff1d(np.arange(n), meta["zero_idx"] if k else [])
    assert np.max(np.abs(r["theta"] - np.sort(meta["theta"][keep]))) <= 10 * n * U
    U1, U2, V1, th = r["U1"], r["U2"], r["V1"], r["theta"]
    assert U1.shape == (m1, rank) and U2.shape == (m2, rank) and V1.shape == (n, rank)
    for X in (U1, U2, V1):
        assert np.linalg.norm(X.T @ X - np.eye(rank), 2) <= 100 * n * U
    assert np.linalg.norm((U1 * np.cos(th)) @ V1.T - A1, 2) <= 100 * n * U
    assert np.linalg.norm((U2 * np.sin(th)) @ V1.T - A2, 2) <= 100 * n * U


@pytest.mark.parametrize("n,k,seed", [(48, 0, 81), (64, 16, 82)])
def test_theta_from_lambda_remark_iv(n, k, seed):
    """Remark (iv): theta from sin(theta) - cos(theta) = Lambda recovers the known
    angles to absolute accuracy O(n u), full rank and rank deficient alike, and
    leaves U1, U2, V1 as the default route gives them."""
    A1, A2, meta = WL.clustered_pair(n, seed, rank_deficient=k)
    a = O.csd(A1, A2)
    b = O.csd(A1, A2, theta_from="lambda")
    keep = np.setdiff1d(np.arange(n), meta["zero_idx"]) if k else np.arange(n)
    th_true = np.sort(meta["theta"][keep])
    assert b["rank"] == n - k
    assert np.max(np.abs(b["theta"] - th_true)) <= 10 * n * U
    assert np.max(np.abs(b["theta"] - a["theta"])) <= 10 * n * U
    res = Mt.residual(A1, A2, b["U1"], b["U2"], b["V1"], b["theta"], ord="fro")
    assert res <= 1e-13 * np.sqrt(n - k)
    # the identity the route rests on, on the known angles themselves
    lam = np.sin(th_true) - np.cos(th_true)
    back = np.pi / 4 + np.arcsin(lam / np.sqrt(2.0))
    assert np.max(np.abs(back - th_true)) <= 4 * U
