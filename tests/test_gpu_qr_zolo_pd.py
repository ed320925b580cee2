"""Blocked Householder QR (general and stacked [R; sqrt(c) I]) and batched Zolo-pd on
the GPU vs the CPU oracle / plain FP64 definitions."""
import numpy as np
import pytest
import torch

from oracle import csd as O
from oracle import zolo_pd as ZP
from oracle import zolotarev as Z
from paper_1804_09002_amd import workloads as WL

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
DEV = torch.device("cuda:0")


def _t(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


@pytest.mark.parametrize("m,n", [(1, 1), (5, 3), (32, 32), (33, 33), (100, 70), (257, 257), (600, 450),
                                 (2000, 100), (4352 - 1, 40)])
def test_qr_general(m, n):
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(m + 7 * n)
    A = rng.standard_normal((3, m, n))
    R, Q = zcsd.qr(_t(A))
    R, Q = R.cpu().numpy(), Q.cpu().numpy()
    for b in range(3):
        assert np.allclose(np.tril(R[b], -1), 0.0, atol=0)
        assert np.linalg.norm(Q[b] @ R[b] - A[b]) <= 50 * max(m, n) * U * np.linalg.norm(A[b])
        assert np.linalg.norm(Q[b].T @ Q[b] - np.eye(n)) <= 50 * max(m, n) * U
        # R agrees with LAPACK's up to the signs of its rows
        Rl = np.linalg.qr(A[b], mode="r")
        sgn = np.sign(np.diag(R[b])) * np.sign(np.diag(Rl))
        assert np.allclose(sgn[:, None] * R[b], Rl, atol=1e-12 * np.abs(Rl).max())


@pytest.mark.parametrize("m,n,zc", [(300, 200, (0, 45, 130)), (600, 450, (3, 31, 32, 127, 128, 300))])
def test_qr_exact_zero_columns(m, n, zc):
    """An exactly zero column gives a Householder step with tau = 0 (H = I).
    The compact-WY factors of the outer blocks must keep such steps decoupled
    (zero row and column of T), as the panel's own factor does, or the
    trailing columns and Q see a different reflector than the panel did."""
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((2, m, n))
    A[:, :, list(zc)] = 0.0
    R, Q = zcsd.qr(_t(A))
    R, Q = R.cpu().numpy(), Q.cpu().numpy()
    for b in range(2):
        assert np.allclose(np.tril(R[b], -1), 0.0, atol=0)
        assert np.linalg.norm(Q[b] @ R[b] - A[b]) <= 50 * m * U * np.linalg.norm(A[b])
        assert np.linalg.norm(Q[b].T @ Q[b] - np.eye(n)) <= 50 * m * U
        # R(:, j) = Q^T A(:, j) = 0 for a zero column; R is unique (up to row
        # signs) only above the first zero column's row, where it matches LAPACK's
        assert np.max(np.abs(R[b][:, list(zc)])) <= 50 * m * U * np.linalg.norm(A[b])
        k = min(zc)
        Rl = np.linalg.qr(A[b], mode="r")
        assert np.allclose(np.abs(R[b][:k]), np.abs(Rl[:k]), atol=1e-12 * np.abs(Rl).max())


@pytest.mark.parametrize("n,c", [(1, 0.3), (31, 1e-6), (64, 0.5), (97, 1e-12), (300, 2.0), (700, 1e-3)])
def test_qr_stacked_structure(n, c):
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(n)
    R0 = np.triu(rng.standard_normal((2, n, n)))
    S = np.concatenate([R0, np.broadcast_to(np.sqrt(c) * np.eye(n), (2, n, n))], axis=1)
    R, Q = zcsd.qr(_t(S), stacked=True)
    R, Q = R.cpu().numpy(), Q.cpu().numpy()
    for b in range(2):
        nrm = np.linalg.norm(S[b])
        assert np.linalg.norm(Q[b] @ R[b] - S[b]) <= 50 * n * U * nrm
        assert np.linalg.norm(Q[b].T @ Q[b] - np.eye(n)) <= 50 * n * U
        # R^T R = R0^T R0 + c I (same triangular factor as the unstructured QR up to row signs)
        Rl = np.linalg.qr(S[b], mode="r")
        sgn = np.sign(np.diag(R[b])) * np.sign(np.diag(Rl))
        assert np.allclose(sgn[:, None] * R[b], Rl, atol=1e-12 * np.abs(Rl).max())


def _zolo_case(n, seed, which):
    A1, A2, meta = WL.uniform_pair(n, seed)
    return A1 if which == 1 else A2


@pytest.mark.parametrize("n,seed", [(40, 1), (129, 2), (300, 3)])
def test_zolo_pd_iterates_match_oracle(n, seed):
    """Forced (l, r): X1, W, H against the oracle's matrix-function iterates."""
    from paper_1804_09002_amd import zcsd
    A = _zolo_case(n, seed, 2)
    smin = np.linalg.svd(A, compute_uv=False).min()
    ell = 0.5 * smin
    r = Z.choose_r(ell)
    ref = ZP.zolo_pd_svd_form(A, ell, r)
    W, H, X1, info = zcsd.zolo_pd(_t(A), r=r, ell=ell, want_X1=True)
    W, H, X1 = W.cpu().numpy(), H.cpu().numpy(), X1.cpu().numpy()
    assert info["r_used"][0] == r and abs(info["ell"][0] - ell) < 1e-15 * ell + 1e-300
    kappa = 1.0 / smin
    assert np.linalg.norm(X1 - ref["X1"]) <= 1e3 * n * U * np.linalg.norm(ref["X1"]) * max(1, kappa ** 0.5)
    assert np.linalg.norm(W - ref["W"]) <= 100 * n * U * kappa
    assert np.linalg.norm(H - ref["H"]) <= 100 * n * U
    assert np.linalg.norm(W.T @ W - np.eye(n)) <= 100 * n * U
    Wp, Hp = O.polar_svd(A)
    assert np.linalg.norm(H - Hp) <= 100 * n * U


@pytest.mark.parametrize("n,seed", [(64, 4), (200, 5)])
def test_zolo_pd_estimates_ell_and_batches(n, seed):
    """Automatic l (lower bound of sigma_min) and r; two matrices in one batch."""
    from paper_1804_09002_amd import zcsd
    A1, A2, meta = WL.uniform_pair(n, seed)
    X = np.stack([A1, A2])
    W, H, _, info = zcsd.zolo_pd(_t(X))
    W, H = W.cpu().numpy(), H.cpu().numpy()
    smin = min(np.linalg.svd(A1, compute_uv=False).min(), np.linalg.svd(A2, compute_uv=False).min())
    assert info["ell"][0] <= smin
    assert info["zolo_resid"] <= U
    for b, A in enumerate((A1, A2)):
        Wp, Hp = O.polar_svd(A)
        assert np.linalg.norm(H[b] - Hp) <= 100 * n * U
        assert np.linalg.norm(W[b] @ H[b] - A) <= 100 * n * U
        assert np.linalg.norm(W[b].T @ W[b] - np.eye(n)) <= 100 * n * U


def test_modified_zolo_pd_rank_deficient():
    """Sec. 5.1: l = eps = 1e-15, r = 8 on a singular A: H correct to O(u), W~ H~ = A."""
    from paper_1804_09002_amd import zcsd
    n = 96
    A1, A2, _ = WL.clustered_pair(n, 8, rank_deficient=7)
    W, H, _, info = zcsd.zolo_pd(_t(A1), r=8, ell=1e-15)
    W, H = W.cpu().numpy(), H.cpu().numpy()
    _, Hp = O.polar_svd(A1)
    assert np.linalg.norm(H - Hp) <= 200 * n * U
    assert np.linalg.norm(W @ H - A1) <= 200 * n * U
    assert np.linalg.svd(W, compute_uv=False).max() <= 1 + 1e-13
