"""Pins of the Algorithm 2 oracle (``oracle.repair``, Sec. 5.1), on the CPU.

* Exact recovery: for a well-conditioned A with its exact polar factors
  (through the SVD, a different factorisation), Q Q~^T reproduces W and
  ||R~ - R|| is at rounding level; a transposed Q~ fails this.
* The modified Zolo-pd of Sec. 5.1 on an A with sigma_min below eps leaves
  W~ visibly non-orthonormal; the repair returns an orthonormal W with
  W H~ = A to O(n u), and the acceptance test passes.
* The identity W H~ - A = Q (R~ - R): ||W H~ - A||_F equals ||R~ - R||_F.
* QR with diag(R) >= 0 is the unique one: it matches the Cholesky factor of
  A^T A (a missing sign fix fails this).
"""
import numpy as np
import pytest

from oracle import csd as O
from oracle import repair as R
from oracle import zolo_pd as Z
from paper_1804_09002_amd import workloads as WL

U = 2.0 ** -53


def test_qr_pos_matches_cholesky_factor():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 40))
    Q, Rf = R.qr_pos(A)
    assert np.all(np.diag(Rf) >= 0)
    L = np.linalg.cholesky(A.T @ A)
    assert np.linalg.norm(Rf - L.T) / np.linalg.norm(L) <= 1e-12
    assert np.linalg.norm(Q @ Rf - A) / np.linalg.norm(A) <= 1e-14


@pytest.mark.parametrize("n", [1, 7, 50])
def test_exact_polar_is_recovered(n):
    rng = np.random.default_rng(10 + n)
    A = rng.standard_normal((n, n)) + 3.0 * np.eye(n)
    W, H = O.polar_svd(A)
    Wr, rel = R.polar_repair(A, H)
    assert rel <= 10 * n * U * np.linalg.cond(A)
    assert np.linalg.norm(Wr - W) <= 1e3 * n * U * np.linalg.cond(A)
    assert R.repair_accepted(rel, n)


@pytest.mark.parametrize("n,seed", [(60, 41), (120, 46)])
def test_modified_zolo_pd_is_repaired(n, seed):
    rng = np.random.default_rng(seed)
    theta = WL.angles_cumsum_clustered(n, rng)
    A1, A2, _ = WL.from_angles(theta, rng)
    for A in (A1, A2):
        sig = np.linalg.svd(A, compute_uv=False)
        if sig[-1] >= 1e-15:
            continue
        pd = Z.zolo_pd_svd_form(A, 1e-15, 8)
        Wt, Ht = pd["W"], pd["H"]
        assert np.linalg.norm(Wt.T @ Wt - np.eye(n), 2) > 1e-8  # the modified Zolo-pd alone fails
        W, rel = R.polar_repair(A, Ht)
        assert np.linalg.norm(W.T @ W - np.eye(n), 2) <= 10 * n * U
        assert np.linalg.norm(W @ Ht - A) / np.linalg.norm(A) <= 100 * n * U
        assert R.repair_accepted(rel, n)
        # W H~ - A = Q (R~ - R): the two Frobenius norms agree
        Q, Ra = R.qr_pos(A)
        _, Rt = R.qr_pos(Ht)
        lhs = np.linalg.norm(W @ Ht - A)
        rhs = np.linalg.norm(Rt - Ra)
        assert abs(lhs - rhs) <= 10 * n * U * np.linalg.norm(A)
        break
    else:
        pytest.fail("workload has no singular value below eps")


def test_repair_rejects_a_wrong_symmetric_factor():
    """A symmetric factor that does not belong to A leaves R~ far from R."""
    rng = np.random.default_rng(5)
    n = 30
    A = rng.standard_normal((n, n))
    _, H = O.polar_svd(A)
    _, rel = R.polar_repair(A, H + 1e-6 * np.eye(n))
    assert not R.repair_accepted(rel, n)
