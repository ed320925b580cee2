"""Complete 2 x 2 CSD on the GPU (zcsd_dcsd2x2, Remark (viii) of Sec. 3) against the oracle.

Orthogonal 2n x 2n inputs: Haar, and built from known factors with clustered
angles.  The GPU angles match the oracle's (and the known ones) to 10 n u;
the four factors are orthogonal to 1e-13 and reproduce A to 1e-13 in the
2-norm; V2 equals the oracle's V2 recomputed from the GPU's own U1, U2, theta
(the extra step of the remark, parity of that step) to 1e-12.  A rank-deficient
first block column is rejected.
"""
import numpy as np
import pytest
import torch

from oracle import csd2x2 as C2
from oracle.repair import qr_pos
from paper_1804_09002_amd import workloads as WL

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
DEV = torch.device("cuda:0")


def _t(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


def _inputs(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "haar":
        return WL.haar(2 * n, rng), None
    th = WL.angles_clustered_ends(n, rng)
    F = [WL.haar(n, rng) for _ in range(4)]
    return C2.reconstruct2x2(*F, th), np.sort(th)


@pytest.mark.parametrize("kind,n,seed", [("haar", 1, 1), ("haar", 33, 2), ("haar", 200, 3),
                                         ("clustered", 130, 4), ("haar", 700, 5)])
def test_csd2x2_against_oracle(kind, n, seed):
    from paper_1804_09002_amd import zcsd
    A, truth = _inputs(kind, n, seed)
    A1, A2, A3, A4 = A[:n, :n], A[n:, :n], A[:n, n:], A[n:, n:]
    U1, U2, V1, V2, th, info = zcsd.csd2x2(_t(A1), _t(A2), _t(A3), _t(A4))
    U1, U2, V1, V2, th = (x.cpu().numpy() for x in (U1, U2, V1, V2, th))
    assert info["rank"] == n
    o = C2.csd2x2(A)
    assert np.max(np.abs(th - o["theta"])) <= 10 * n * U
    if truth is not None:
        assert np.max(np.abs(th - truth)) <= 10 * n * U
    for X in (U1, U2, V1, V2):
        assert np.linalg.norm(X.T @ X - np.eye(n), 2) <= 1e-13
    Ah = C2.reconstruct2x2(U1, U2, V1, V2, th)
    assert np.linalg.norm(Ah - A, 2) <= 1e-13
    X = -A3.T @ (U1 * np.sin(th)) + A4.T @ (U2 * np.cos(th))
    V2o, _ = qr_pos(X)
    assert np.max(np.abs(V2 - V2o)) <= 1e-12


def test_csd2x2_rejects_rank_deficient():
    from paper_1804_09002_amd import zcsd
    n = 40
    A, _ = _inputs("haar", n, 7)
    A1 = A[:n, :n].copy()
    A2 = A[n:, :n].copy()
    A1[:, 0] = 0.0
    A2[:, 0] = 0.0  # first block column of rank n - 1
    with pytest.raises(zcsd.ZcsdError):
        zcsd.csd2x2(_t(A1), _t(A2), _t(A[:n, n:]), _t(A[n:, n:]))
