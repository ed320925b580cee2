"""Mixed-precision mode: the FP32-accumulate product and the mixed CSD.

The product on the FP32 matrix cores is compared with the FP64 product on the
CPU against the FP32 rounding bound of an inner product of length k.  The
mixed CSD (FP64 polars, Zolo-eig products in FP32, FP64 refinement of V1) must
meet the same targets as the FP64 path: angles against the oracle (and the
known angles of the construction), 2-norm backward error and orthogonality.
"""
import numpy as np
import pytest
import torch

from oracle import csd as O
from oracle import metrics as Mt
from paper_1804_09002_amd import workloads as WL

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
U32 = 2.0 ** -24
DEV = torch.device("cuda:0")


def _t(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


@pytest.mark.parametrize("ta,tb,m,n,k", [(False, False, 300, 200, 1000), (True, False, 130, 257, 129),
                                         (False, True, 64, 65, 17), (True, True, 1024, 1024, 256),
                                         (False, False, 1, 1, 1)])
def test_dgemm_f32acc_within_fp32_bound(ta, tb, m, n, k):
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(m + 7 * n + 13 * k)
    A = rng.standard_normal((k, m) if ta else (m, k))
    B = rng.standard_normal((n, k) if tb else (k, n))
    C0 = rng.standard_normal((m, n))
    opA = A.T if ta else A
    opB = B.T if tb else B
    ref = 0.5 * opA @ opB - 2.0 * C0
    got = zcsd.dgemm(_t(A), _t(B), transA=ta, transB=tb, alpha=0.5, beta=-2.0, C_=_t(C0),
                     f32acc=True).cpu().numpy()
    bound = (k + 2) * U32 * (0.5 * np.abs(opA) @ np.abs(opB)) + 4 * U * np.abs(2.0 * C0)
    assert np.all(np.abs(got - ref) <= bound)
    if k >= 16:  # and it really is the FP32 path
        assert np.max(np.abs(got - ref)) > 1e3 * U * np.max(np.abs(ref))


def _check(A1, A2, U1, U2, V1, th, r):
    U1, U2, V1, th = U1[:, :r], U2[:, :r], V1[:, :r], th[:r]
    assert np.all(np.diff(th) >= 0)
    A = np.vstack([A1, A2])
    R = np.vstack([(U1 * np.cos(th)) @ V1.T - A1, (U2 * np.sin(th)) @ V1.T - A2])
    res = np.linalg.norm(R, 2) / np.linalg.norm(A, 2)
    assert res <= 1e-13, res
    for X in (U1, U2, V1):
        assert np.linalg.norm(X.T @ X - np.eye(r), 2) <= 1e-13


@pytest.mark.parametrize("case", ["haar64", "haar257", "uniform1024", "clustered256", "rankdef200"])
def test_mixed_csd_meets_fp64_targets(case):
    from paper_1804_09002_amd import zcsd
    truth = None
    if case == "haar64":
        A1, A2, _ = WL.haar_stiefel_pair(64, 71)
    elif case == "haar257":
        A1, A2, _ = WL.haar_stiefel_pair(257, 72)
    elif case == "uniform1024":
        A1, A2, meta = WL.uniform_pair(1024, 73)
        truth = np.sort(meta["theta"])
    elif case == "clustered256":
        A1, A2, meta = WL.clustered_pair(256, 74)
        truth = np.sort(meta["theta"])
    else:
        A1, A2, meta = WL.clustered_pair(200, 75, rank_deficient=13)
    n = A1.shape[0]
    U1, U2, V1, th, info = zcsd.csd(_t(A1), _t(A2), prec="mixed_fp32")
    U1, U2, V1, th = (x.cpu().numpy() for x in (U1, U2, V1, th))
    o = O.csd(A1, A2)
    r = info["rank"]
    assert r == o["rank"]
    assert np.max(np.abs(th[:r] - o["theta"])) <= 10 * n * U
    if truth is not None:
        assert np.max(np.abs(th - truth)) <= 10 * n * U
    _check(A1, A2, U1, U2, V1, th, r)
    assert info["refine_iters"] >= 1


def test_mixed_n4096_bench_configuration():
    """The n = 4096 workload in mixed mode: the FP64 targets hold on the device."""
    from paper_1804_09002_amd import zcsd
    n = 4096
    A1, A2, meta = WL.uniform_pair(n, 4)
    a1, a2 = _t(A1), _t(A2)
    U1, U2, V1, th, info = zcsd.csd(a1, a2, prec="mixed_fp32")
    assert info["rank"] == n
    truth = torch.tensor(np.sort(meta["theta"]), device=DEV)
    assert float((th - truth).abs().max()) <= 10 * n * U
    c, s = torch.cos(th), torch.sin(th)
    R1 = (U1 * c) @ V1.T - a1
    R2 = (U2 * s) @ V1.T - a2
    # 2-norms by power iteration on the symmetric products
    def n2(E, it=60):
        x = torch.ones(E.shape[0], dtype=torch.float64, device=DEV) / E.shape[0] ** 0.5
        lam = 0.0
        for _ in range(it):
            y = E @ x
            lam = float(torch.linalg.vector_norm(y))
            x = y / lam
        return lam
    res = (n2(R1.T @ R1 + R2.T @ R2) / n2(a1.T @ a1 + a2.T @ a2)) ** 0.5
    assert res <= 1e-13, res
    I = torch.eye(n, dtype=torch.float64, device=DEV)
    for X in (U1, U2, V1):
        assert n2(X.T @ X - I) <= 1e-13
