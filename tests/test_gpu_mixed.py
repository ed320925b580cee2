"""Mixed-precision mode: the FP32-accumulate product and the mixed CSD.

The product on the FP32 matrix cores is compared with the FP64 product on the
CPU against the FP32 rounding bound of an inner product of length k.  The
mixed CSD (iteration 2 of the polars and all of Zolo-eig on the FP32 matrix
cores, FP64 Newton-Schulz steps on the polar factors and V1) is held to its
stated tolerance TAU_MIXED: angles against the oracle (and the known angles
of the construction), the 2-norm backward error and the orthogonality of U1,
U2, V1.
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


# the mixed mode's stated tolerance for every output measure: 2-norm backward
# error, orthogonality of U1, U2, V1, and the angles (FP32 products: unit
# roundoff 2^-24 ~ 6e-8, accumulated over inner dimensions up to n; measured
# 2-4e-6 backward error, orthogonality below 1e-9 after the FP64
# Newton-Schulz steps, angles within 1e-7 at n = 1024 and 4096)
TAU_MIXED = 1e-5


def _check(A1, A2, U1, U2, V1, th, r):
    """2-norm backward error (returned) and orthogonality of the r valid columns."""
    U1, U2, V1, th = U1[:, :r], U2[:, :r], V1[:, :r], th[:r]
    assert np.all(np.diff(th) >= 0)
    A = np.vstack([A1, A2])
    R = np.vstack([(U1 * np.cos(th)) @ V1.T - A1, (U2 * np.sin(th)) @ V1.T - A2])
    res = np.linalg.norm(R, 2) / np.linalg.norm(A, 2)
    for X in (U1, U2, V1):
        assert np.linalg.norm(X.T @ X - np.eye(r), 2) <= TAU_MIXED
    return res


@pytest.mark.parametrize("case", ["haar64", "haar257", "uniform1024", "clustered256", "rankdef200"])
def test_mixed_csd_meets_stated_tolerance(case):
    """The mixed mode on the FP32 matrix cores (info.lowp_products > 0, no FP64
    fallback exists): angles within TAU_MIXED of the oracle's (and of the
    construction's), backward error and orthogonality within TAU_MIXED; the
    FP64 mode on the same input runs no FP32 product."""
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
    assert info["lowp_products"] > 0
    U1, U2, V1, th = (x.cpu().numpy() for x in (U1, U2, V1, th))
    o = O.csd(A1, A2)
    r = info["rank"]
    assert r == o["rank"]
    dth = float(np.max(np.abs(th[:r] - o["theta"])))
    res = _check(A1, A2, U1, U2, V1, th, r)
    print(f"mixed {case}: max |dtheta| {dth:.2e}, backward {res:.2e}, "
          f"FP32 products {info['lowp_products']}", flush=True)
    assert dth <= TAU_MIXED
    assert res <= TAU_MIXED
    if truth is not None:
        assert np.max(np.abs(th - truth)) <= TAU_MIXED
    *_, info64 = zcsd.csd(_t(A1), _t(A2))
    assert info64["lowp_products"] == 0


def test_mixed_n4096_bench_configuration():
    """The n = 4096 workload in mixed mode: the stated tolerance on the device."""
    from paper_1804_09002_amd import zcsd
    n = 4096
    A1, A2, meta = WL.uniform_pair(n, 4)
    a1, a2 = _t(A1), _t(A2)
    U1, U2, V1, th, info = zcsd.csd(a1, a2, prec="mixed_fp32")
    assert info["rank"] == n and info["lowp_products"] > 0
    truth = torch.tensor(np.sort(meta["theta"]), device=DEV)
    dth = float((th - truth).abs().max())
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
    print(f"mixed n=4096: max |dtheta| {dth:.2e}, backward {res:.2e}", flush=True)
    assert dth <= TAU_MIXED
    assert res <= TAU_MIXED, res
    I = torch.eye(n, dtype=torch.float64, device=DEV)
    for X in (U1, U2, V1):
        assert n2(X.T @ X - I) <= TAU_MIXED
