"""The accuracy study of Sec. 6 on the GPU path against the CPU oracle.

Test classes 1-4 and the noisy 1'-4' (real analogues, ``paper_test_class``) at
three of the paper's sizes n = nint(30 * 2^(j/2)) (j = 0, 3, 6).  For each
input the GPU decomposition must have the same rank as the oracle's, a scaled
residual ||A_hat - A||_2 / d(A) within a small factor of the oracle's (the
backward stability of Theorem 4.1: the error is a modest multiple of the
distance d(A) to the partial isometries, plus rounding), orthonormal factors
to 1e-13, and, on the exact partial isometries (classes 1-4), the oracle's
angles to 10 n u.
"""
import numpy as np
import pytest
import torch

from oracle import csd as O
from oracle import metrics as Mt
from paper_1804_09002_amd import workloads as WL

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
DEV = torch.device("cuda:0")


@pytest.mark.parametrize("n", [30, 85, 240])
@pytest.mark.parametrize("cls", list(WL.PAPER_CLASSES))
def test_paper_class_against_oracle(cls, n):
    from paper_1804_09002_amd import zcsd
    from paper_1804_09002_amd.accuracy_study import measures
    rng = np.random.default_rng(11 * 100003 + n)
    A1, A2 = WL.paper_test_class(cls, n, rng)
    U1, U2, V1, th, info = zcsd.csd(torch.tensor(A1, device=DEV), torch.tensor(A2, device=DEV))
    U1, U2, V1, th = (x.cpu().numpy() for x in (U1, U2, V1, th))
    o = O.csd(A1, A2)
    r = o["rank"]
    assert info["rank"] == r
    if cls in ("1", "2"):
        assert r == n
    if cls in ("3", "4", "3'", "4'"):
        assert r == int(np.rint(3 * n / 4))
    g = measures(A1, A2, U1, U2, V1, th, r)
    # the oracle's own measures on the same input (the metric functions of the oracle)
    A = np.vstack([A1, A2])
    dA = Mt.d_partial_isometry(A)
    assert abs(dA - g["dA"]) <= 1e-12 * max(dA, 1e-300)
    o_res = Mt.residual(A1, A2, o["U1"], o["U2"], o["V1"], o["theta"]) / dA
    assert g["res_dA"] <= max(10.0 * o_res, 100.0), (g["res_dA"], o_res)
    if cls.endswith("'"):
        assert g["res_dA"] <= 10.0  # the noise dominates: a modest multiple of d(A)
    assert max(g["orth_u"]) * U <= 1e-13
    if not cls.endswith("'"):
        assert np.max(np.abs(th[:r] - o["theta"])) <= 10 * n * U
