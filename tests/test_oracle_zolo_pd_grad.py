"""Pins of the Zolo-pd iterate oracle and of the gradient formulas (CPU)."""
import numpy as np
import pytest

from oracle import csd as O
from oracle import grad as Gd
from oracle import zolo_pd as ZP
from oracle import zolotarev as Z
from paper_1804_09002_amd import workloads as WL

U = 2.0 ** -53


@pytest.mark.parametrize("n,seed,r", [(20, 1, 3), (48, 2, 5)])
def test_zolo_iterates_match_svd_form(n, seed, r):
    """The rational matrix iteration equals P diag(Z_k(sigma)) Q^T (Sec. 5: same singular vectors)."""
    A1, A2, meta = WL.uniform_pair(n, seed)
    smin = np.linalg.svd(A2, compute_uv=False).min()
    ell = 0.5 * smin
    a = ZP.zolo_pd(A2, ell, r)
    b = ZP.zolo_pd_svd_form(A2, ell, r)
    kappa = 1 / smin
    assert np.max(np.abs(a["X1"] - b["X1"])) <= 100 * kappa * U
    assert np.max(np.abs(a["X2"] - b["X2"])) <= 100 * kappa * U


@pytest.mark.parametrize("n,seed", [(32, 3), (64, 4)])
def test_zolo_pd_reaches_polar_factor(n, seed):
    A1, A2, _ = WL.uniform_pair(n, seed)
    for A in (A1, A2):
        smin = np.linalg.svd(A, compute_uv=False).min()
        ell = 0.5 * smin
        r = Z.choose_r(ell)
        out = ZP.zolo_pd(A, ell, r)
        W, H = O.polar_svd(A)
        assert np.linalg.norm(out["W"] - W) <= 1e3 * U / smin
        assert np.linalg.norm(out["H"] - H) <= 1e3 * U
        assert np.linalg.norm(out["W"].T @ out["W"] - np.eye(n)) <= 1e3 * U


def test_modified_zolo_pd_on_rank_deficient_sec51():
    """Sec. 5.1: with eps = 1e-15, the modified Zolo-pd gives H with ||H~ - H|| = O(u)
    although W~ is not orthogonal; ||W~ H~ - A|| = O(u)."""
    n, k = 24, 5
    A1, A2, _ = WL.clustered_pair(n, 7, rank_deficient=k)
    out = ZP.zolo_pd_svd_form(A1, 1e-15, 8)
    _, H = O.polar_svd(A1)
    assert np.linalg.norm(out["H"] - H) <= 1e3 * U
    assert np.linalg.norm(out["W"] @ out["H"] - A1) <= 1e3 * U
    sw = np.linalg.svd(out["W"], compute_uv=False)
    assert sw.max() <= 1 + 1e-14


def _csd_loss(A1, A2, g, G1, G2):
    o = O.csd(A1, A2, rank_mode="full")
    return Gd.csd_loss(o["U1"], o["U2"], o["V1"], o["theta"], o["W1"], o["W2"], g, G1, G2)


@pytest.mark.parametrize("n,seed", [(4, 1), (6, 2)])
def test_gradient_full_fd(n, seed):
    """Every entry of the closed-form gradient against central differences of the oracle."""
    A1, A2, _ = WL.uniform_pair(n, seed)
    rng = np.random.default_rng(seed + 100)
    g = rng.standard_normal(n)
    G1 = rng.standard_normal((n, n))
    G2 = rng.standard_normal((n, n))
    o = O.csd(A1, A2)
    gA1, gA2 = Gd.csd_loss_grad(o["U1"], o["U2"], o["V1"], o["theta"], g, G1, G2)
    h = 1e-6
    for which, gA in ((0, gA1), (1, gA2)):
        fd = np.zeros((n, n))
        for i in range(n):
            for j in range(n):
                P = [A1.copy(), A2.copy()]
                M = [A1.copy(), A2.copy()]
                P[which][i, j] += h
                M[which][i, j] -= h
                fd[i, j] = (_csd_loss(P[0], P[1], g, G1, G2) - _csd_loss(M[0], M[1], g, G1, G2)) / (2 * h)
        assert np.max(np.abs(fd - gA)) <= 1e-7 * max(1.0, np.max(np.abs(gA)))


def test_gradient_fd_h_sweep_second_order():
    n = 5
    A1, A2, _ = WL.uniform_pair(n, 9)
    rng = np.random.default_rng(10)
    g = rng.standard_normal(n)
    G1 = rng.standard_normal((n, n))
    G2 = rng.standard_normal((n, n))
    o = O.csd(A1, A2)
    gA1, gA2 = Gd.csd_loss_grad(o["U1"], o["U2"], o["V1"], o["theta"], g, G1, G2)
    D1 = rng.standard_normal((n, n))
    D2 = rng.standard_normal((n, n))
    exact = np.sum(gA1 * D1) + np.sum(gA2 * D2)
    errs = []
    for h in (1e-3, 1e-4):
        fd = (_csd_loss(A1 + h * D1, A2 + h * D2, g, G1, G2) - _csd_loss(A1 - h * D1, A2 - h * D2, g, G1, G2)) / (2 * h)
        errs.append(abs(fd - exact))
    # central differences are second order: shrinking h by 10 cuts the error ~100x
    assert errs[1] < errs[0] / 30
