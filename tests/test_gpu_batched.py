"""Batched Zolo-csd (zcsd_dcsd_batched) on ragged sizes vs the oracle and the
single-problem path.

Per problem the checks are those of the single path: angles against the oracle
(and against the known angles of the construction), and self-certifying
checks of the GPU output (2-norm backward error, orthogonality of the valid
columns), since columns are unique only up to sign and rotations inside
clusters of equal angles.
"""
import numpy as np
import pytest
import torch

from oracle import csd as O
from paper_1804_09002_amd import workloads as WL

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
DEV = torch.device("cuda:0")


def _t(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


def _norm2(E):
    return float(torch.linalg.matrix_norm(E, ord=2)) if E.numel() else 0.0


def _self_checks(A1, A2, U1, U2, V1, th, r):
    """2-norm backward error and orthogonality of the r valid columns (on the device)."""
    c, s = torch.cos(th[:r]), torch.sin(th[:r])
    R = torch.cat([(U1[:, :r] * c) @ V1[:, :r].T - A1, (U2[:, :r] * s) @ V1[:, :r].T - A2])
    A = torch.cat([A1, A2])
    res = _norm2(R) / max(_norm2(A), 1e-300)
    I = torch.eye(r, dtype=torch.float64, device=DEV)
    orth = max(_norm2(X[:, :r].T @ X[:, :r] - I) for X in (U1, U2, V1)) if r else 0.0
    return res, orth


def test_batched_ragged_matches_oracle_and_single_path():
    from paper_1804_09002_amd import zcsd
    sizes = [1, 2, 7, 8, 9, 15, 16, 17, 33, 64, 65, 100, 130]
    A1s, A2s, truth = [], [], []
    for k, n in enumerate(sizes):
        A1, A2, meta = WL.uniform_pair(n, 500 + k)
        A1s.append(A1); A2s.append(A2); truth.append(np.sort(meta["theta"]))
    # one rank-deficient member (Algorithm 3) and one clustered member
    A1, A2, meta = WL.clustered_pair(40, 540, rank_deficient=5)
    A1s.append(A1); A2s.append(A2); truth.append(None)
    A1, A2, meta = WL.clustered_pair(48, 541)
    A1s.append(A1); A2s.append(A2); truth.append(None)
    out = zcsd.csd_batched([_t(a) for a in A1s], [_t(a) for a in A2s])
    for k, (U1, U2, V1, th, r) in enumerate(out):
        n = A1s[k].shape[0]
        o = O.csd(A1s[k], A2s[k])
        assert r == o["rank"], (k, r, o["rank"])
        thh = th.cpu().numpy()
        assert np.all(np.diff(thh[:r]) >= 0) and np.all(thh[r:] == 0.0)
        assert np.max(np.abs(thh[:r] - o["theta"])) <= 10 * max(n, 8) * U, k
        if truth[k] is not None:
            assert np.max(np.abs(thh[:r] - truth[k])) <= 10 * max(n, 8) * U, k
        res, orth = _self_checks(_t(A1s[k]), _t(A2s[k]), U1, U2, V1, th, r)
        assert res <= 1e-13 and orth <= 1e-13, (k, n, res, orth)
        assert torch.all(U1[:, r:] == 0) and torch.all(V1[:, r:] == 0)
        if k in (6, 11):  # same angles as the single path
            s1, s2, sv, sth, info = zcsd.csd(_t(A1s[k]), _t(A2s[k]))
            assert float((sth - th).abs().max()) <= 10 * n * U


def _self_checks_fro(A1, A2, U1, U2, V1, th, r):
    """Frobenius-norm versions (cheap enough for thousands of problems)."""
    c, s = torch.cos(th[:r]), torch.sin(th[:r])
    R = torch.cat([(U1[:, :r] * c) @ V1[:, :r].T - A1, (U2[:, :r] * s) @ V1[:, :r].T - A2])
    res = float(torch.linalg.norm(R) / torch.linalg.norm(torch.cat([A1, A2])))
    I = torch.eye(r, dtype=torch.float64, device=DEV)
    orth = max(float(torch.linalg.norm(X[:, :r].T @ X[:, :r] - I)) for X in (U1, U2, V1))
    return res, orth


def test_batched_rejects_bad_input():
    from paper_1804_09002_amd import zcsd
    A1, A2, _ = WL.uniform_pair(8, 1)
    bad = A1.copy()
    bad[3, 2] = np.nan
    with pytest.raises(zcsd.ZcsdError):
        zcsd.csd_batched([_t(A1), _t(bad)], [_t(A2), _t(A2)])
    with pytest.raises(ValueError):
        zcsd.csd_batched([_t(A1)], [_t(A2[:4, :4])])


def test_batched_workload_2048_log_uniform_sizes():
    """2048 problems, n log-uniform in [8, 256] (seed 5), uniform angles: every
    problem passes the self-certifying checks and matches its known angles;
    three sampled problems match the oracle."""
    from paper_1804_09002_amd import zcsd
    sizes = WL.batched_sizes(2048, 5)
    rng = np.random.default_rng(5)
    A1s, A2s, truth = [], [], []
    for n in sizes:
        A1, A2, meta = WL.uniform_pair(int(n), int(rng.integers(1 << 31)))
        A1s.append(_t(A1)); A2s.append(_t(A2)); truth.append(np.sort(meta["theta"]))
    out = zcsd.csd_batched(A1s, A2s)
    worst_res = worst_orth = worst_th = 0.0
    for k, (U1, U2, V1, th, r) in enumerate(out):
        n = int(sizes[k])
        assert r == n
        worst_th = max(worst_th, float(np.max(np.abs(th.cpu().numpy() - truth[k]))) / n)
        res, orth = _self_checks_fro(A1s[k], A2s[k], U1, U2, V1, th, r)
        # Frobenius norms grow like sqrt(n) over the 2-norm targets of 1e-13
        lim = 1e-13 * max(1.0, np.sqrt(n) / 4)
        worst_res, worst_orth = max(worst_res, res / lim), max(worst_orth, orth / lim)
    assert worst_res <= 1.0 and worst_orth <= 1.0, (worst_res, worst_orth)
    assert worst_th <= 10 * U, worst_th
    for k in (0, 1000, 2047):
        o = O.csd(A1s[k].cpu().numpy(), A2s[k].cpu().numpy())
        assert np.max(np.abs(out[k][3].cpu().numpy() - o["theta"])) <= 10 * int(sizes[k]) * U
