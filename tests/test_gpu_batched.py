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


def test_batched_member_below_eps_takes_algorithm2():
    """A full-rank member whose angles reach 1e-18 of 0 and pi/2 (test class 2
    of Sec. 6, sigma_min(A_i) < eps) shares a size class with a uniform member:
    the class's lower bound l reaches eps, the class runs through the single
    path with Algorithm 2 (Sec. 5.1), and every member meets the FP64 targets
    and the oracle's angles."""
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(41)
    n_bad = 44
    theta = WL.angles_cumsum_clustered(n_bad, rng)
    assert min(np.min(theta), np.min(np.pi / 2 - theta)) < 1e-15
    A1b, A2b, _ = WL.from_angles(theta, rng)
    A1u, A2u, _ = WL.uniform_pair(48, 48)     # same size class (48) as n = 44
    A1o, A2o, _ = WL.uniform_pair(20, 49)     # another class, batched as usual
    A1s, A2s = [A1b, A1u, A1o], [A2b, A2u, A2o]
    a1, sizes, offs = zcsd.pack_ragged([_t(a) for a in A1s])
    a2, _, _ = zcsd.pack_ragged([_t(a) for a in A2s])
    U1, U2, V1, th, ranks, info = zcsd.csd_batched_packed(a1, a2, sizes, offs)
    assert info["repair"] >= 1
    t0 = 0
    for k, n in enumerate(sizes):
        o = offs[k]
        u1, u2, v1 = (X[o:o + n * n].view(n, n).t() for X in (U1, U2, V1))
        t = th[t0:t0 + n]
        t0 += n
        assert ranks[k] == n
        ref = O.csd(A1s[k], A2s[k])
        assert np.max(np.abs(t.cpu().numpy() - ref["theta"])) <= 10 * n * U, k
        res, orth = _self_checks(_t(A1s[k]), _t(A2s[k]), u1, u2, v1, t, n)
        assert res <= 1e-13 and orth <= 1e-13, (k, n, res, orth)


def test_batched_many_rank_deficient_members_in_one_class():
    """4100 rank-deficient problems of size 8 in one size class: more members
    than one launch grid of the polars can hold (2 polars x 8 terms x 4100 >
    65535), so the class is split into chunks; every member keeps rank 7, the
    FP64 targets and its known angles, and sampled members match the oracle."""
    from paper_1804_09002_amd import zcsd
    count, n = 4100, 8
    rng = np.random.default_rng(51)
    A1s, A2s, truth = [], [], []
    for _ in range(count):
        theta = WL.angles_uniform(n, rng)
        z = np.array([int(rng.integers(n))])
        A1, A2, meta = WL.from_angles(theta, rng, zero_idx=z)
        A1s.append(A1); A2s.append(A2); truth.append(np.sort(np.delete(theta, z)))
    a1 = _t(np.concatenate([a.T.reshape(-1) for a in A1s]))
    a2 = _t(np.concatenate([a.T.reshape(-1) for a in A2s]))
    sizes, offs = [n] * count, [k * n * n for k in range(count)]
    U1, U2, V1, th, ranks, info = zcsd.csd_batched_packed(a1, a2, sizes, offs)
    assert all(r == n - 1 for r in ranks)
    cm = lambda X: X.view(count, n, n).transpose(1, 2)
    u1, u2, v1, t = cm(U1), cm(U2), cm(V1), th.view(count, n)
    A1t, A2t = cm(a1), cm(a2)
    r = n - 1
    c, s = torch.cos(t[:, :r]), torch.sin(t[:, :r])
    R1 = (u1[:, :, :r] * c[:, None, :]) @ v1[:, :, :r].transpose(1, 2) - A1t
    R2 = (u2[:, :, :r] * s[:, None, :]) @ v1[:, :, :r].transpose(1, 2) - A2t
    res = torch.sqrt((R1 ** 2).sum((1, 2)) + (R2 ** 2).sum((1, 2))) / np.sqrt(r)
    assert float(res.max()) <= 1e-13
    I = torch.eye(r, dtype=torch.float64, device=DEV)
    for X in (u1, u2, v1):
        Xr = X[:, :, :r]
        E = Xr.transpose(1, 2) @ Xr - I
        assert float(torch.sqrt((E ** 2).sum((1, 2))).max()) <= 1e-13
    th_true = torch.tensor(np.stack(truth), device=DEV)
    assert float((t[:, :r] - th_true).abs().max()) <= 10 * n * U
    assert float(t[:, r:].abs().max()) == 0.0
    for k in (0, 2049, count - 1):
        ref = O.csd(A1s[k], A2s[k])
        assert ref["rank"] == r
        assert np.max(np.abs(t[k, :r].cpu().numpy() - ref["theta"])) <= 10 * n * U
