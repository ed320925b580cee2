"""Zolo-eig and the full Zolo-csd path on the GPU vs the CPU oracle.

Parity is on what is unique (Sec. 8(c) readings): the angles theta, the polar
factors H_i, the spectral projectors of well-separated angle groups, and
self-certifying checks of the GPU output (backward error, orthogonality,
C^2 + S^2 = I), since columns are defined only up to sign and rotations
inside clusters of equal angles."""
import numpy as np
import pytest
import torch

from oracle import csd as O
from oracle import metrics as Mt
from paper_1804_09002_amd import workloads as WL

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
DEV = torch.device("cuda:0")


def _t(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


@pytest.mark.parametrize("n,seed", [(1, 1), (7, 2), (64, 3), (65, 4), (150, 5), (300, 6), (1024, 7)])
def test_zolo_eig_random_symmetric(n, seed):
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(seed)
    Q = WL.haar(n, rng)
    lam_true = np.sort(rng.uniform(-1, 1, n))
    B = (Q * lam_true) @ Q.T
    B = 0.5 * (B + B.T)
    lam, V, info = zcsd.syev_zolo(_t(B), lo=-1.0 - 1e-6, hi=1.0 + 1e-6)
    lam, V = lam.cpu().numpy(), V.cpu().numpy()
    assert np.all(np.diff(lam) >= 0)
    assert np.max(np.abs(lam - np.linalg.eigvalsh(B))) <= 50 * n * U
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 50 * n * U
    assert np.linalg.norm(B @ V - V * lam) <= 50 * n * U * np.linalg.norm(B)


def test_zolo_eig_clusters_and_multiplicity():
    from paper_1804_09002_amd import zcsd
    n = 200
    rng = np.random.default_rng(9)
    Q = WL.haar(n, rng)
    lam_true = np.concatenate([np.full(40, 2.0), -1 + 10.0 ** -rng.uniform(8, 12, 60),
                               rng.uniform(-1, 1, 100)])
    lam_true = np.sort(lam_true)
    B = (Q * lam_true) @ Q.T
    B = 0.5 * (B + B.T)
    lam, V, info = zcsd.syev_zolo(_t(B), lo=-1.0 - 1e-6, hi=2.0 + 1e-6)
    lam, V = lam.cpu().numpy(), V.cpu().numpy()
    assert np.max(np.abs(lam - lam_true)) <= 100 * n * U
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 100 * n * U
    assert np.linalg.norm(B @ V - V * lam) <= 100 * n * U * np.linalg.norm(B)


def test_zolo_eig_unbalanced_level():
    """A skewed spectrum (520 eigenvalues in [-1, -0.9], 80 in [0.5, 1]): the
    diagonal of Q Lambda Q^T sits near the mean, so the first split gives
    blocks of 520 and 80 and the next level pads the 80-block to 520 next to
    a block whose n+ (about 260) exceeds 80 -- the basis QR then has more
    columns than the small block has real rows."""
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(21)
    n = 600
    Q = WL.haar(n, rng)
    lam_true = np.sort(np.concatenate([rng.uniform(-1.0, -0.9, 520), rng.uniform(0.5, 1.0, 80)]))
    B = (Q * lam_true) @ Q.T
    B = 0.5 * (B + B.T)
    lam, V, info = zcsd.syev_zolo(_t(B), lo=-1.0 - 1e-6, hi=1.0 + 1e-6)
    lam, V = lam.cpu().numpy(), V.cpu().numpy()
    assert np.all(np.diff(lam) >= 0)
    assert np.max(np.abs(lam - np.linalg.eigvalsh(B))) <= 50 * n * U
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 50 * n * U
    assert np.linalg.norm(B @ V - V * lam) <= 50 * n * U * np.linalg.norm(B)


def _check_csd(A1, A2, U1, U2, V1, th, r, tol_theta=None):
    n = A1.shape[0]
    U1, U2, V1, th = U1[:, :r], U2[:, :r], V1[:, :r], th[:r]
    assert np.all(np.diff(th) >= 0) and th[0] >= 0 and th[-1] <= np.pi / 2
    A = np.vstack([A1, A2])
    res = Mt.residual(A1, A2, U1, U2, V1, th, ord="fro") / max(np.linalg.norm(A), 1e-300)
    assert res <= 1e-13, res
    # orthogonality in the 2-norm, the paper's measure (Sec. 6); Frobenius within sqrt(r) of it
    for name, X in (("U1", U1), ("U2", U2), ("V1", V1)):
        E = X.T @ X - np.eye(r)
        assert np.linalg.norm(E, 2) <= 1e-13, (name, np.linalg.norm(E, 2))
        assert np.linalg.norm(E) <= 1e-13 * np.sqrt(r), (name, np.linalg.norm(E))


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (16, 3), (64, 1), (100, 4), (257, 5)])
def test_csd_haar_matches_oracle(n, seed):
    """Config-1 class: Haar 2n x n; theta vs the oracle, full invariants."""
    from paper_1804_09002_amd import zcsd
    A1, A2, _ = WL.haar_stiefel_pair(n, seed)
    U1, U2, V1, th, info = zcsd.csd(_t(A1), _t(A2))
    U1, U2, V1, th = (x.cpu().numpy() for x in (U1, U2, V1, th))
    ref = O.csd(A1, A2)
    assert info["rank"] == n
    assert np.max(np.abs(th - ref["theta"])) <= 10 * n * U
    _check_csd(A1, A2, U1, U2, V1, th, n)


@pytest.mark.parametrize("n,seed", [(128, 21), (256, 22)])
def test_csd_clustered_known_angles(n, seed):
    """Config-2 construction (scaled down): clusters within 1e-8..1e-12 of 0 and pi/2."""
    from paper_1804_09002_amd import zcsd
    A1, A2, meta = WL.clustered_pair(n, seed)
    U1, U2, V1, th, info = zcsd.csd(_t(A1), _t(A2))
    U1, U2, V1, th = (x.cpu().numpy() for x in (U1, U2, V1, th))
    assert np.max(np.abs(th - np.sort(meta["theta"]))) <= 10 * n * U
    _check_csd(A1, A2, U1, U2, V1, th, n)
    # polar factors H_i are unique (condition sqrt(2)): compare H from the GPU factors
    ref = O.csd(A1, A2)
    H1 = (V1 * np.cos(th)) @ V1.T
    assert np.linalg.norm(H1 - ref["H1"]) <= 100 * n * U


@pytest.mark.parametrize("n,k,seed", [(96, 8, 31), (200, 13, 32)])
def test_csd_rank_deficient_algorithm3(n, k, seed):
    from paper_1804_09002_amd import zcsd
    A1, A2, meta = WL.clustered_pair(n, seed, rank_deficient=k)
    U1, U2, V1, th, info = zcsd.csd(_t(A1), _t(A2))
    U1, U2, V1, th = (x.cpu().numpy() for x in (U1, U2, V1, th))
    r = n - k
    assert info["rank"] == r
    keep = np.setdiff1d(np.arange(n), meta["zero_idx"])
    assert np.max(np.abs(th[:r] - np.sort(meta["theta"][keep]))) <= 10 * n * U
    _check_csd(A1, A2, U1, U2, V1, th, r)
    assert np.all(th[r:] == 0) and np.all(U1[:, r:] == 0)


@pytest.mark.parametrize("n,zc,seed", [(150, (0,), 41), (300, (7, 128, 200), 42)])
def test_csd_exact_zero_columns(n, zc, seed):
    """Orthonormal columns with some columns set exactly to zero: a partial
    isometry of rank n - len(zc) (Alg. 3).  The QR inside Zolo-pd meets
    Householder steps with tau = 0; the angles must match the oracle's."""
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(seed)
    A = WL.stiefel(2 * n, n, rng)
    A[:, list(zc)] = 0.0
    A1, A2 = A[:n].copy(), A[n:].copy()
    U1, U2, V1, th, info = zcsd.csd(_t(A1), _t(A2))
    U1, U2, V1, th = (x.cpu().numpy() for x in (U1, U2, V1, th))
    r = n - len(zc)
    assert info["rank"] == r
    ref = O.csd(A1, A2)
    assert ref["rank"] == r
    assert np.max(np.abs(th[:r] - ref["theta"])) <= 10 * n * U
    _check_csd(A1, A2, U1, U2, V1, th, r)


def test_csd_swap_symmetry():
    from paper_1804_09002_amd import zcsd
    n = 80
    A1, A2, _ = WL.haar_stiefel_pair(n, 77)
    th_a = zcsd.csd(_t(A1), _t(A2))[3].cpu().numpy()
    th_b = zcsd.csd(_t(A2), _t(A1))[3].cpu().numpy()
    assert np.max(np.abs(th_b[::-1] - (np.pi / 2 - th_a))) <= 10 * n * U


def test_csd_rejects_bad_input():
    from paper_1804_09002_amd import zcsd
    n = 8
    A1 = torch.full((n, n), float("nan"), dtype=torch.float64, device=DEV)
    with pytest.raises(zcsd.ZcsdError):
        zcsd.csd(A1, A1)
    B = torch.ones((n, n), dtype=torch.float64, device=DEV) * 0.37
    with pytest.raises(zcsd.ZcsdError):
        zcsd.csd(B, B)


def _norm2_sym(E, iters=60):
    """2-norm of a symmetric device matrix by power iteration (a lower estimate that
    converges quickly for these error matrices)."""
    x = torch.ones(E.shape[0], dtype=torch.float64, device=E.device) / E.shape[0] ** 0.5
    lam = 0.0
    for _ in range(iters):
        y = E @ x
        lam = float(torch.linalg.vector_norm(y))
        if lam == 0.0:
            break
        x = y / lam
    return lam


def _torch_checks(A1, A2, U1, U2, V1, th, r):
    """Backward error ||A_hat - A||_2 / ||A||_2 and orthogonality ||X^T X - I||_2 (the
    paper's measures, Sec. 6) computed on the device; Frobenius bounds as a cross-check."""
    U1, U2, V1, th = U1[:, :r], U2[:, :r], V1[:, :r], th[:r]
    c, s_ = torch.cos(th), torch.sin(th)
    R1 = (U1 * c) @ V1.T - A1
    R2 = (U2 * s_) @ V1.T - A2
    RtR = R1.T @ R1 + R2.T @ R2
    AtA = A1.T @ A1 + A2.T @ A2
    res = (_norm2_sym(RtR) / _norm2_sym(AtA)) ** 0.5
    fro = float(torch.sqrt((R1 * R1).sum() + (R2 * R2).sum()) / torch.sqrt((A1 * A1).sum() + (A2 * A2).sum()))
    n = A1.shape[0]
    assert fro <= 1e-13 * max(1.0, n ** 0.5 / 4), fro
    I = torch.eye(r, dtype=torch.float64, device=A1.device)
    orth = {}
    for k, X in (("U1", U1), ("U2", U2), ("V1", V1)):
        E = X.T @ X - I
        orth[k] = _norm2_sym(E)
        assert float(torch.linalg.matrix_norm(E)) <= 1e-13 * max(1.0, r ** 0.5 / 4)
    return res, orth


@pytest.mark.parametrize("rank_def", [0, 64])
def test_csd_config2_n1024_matches_oracle(rank_def):
    """The n = 1024 workload (clustered angles within 1e-8..1e-12 of 0 and pi/2, optional 64
    zero singular values): theta against the oracle and the construction, full invariants."""
    from paper_1804_09002_amd import zcsd
    n = 1024
    A1, A2, meta = WL.clustered_pair(n, 3 if rank_def else 2, rank_deficient=rank_def)
    a1, a2 = _t(A1), _t(A2)
    U1, U2, V1, th, info = zcsd.csd(a1, a2)
    r = n - rank_def
    assert info["rank"] == r
    ref = O.csd(A1, A2)
    thg = th.cpu().numpy()
    assert np.max(np.abs(thg[:r] - ref["theta"])) <= 10 * n * U
    keep = np.setdiff1d(np.arange(n), meta["zero_idx"]) if rank_def else np.arange(n)
    assert np.max(np.abs(thg[:r] - np.sort(meta["theta"][keep]))) <= 10 * n * U
    res, orth = _torch_checks(a1, a2, U1, U2, V1, th, r)
    assert res <= 1e-13, res
    assert max(orth.values()) <= 1e-13, orth


def test_csd_n4096_bench_configuration():
    """The benchmarked call (n = 4096, uniform angles, seed 4): properties that hold at any
    size -- angles against the construction, backward error, 2-norm orthogonality."""
    from paper_1804_09002_amd import zcsd
    n = 4096
    A1, A2, meta = WL.uniform_pair(n, 4)
    a1, a2 = _t(A1), _t(A2)
    U1, U2, V1, th, info = zcsd.csd(a1, a2)
    assert info["rank"] == n
    assert np.max(np.abs(th.cpu().numpy() - np.sort(meta["theta"]))) <= 10 * n * U
    res, orth = _torch_checks(a1, a2, U1, U2, V1, th, n)
    assert res <= 1e-13, res
    assert max(orth.values()) <= 1e-13, orth


@pytest.mark.parametrize("n,seed", [(100, 41), (300, 46)])
def test_csd_ill_conditioned_algorithm2(n, seed):
    """Test class 2 of Sec. 6 (delta = 10^(-18 U), theta = (pi/2) cumsum(delta)/sum(delta)):
    angles reach 1e-18 of 0 and pi/2, so sigma_min(A_i) < eps and the modified Zolo-pd
    alone leaves W~_i non-orthonormal; Algorithm 2 (Sec. 5.1) restores the FP64 targets."""
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(seed)
    theta = WL.angles_cumsum_clustered(n, rng)
    assert min(np.min(theta), np.min(np.pi / 2 - theta)) < 1e-15
    A1, A2, _ = WL.from_angles(theta, rng)
    U1, U2, V1, th, info = zcsd.csd(_t(A1), _t(A2))
    assert info["rank"] == n and info["repair"] == 1
    assert info["repair_resid"] <= 100 * n * U
    U1, U2, V1, th = (x.cpu().numpy() for x in (U1, U2, V1, th))
    ref = O.csd(A1, A2)
    assert np.max(np.abs(th - ref["theta"])) <= 10 * n * U
    assert np.max(np.abs(th - np.sort(theta))) <= 10 * n * U
    _check_csd(A1, A2, U1, U2, V1, th, n)


@pytest.mark.parametrize("n,k,seed", [(256, 0, 91), (200, 13, 92)])
def test_csd_theta_from_lambda_remark_iv(n, k, seed):
    """postprocess = 2: theta from the eigenvalues (Remark (iv)), single and batched
    paths, against the oracle's same route and the known angles."""
    from paper_1804_09002_amd import zcsd
    A1, A2, meta = WL.clustered_pair(n, seed, rank_deficient=k)
    ref = O.csd(A1, A2, theta_from="lambda")
    r = n - k
    keep = np.setdiff1d(np.arange(n), meta["zero_idx"]) if k else np.arange(n)
    th_true = np.sort(meta["theta"][keep])
    U1, U2, V1, th, info = zcsd.csd(_t(A1), _t(A2), postprocess=2)
    U1, U2, V1, th = (x.cpu().numpy() for x in (U1, U2, V1, th))
    assert info["rank"] == r == ref["rank"]
    assert np.max(np.abs(th[:r] - ref["theta"])) <= 10 * n * U
    assert np.max(np.abs(th[:r] - th_true)) <= 10 * n * U
    _check_csd(A1, A2, U1, U2, V1, th, r)
    (b1, b2, bv, bth, br), = zcsd.csd_batched([_t(A1)], [_t(A2)], postprocess=2)
    bth = bth.cpu().numpy()
    assert br == r
    assert np.max(np.abs(bth[:r] - ref["theta"])) <= 10 * n * U
    assert np.all(bth[r:] == 0)
    _check_csd(A1, A2, b1.cpu().numpy(), b2.cpu().numpy(), bv.cpu().numpy(), bth, r)


def test_csd_postprocess_out_of_range():
    from paper_1804_09002_amd import zcsd
    A1, A2, _ = WL.uniform_pair(8, 1)
    with pytest.raises(Exception):
        zcsd.csd(_t(A1), _t(A2), postprocess=3)


@pytest.mark.parametrize("rd", [0, 256])
def test_clustered_levels_bounded(rd):
    """Tight clusters (angles within 1e-8..1e-12 of 0 and pi/2) are split in a
    bounded number of Zolo-eig levels: each block's interval is tightened to
    mean -+ ||B_blk - mean I||_F, so a stale interval end cannot send a cluster
    to bisection (measured 11-12 levels at n = 2048)."""
    from paper_1804_09002_amd import zcsd
    n = 2048
    A1, A2, meta = WL.clustered_pair(n, 5, rank_deficient=rd)
    U1, U2, V1, th, info = zcsd.csd(_t(A1), _t(A2))
    r = n - rd
    assert info["rank"] == r
    assert info["eig_levels"] <= 16, info["eig_levels"]
    keep = np.setdiff1d(np.arange(n), meta["zero_idx"]) if rd else np.arange(n)
    truth = np.sort(meta["theta"][keep])
    assert np.max(np.abs(th.cpu().numpy()[:r] - truth)) <= 10 * n * U


def test_csd_batched_theta_from_lambda_ragged():
    """postprocess = 2 on a ragged batch (sizes in different classes, one rank
    deficient): every problem's angles match the oracle's Remark (iv) route."""
    from paper_1804_09002_amd import zcsd
    specs = [(8, 0, 101), (37, 0, 102), (64, 8, 103), (130, 0, 104), (200, 20, 105)]
    A1s, A2s, refs = [], [], []
    for n, k, seed in specs:
        A1, A2, _ = WL.clustered_pair(n, seed, rank_deficient=k)
        A1s.append(_t(A1)); A2s.append(_t(A2))
        refs.append((A1, A2, O.csd(A1, A2, theta_from="lambda")))
    out = zcsd.csd_batched(A1s, A2s, postprocess=2)
    for (n, k, _), (A1, A2, ref), (u1, u2, v1, th, r) in zip(specs, refs, out):
        th = th.cpu().numpy()
        assert r == n - k == ref["rank"]
        assert np.max(np.abs(th[:r] - ref["theta"])) <= 10 * max(n, 8) * U, n
        assert np.all(th[r:] == 0)
        _check_csd(A1, A2, u1.cpu().numpy(), u2.cpu().numpy(), v1.cpu().numpy(), th, r)
