"""FP64 MFMA GEMM kernel vs a plain FP64 CPU product (element by element)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _ref(A, B, ta, tb, alpha, beta, C0):
    a = A.T if ta else A
    b = B.T if tb else B
    out = alpha * (a @ b)
    bound = abs(alpha) * (np.abs(a) @ np.abs(b))
    if C0 is not None and beta != 0:
        out = out + beta * C0
        bound = bound + abs(beta) * np.abs(C0)
    return out, bound


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (7, 5, 3), (64, 64, 16), (65, 63, 17), (130, 257, 129),
                                   (300, 200, 1000), (1024, 1024, 256)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_dgemm_matches_cpu(m, n, k, ta, tb):
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(m * 1000 + n * 10 + k)
    A = rng.standard_normal((k, m) if ta else (m, k))
    B = rng.standard_normal((n, k) if tb else (k, n))
    C0 = rng.standard_normal((m, n))
    alpha, beta = 0.75, -0.5
    dev = torch.device("cuda:0")
    out = zcsd.dgemm(torch.tensor(A, device=dev), torch.tensor(B, device=dev), ta, tb, alpha, beta,
                     torch.tensor(C0, device=dev)).cpu().numpy()
    ref, bound = _ref(A, B, ta, tb, alpha, beta, C0)
    err = np.abs(out - ref)
    assert np.all(err <= 2 * (k + 2) * U * bound + 1e-300), float(np.max(err / (bound + 1e-300)))


def test_dgemm_batched_and_beta_zero_ignores_nan():
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(7)
    bs, m, n, k = 5, 96, 80, 48
    A = rng.standard_normal((bs, m, k))
    B = rng.standard_normal((bs, k, n))
    dev = torch.device("cuda:0")
    Cn = torch.full((bs, m, n), float("nan"), dtype=torch.float64, device=dev)
    out = zcsd.dgemm(torch.tensor(A, device=dev), torch.tensor(B, device=dev), C_=Cn, beta=0.0).cpu().numpy()
    ref = np.einsum("bik,bkj->bij", A, B)
    assert np.all(np.isfinite(out))
    assert np.max(np.abs(out - ref)) <= 4 * k * U * np.max(np.abs(A)) * np.max(np.abs(B)) * k


def test_dgemm_empty_k_scales_c():
    from paper_1804_09002_amd import zcsd
    dev = torch.device("cuda:0")
    A = torch.zeros((4, 0), dtype=torch.float64, device=dev)
    B = torch.zeros((0, 3), dtype=torch.float64, device=dev)
    C0 = torch.ones((4, 3), dtype=torch.float64, device=dev)
    out = zcsd.dgemm(A, B, alpha=1.0, beta=2.0, C_=C0)
    assert torch.all(out == 2.0)
