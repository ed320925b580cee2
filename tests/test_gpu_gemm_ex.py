"""The product kernels' structure options against a plain FP64 CPU product,
element by element (zcsd_dgemm_ex on column-major buffers).

* the 128 x 128 tile kernel (chosen from 512 output tiles on; interior tiles
  load and store without bounds checks), all four transpose cases, with
  partial edge tiles;
* triangular operands (tri bits 1, 2, 4, 8 within k segments): the kernel
  skips k ranges whose products are exact zeros, so its result must be
  bit-identical to the dense product of the same operands;
* symmetric products (only tiles on or above the diagonal) and upper-only
  products with beta != 0 (tiles below the diagonal keep their contents);
* the deterministic split of k across workgroups with a caller workspace,
  with room for all splits and for fewer;
* the same options on the FP32 matrix-core kernel, against the FP32 bound.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
U32 = 2.0 ** -24
DEV = torch.device("cuda:0")


def _cm(X):
    """(batch, rows, cols) numpy -> device (batch, cols, rows): column-major buffers."""
    return torch.tensor(np.ascontiguousarray(np.swapaxes(X, 1, 2)), device=DEV)


def _back(T):
    return np.swapaxes(T.cpu().numpy(), 1, 2)


def _op(X, t):
    return np.swapaxes(X, 1, 2) if t else X


def _bound(Aop, Bop, alpha, beta, C0, k, f32):
    prod = abs(alpha) * np.einsum("bik,bkj->bij", np.abs(Aop), np.abs(Bop))
    lin = abs(beta) * np.abs(C0)
    if f32:
        return (k + 4) * U32 * prod + 4 * U * lin + 1e-300
    return 2 * (k + 2) * U * (prod + lin) + 1e-300


def _run(A, B, C0, ta, tb, alpha, beta, f32=False, flags=0, tri=0, kseg=0, ws=None):
    from paper_1804_09002_amd import zcsd
    Aop, Bop = _op(A, ta), _op(B, tb)
    bs, m, k = Aop.shape
    n = Bop.shape[2]
    C = _cm(C0)
    zcsd.dgemm_ex(_cm(A), _cm(B), C, ta, tb, m, n, k, alpha, beta,
                  flags=flags | (zcsd.GEMM_F32ACC if f32 else 0), tri=tri, kseg=kseg, ws=ws)
    ref = alpha * np.einsum("bik,bkj->bij", Aop, Bop) + beta * C0
    return _back(C), ref, _bound(Aop, Bop, alpha, beta, C0, k, f32), C


def _operands(rng, bs, m, n, k, ta, tb):
    A = rng.standard_normal((bs, k, m) if ta else (bs, m, k))
    B = rng.standard_normal((bs, n, k) if tb else (bs, k, n))
    return A, B, rng.standard_normal((bs, m, n))


@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("bs,m,n,k", [(8, 1024, 1024, 320), (9, 1000, 1030, 200)])
def test_large_tile_kernel(bs, m, n, k, ta, tb, f32):
    """Enough tiles for the 128 x 128 kernel (8 x 64 = 512 and 9 x 72 = 648)."""
    rng = np.random.default_rng(bs * 7 + m + 3 * n + k + 2 * ta + tb)
    A, B, C0 = _operands(rng, bs, m, n, k, ta, tb)
    out, ref, bound, _ = _run(A, B, C0, ta, tb, 0.75, -0.5, f32)
    err = np.abs(out - ref)
    assert np.all(err <= bound), float(np.max(err / bound))


def _tri_operands(rng, bs, m, n, nseg, kseg, tri, ta, tb):
    """op(A) (m x nseg*kseg) and op(B) (nseg*kseg x n) with the zero pattern of
    `tri` inside every segment, stored with the requested transposes."""
    k = nseg * kseg
    Aop = rng.standard_normal((bs, m, k))
    Bop = rng.standard_normal((bs, k, n))
    kk = np.arange(k) % kseg
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    if tri & 1:
        Aop[:, kk[None, :] < i] = 0.0
    if tri & 2:
        Aop[:, kk[None, :] > i] = 0.0
    if tri & 4:
        Bop[:, kk[:, None] > j] = 0.0
    if tri & 8:
        Bop[:, kk[:, None] < j] = 0.0
    A = np.swapaxes(Aop, 1, 2).copy() if ta else Aop
    B = np.swapaxes(Bop, 1, 2).copy() if tb else Bop
    return A, B


@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("tri,ta,tb", [(1 | 8, False, True), (4, True, False), (1, False, False),
                                       (2, True, False), (8, False, False), (1 | 4, False, False),
                                       (2 | 8, False, True)])
@pytest.mark.parametrize("bs,m,n,nseg,kseg", [(2, 200, 200, 3, 200), (8, 1024, 1024, 1, 1024)])
def test_triangular_operands_skip_exact_zeros(bs, m, n, nseg, kseg, tri, ta, tb, f32):
    """Skipping is exact: the result equals the dense product of the same operands
    bit for bit (a skipped term would add an exact zero), and the CPU product to
    the rounding bound.  The second shape reaches the 128 x 128 kernel."""
    rng = np.random.default_rng(tri * 101 + bs + m + nseg)
    A, B = _tri_operands(rng, bs, m, n, nseg, kseg, tri, ta, tb)
    C0 = rng.standard_normal((bs, m, n))
    out, ref, bound, Ct = _run(A, B, C0, ta, tb, 1.25, 0.5, f32, tri=tri, kseg=kseg)
    dense, _, _, Cd = _run(A, B, C0, ta, tb, 1.25, 0.5, f32)
    assert torch.equal(Ct, Cd)
    assert np.all(np.abs(out - ref) <= bound), float(np.max(np.abs(out - ref) / bound))


@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("bs,n,k", [(1, 300, 77), (4, 1024, 256)])
def test_symmetric_and_upper_only(bs, n, k, f32):
    """ZCSD_GEMM_SYM_UPPER (beta = 0) and ZCSD_GEMM_UPPER_ONLY (beta != 0): every
    entry on or above the diagonal is the product; an entry below it is either
    untouched (a tile below the diagonal) or the product."""
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(bs + n + k)
    X = rng.standard_normal((bs, k, n))
    C0 = rng.standard_normal((bs, n, n))
    iu = np.triu(np.ones((n, n), dtype=bool))
    # symmetric: X^T X, C filled with NaN (beta = 0 never reads it)
    C = _cm(np.full((bs, n, n), np.nan))
    zcsd.dgemm_ex(_cm(X), _cm(X), C, True, False, n, n, k, 1.0, 0.0,
                  flags=zcsd.GEMM_SYM_UPPER | (zcsd.GEMM_F32ACC if f32 else 0))
    got = _back(C)
    ref = np.einsum("bki,bkj->bij", X, X)
    bound = _bound(np.swapaxes(X, 1, 2), X, 1.0, 0.0, np.zeros_like(ref), k, f32)
    assert np.all(np.isfinite(got[:, iu]))
    assert np.all(np.abs(got[:, iu] - ref[:, iu]) <= bound[:, iu])
    low = ~iu
    computed = np.isfinite(got[:, low])
    assert np.all(np.abs(got[:, low][computed] - ref[:, low][computed]) <= bound[:, low][computed])
    assert not np.all(computed) or n <= 64  # some tiles below the diagonal were skipped
    # upper only, beta != 0
    Y = rng.standard_normal((bs, n, k))
    out, ref2, bound2, _ = _run(Y, X, C0, False, False, -0.5, 2.0, f32, flags=zcsd.GEMM_UPPER_ONLY)
    assert np.all(np.abs(out[:, iu] - ref2[:, iu]) <= bound2[:, iu])
    kept = out[:, low] == C0[:, low]
    assert np.all(np.abs(out[:, low][~kept] - ref2[:, low][~kept]) <= bound2[:, low][~kept])


@pytest.mark.parametrize("ws_splits", [16, 3])
@pytest.mark.parametrize("ta,tb", [(True, False), (False, False)])
def test_split_k_with_workspace(ta, tb, ws_splits):
    """Few output tiles (2 x 2 x 2 of 64 x 64) and k = 4096: the product splits k
    across workgroups into the workspace and reduces the partials in a fixed
    order; a workspace with room for 3 partial products limits it to 3 splits.
    Matches the CPU product and the unsplit product to the rounding bound."""
    from paper_1804_09002_amd import zcsd
    bs, m, n, k = 2, 128, 128, 4096
    rng = np.random.default_rng(ws_splits + 2 * ta + tb)
    A, B, C0 = _operands(rng, bs, m, n, k, ta, tb)
    ws = torch.empty(ws_splits * bs * m * n, dtype=torch.float64, device=DEV)
    out, ref, bound, _ = _run(A, B, C0, ta, tb, 0.5, 1.5, ws=ws)
    assert np.all(np.abs(out - ref) <= bound), float(np.max(np.abs(out - ref) / bound))
    plain, _, _, _ = _run(A, B, C0, ta, tb, 0.5, 1.5)
    assert np.all(np.abs(out - plain) <= 2 * bound)
    assert not np.array_equal(out, plain)  # the split really ran (different summation order)


def test_dgemm_ex_rejects_bad_options():
    from paper_1804_09002_amd import zcsd
    A = torch.zeros((1, 8, 8), dtype=torch.float64, device=DEV)
    C = torch.zeros((1, 8, 8), dtype=torch.float64, device=DEV)
    for kw in ({"flags": 8}, {"tri": 16, "kseg": 8}, {"tri": 1, "kseg": 3},
               {"flags": zcsd.GEMM_SYM_UPPER, "beta": 1.0}):
        beta = kw.pop("beta", 0.0)
        with pytest.raises(zcsd.ZcsdError):
            zcsd.dgemm_ex(A, A, C, False, False, 8, 8, 8, 1.0, beta, **kw)
