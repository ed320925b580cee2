"""The allocation-free backward (zcsd_dcsd_backward_noalloc) against the
arena-backed entry point (zcsd_dcsd_backward) through the C ABI.

Two calls in a row share the device's fixed scratch array: the first takes
several passes over its batch (n = 1024 leaves room for four problems per
pass), the second is smaller (one pass at n = 256) and must not see anything
the first left behind.  Both are checked element by element against the
arena-backed entry point on the same inputs (the same kernels run on both
paths, so the results agree to rounding).  Sizes beyond the array's limit are
rejected on the host before anything is enqueued.
"""
import numpy as np
import pytest
import torch

from paper_1804_09002_amd import workloads as WL

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _inputs(batch, n, seed):
    """Decompositions built from known factors (uniform angles) and seeded
    Gaussian cotangents, as device tensors (batch, n, n) / (batch, n)."""
    rng = np.random.default_rng(seed)
    U1, U2, V1, th = [], [], [], []
    for _ in range(batch):
        u1, u2, v1 = (WL.haar(n, rng) for _ in range(3))
        t = WL.angles_uniform(n, rng)
        U1.append(u1); U2.append(u2); V1.append(v1); th.append(t)
    t = lambda x: torch.tensor(np.ascontiguousarray(np.stack(x)), device=DEV)
    g = torch.tensor(rng.standard_normal((batch, n)), device=DEV)
    G1 = torch.tensor(rng.standard_normal((batch, n, n)), device=DEV)
    G2 = torch.tensor(rng.standard_normal((batch, n, n)), device=DEV)
    return t(U1), t(U2), t(V1), t(th), g, G1, G2


def _agree(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    scale = np.max(np.abs(b))
    assert np.all(np.isfinite(a))
    err = np.max(np.abs(a - b))
    assert err <= 1e-13 * scale, (err, scale)


def test_noalloc_backward_matches_arena_backward_twice():
    from paper_1804_09002_amd import zcsd
    for case, (batch, n, seed) in enumerate([(6, 1024, 31), (3, 256, 32)]):
        print(f"no-alloc backward call {case}: batch={batch} n={n} seed={seed}", flush=True)
        args = _inputs(batch, n, seed)
        ref1, ref2 = zcsd.csd_backward(*args)
        got1, got2 = zcsd.csd_backward_noalloc(*args)
        torch.cuda.synchronize()
        _agree(got1, ref1)
        _agree(got2, ref2)


def test_noalloc_backward_partial_cotangents():
    """NULL cotangents (angles only, one polar only) take the same route."""
    from paper_1804_09002_amd import zcsd
    U1, U2, V1, th, g, G1, G2 = _inputs(2, 96, 33)
    for kw in ({"g_theta": g}, {"G_W1": G1}, {"G_W2": G2, "g_theta": g}):
        ref = zcsd.csd_backward(U1, U2, V1, th, **kw)
        got = zcsd.csd_backward_noalloc(U1, U2, V1, th, **kw)
        torch.cuda.synchronize()
        _agree(got[0], ref[0])
        _agree(got[1], ref[1])


def test_noalloc_backward_rejects_n_beyond_scratch():
    from paper_1804_09002_amd import zcsd
    n = 2049
    z = torch.zeros((1, n, n), dtype=torch.float64, device=DEV)
    th = torch.zeros((1, n), dtype=torch.float64, device=DEV)
    with pytest.raises(zcsd.ZcsdError) as e:
        zcsd.csd_backward_noalloc(z, z, z, th, th, None, None)
    assert e.value.status == zcsd.ZCSD_EINVAL
