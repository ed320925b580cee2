"""The Sec. 6 test-class generators (CPU): shapes, ranks and structure."""
import numpy as np
import pytest

from paper_1804_09002_amd import workloads as WL


def test_paper_sizes():
    assert WL.paper_sizes() == [30, 42, 60, 85, 120, 170, 240, 339, 480, 679]


@pytest.mark.parametrize("cls", list(WL.PAPER_CLASSES))
def test_paper_classes(cls):
    n = 40
    A1, A2 = WL.paper_test_class(cls, n, np.random.default_rng(3))
    assert A1.shape == (n, n) and A2.shape == (n, n)
    A = np.vstack([A1, A2])
    sig = np.linalg.svd(A, compute_uv=False)
    r = n if cls[0] in "12" else int(np.rint(3 * n / 4))
    # a partial isometry: r singular values at 1, the rest at 0 (up to the noise)
    tol = 1e-13 if not cls.endswith("'") else 1e-8
    assert np.all(np.abs(sig[:r] - 1.0) <= tol)
    assert np.all(sig[r:] <= tol)
    if cls.endswith("'"):
        assert np.max(np.minimum(sig, np.abs(1 - sig))) > 1e-11  # the noise is there


def test_unknown_class_rejected():
    with pytest.raises(ValueError):
        WL.paper_test_class("5", 10, np.random.default_rng(0))
