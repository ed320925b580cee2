"""Host-side checks of the complex CSD binding (no GPU needed): argument
validation happens before the library is called."""
import numpy as np
import pytest
import torch

from paper_1804_09002_amd import workloads as WL


def test_rejects_non_device_or_real_tensors():
    from paper_1804_09002_amd import zcsd
    a = torch.zeros((4, 4), dtype=torch.complex128)
    with pytest.raises(TypeError):
        zcsd.csd_complex(a, a)            # host tensors
    with pytest.raises(TypeError):
        zcsd.csd_complex(a.real, a.real)  # real tensors


def test_complex_workloads_are_partial_isometries():
    for kind, k, mult in (("uniform", 0, 1), ("clustered", 3, 1), ("repeated", 0, 4), ("haar", 0, 1)):
        A1, A2, meta = WL.complex_pair(16, 3, kind=kind, rank_deficient=k, mult=mult)
        A = np.vstack([A1, A2])
        assert A.dtype == np.complex128 and np.abs(A.imag).max() > 0.05
        s = np.linalg.svd(A, compute_uv=False)
        assert np.sum(s > 0.5) == 16 - k
        assert np.max(np.minimum(np.abs(s - 1), s)) <= 1e-14
        if kind == "repeated":
            assert len(np.unique(np.round(meta["theta"], 14))) == 4
