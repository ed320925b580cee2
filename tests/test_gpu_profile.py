"""The library's per-kernel event profiler (zcsd_profile_*), which bench.py's
roofline figure rests on.

A product's record counts its launches and its algorithmic flops (2mnk of
the tiles it computes) and sums the event-timed durations; the matrix
products attach their events to the dispatch itself.  Checked: counts and
flops of known products, durations positive and consistent with the wall
clock, the name filter, and that profiling changes no result.
"""
import time

import pytest
import torch

pytestmark = pytest.mark.gpu


def test_profile_counts_flops_and_times_products():
    from paper_1804_09002_amd import zcsd
    g = torch.Generator(device="cpu").manual_seed(3)
    A = torch.randn(8, 1024, 1024, dtype=torch.float64, generator=g).to("cuda:0")
    B = torch.randn(8, 1024, 1024, dtype=torch.float64, generator=g).to("cuda:0")
    ref = zcsd.dgemm(A, B)
    torch.cuda.synchronize()
    with zcsd.profile() as p:
        t0 = time.perf_counter()
        for _ in range(3):
            C = zcsd.dgemm(A, B)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3
    st = p.stats()
    # 8 x 1024^2 outputs: 512 tiles of 128 x 128, at the default threshold
    # of 512 the 128 x 128 tiling
    rec = st["dgemm_128x128_NN"]
    assert rec["launches"] == 3
    assert rec["flops"] == pytest.approx(3 * 2.0 * 8 * 1024 ** 3, rel=1e-12)
    assert 0.0 < rec["ms"] <= wall_ms
    assert torch.equal(C, ref)


def test_profile_filter_records_only_the_named_kernel():
    from paper_1804_09002_amd import zcsd
    g = torch.Generator(device="cpu").manual_seed(4)
    A = torch.randn(2048, 2048, dtype=torch.float64, generator=g).to("cuda:0")
    saved = zcsd.get_tuning()
    try:
        zcsd.set_tuning(gemm_tile128_min=1)
        with zcsd.profile(only="dgemm_128x128_NN") as p:
            zcsd.dgemm(A, A)
            zcsd.dgemm(A, A, transA=True)
            torch.cuda.synchronize()
        st = p.stats()
    finally:
        zcsd.set_tuning(**saved)
    assert set(st) == {"dgemm_128x128_NN"}
    assert st["dgemm_128x128_NN"]["launches"] == 1
    assert st["dgemm_128x128_NN"]["flops"] == pytest.approx(2.0 * 2048 ** 3, rel=1e-12)
    assert st["dgemm_128x128_NN"]["ms"] > 0.0
