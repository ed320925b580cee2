"""Batched-path tuning (zcsd_set_tuning) and its autotuner.

The tuning changes how problems are grouped (class padding) and how many
worker streams run the groups, never the arithmetic of a problem: results
under another setting agree with the default's to rounding and with the
oracle.  The autotuner's search returns one of its candidates and leaves the
handle's setting as it found it.
"""
import numpy as np
import pytest
import torch

from oracle import csd as O
from paper_1804_09002_amd import workloads as WL

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
DEFAULT = {"batched_workers": 4, "class_step_small": 8, "class_step_mid": 16, "class_step_large": 64,
           "one_workgroup_max_n": 56, "gemm_tile128_min": 512}


def test_tuning_roundtrip_and_validation():
    from paper_1804_09002_amd import zcsd
    assert zcsd.get_tuning() == DEFAULT
    zcsd.set_tuning(batched_workers=2, class_step_mid=32)
    assert zcsd.get_tuning() == {**DEFAULT, "batched_workers": 2, "class_step_mid": 32}
    for bad in ({"batched_workers": 0}, {"batched_workers": 17}, {"class_step_small": 0},
                {"class_step_large": 257}, {"one_workgroup_max_n": 65}, {"gemm_tile128_min": 0}):
        with pytest.raises(zcsd.ZcsdError):
            zcsd.set_tuning(**bad)
    st = zcsd.lib().zcsd_set_tuning(zcsd.handle(), 99, 1)
    assert st == zcsd.ZCSD_EINVAL
    zcsd.set_tuning(**DEFAULT)
    assert zcsd.get_tuning() == DEFAULT


def test_batched_results_do_not_depend_on_tuning():
    from paper_1804_09002_amd import zcsd
    sizes = [int(n) for n in WL.batched_sizes(40, 17, 8, 120)]
    rng = np.random.default_rng(17)
    A1s, A2s, np1, np2 = [], [], [], []
    for n in sizes:
        A1, A2, _ = WL.uniform_pair(n, int(rng.integers(1 << 31)))
        np1.append(A1)
        np2.append(A2)
        A1s.append(torch.tensor(A1, device="cuda:0"))
        A2s.append(torch.tensor(A2, device="cuda:0"))
    a1, szs, offs = zcsd.pack_ragged(A1s)
    a2, _, _ = zcsd.pack_ragged(A2s)
    ref = zcsd.csd_batched_packed(a1, a2, szs, offs)[3].cpu().numpy()
    try:
        zcsd.set_tuning(batched_workers=1, class_step_small=4, class_step_mid=32, class_step_large=64,
                        one_workgroup_max_n=24)
        got = zcsd.csd_batched_packed(a1, a2, szs, offs)[3].cpu().numpy()
    finally:
        zcsd.set_tuning(**DEFAULT)
    assert np.max(np.abs(got - ref)) <= 10 * 120 * U
    t_off = 0
    for k, n in enumerate(sizes):
        if k % 8 == 0:
            o = O.csd(np1[k], np2[k])
            assert np.max(np.abs(got[t_off:t_off + n] - o["theta"])) <= 10 * n * U
        t_off += n


def test_autotune_search_small_workload(tmp_path):
    from paper_1804_09002_amd import autotune, zcsd
    res = autotune.search(count=48, lo=8, hi=48, seed=3, reps=1, workers=(1, 2),
                          steps=((8, 16, 64), (16, 16, 64)), one_wg=(56, 64, 0), log=lambda m: None)
    # the candidate equal to the handle's current limit (56) is not timed again
    assert len(res["timings"]) == 6
    assert res["best"]["one_workgroup_max_n"] in (56, 64, 0)
    assert res["best"]["batched_workers"] in (1, 2)
    assert (res["best"]["class_step_small"], res["best"]["class_step_mid"]) in ((8, 16), (16, 16))
    assert zcsd.get_tuning() == DEFAULT
    path = tmp_path / "tuning.json"
    import json
    path.write_text(json.dumps(res))
    try:
        autotune.apply(str(path))
        assert zcsd.get_tuning()["batched_workers"] == res["best"]["batched_workers"]
    finally:
        zcsd.set_tuning(**DEFAULT)


def test_gemm_tiling_threshold_changes_tiles_not_results():
    """The tiling threshold picks 128 x 128 or 64 x 64 output tiles; a product
    (4 x 300 x 260 x 200: 36 tiles of 128) and a CSD (n = 300) give the same
    results either way, to rounding, and match a float64 torch product."""
    from paper_1804_09002_amd import zcsd
    g = torch.Generator(device="cpu").manual_seed(5)
    A = torch.randn(4, 300, 200, dtype=torch.float64, generator=g).to("cuda:0")
    B = torch.randn(4, 200, 260, dtype=torch.float64, generator=g).to("cuda:0")
    ref = torch.matmul(A, B)
    out = {}
    try:
        for t in (1, 1 << 24):
            zcsd.set_tuning(gemm_tile128_min=t)
            out[t] = zcsd.dgemm(A, B)
        assert float((out[1] - ref).abs().max()) <= 1e-12
        assert float((out[1 << 24] - ref).abs().max()) <= 1e-12
        A1, A2, meta = WL.uniform_pair(300, 31)
        th = {}
        for t in (1, 1 << 24):
            zcsd.set_tuning(gemm_tile128_min=t)
            th[t] = zcsd.csd(torch.tensor(A1, device="cuda:0"), torch.tensor(A2, device="cuda:0"))[3]
        assert float((th[1] - th[1 << 24]).abs().max()) <= 10 * 300 * U
        assert np.max(np.abs(th[1].cpu().numpy() - np.sort(meta["theta"]))) <= 10 * 300 * U
    finally:
        zcsd.set_tuning(**DEFAULT)


def test_tile_search_uses_and_fills_its_cache(tmp_path):
    from paper_1804_09002_amd import autotune, zcsd
    cache = str(tmp_path / "tiles.json")
    res = autotune.search_tiles(160, "fp64", reps=1, candidates=(1, 768), cache=cache,
                                log=lambda m: None)
    assert res["gemm_tile128_min"] in (1, 768) and len(res["timings"]) == 2
    assert zcsd.get_tuning() == DEFAULT
    import json
    with open(cache) as f:
        assert json.load(f)["n=160,prec=fp64"]["gemm_tile128_min"] == res["gemm_tile128_min"]
    # a cached entry is returned as stored, without timing again
    again = autotune.search_tiles(160, "fp64", reps=1, candidates=(7,), cache=cache, log=lambda m: None)
    assert again == res
    try:
        assert autotune.apply_tiles(cache, 200) == res["gemm_tile128_min"]
        assert zcsd.get_tuning()["gemm_tile128_min"] == res["gemm_tile128_min"]
        assert autotune.apply_tiles(cache, 200, prec="mixed_fp32") is None
    finally:
        zcsd.set_tuning(**DEFAULT)
