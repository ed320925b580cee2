"""Autotuner of the batched path (zcsd_dcsd_batched) for a workload.

    python -m paper_1804_09002_amd.autotune [--count 2048] [--lo 8] [--hi 256]
        [--seed 5] [--reps 3] [--out tuning.json]
    python -m paper_1804_09002_amd.autotune --tiles 1024,2048,4096
        [--prec fp64|mixed_fp32] [--cache tiles.json]

The batched path groups problems into size classes padded to a multiple of a
step and runs the groups on several worker streams (include/zcsd.h,
zcsd_set_tuning).  For a synthetic workload with the given size distribution
(n log-uniform in [lo, hi], uniform angles, as the bench's batched leg), this
times one batched call per candidate setting after two warm-up calls (mean of
`reps` calls): first the number of workers at the default steps, then the
class steps at the best number of workers, then the largest size that runs
as one-workgroup CSDs (coordinate descent).  It prints
the timings and writes the best setting with them to `--out` as JSON;
`apply(path)` sets a written file's setting on the current device's handle.
The library's defaults are this search's result for the bench workload.

`search_tiles(n, prec, cache=path)` does the same for the matrix products of
the single path: it picks, per problem size and precision, the threshold
above which products take 128 x 128 output tiles instead of 64 x 64, and keeps
its results in a JSON cache that `apply_tiles(path, n, prec)` reads.
"""
from __future__ import annotations

import argparse
import json
import time

WORKERS = (1, 2, 3, 4, 6, 8)
STEPS = ((4, 8, 32), (8, 16, 64), (8, 32, 64), (16, 16, 64), (16, 32, 64))
ONE_WG = (56, 48, 32, 64, 16, 0)


def workload(count, lo, hi, seed):
    import numpy as np
    import torch

    from . import workloads as WL
    from . import zcsd
    sizes = [int(n) for n in WL.batched_sizes(count, seed, lo, hi)]
    rng = np.random.default_rng(seed)
    A1s, A2s = [], []
    for n in sizes:
        A1, A2, _ = WL.uniform_pair(n, int(rng.integers(1 << 31)))
        A1s.append(torch.tensor(A1, device="cuda:0"))
        A2s.append(torch.tensor(A2, device="cuda:0"))
    a1, sizes, offs = zcsd.pack_ragged(A1s)
    a2, _, _ = zcsd.pack_ragged(A2s)
    return a1, a2, sizes, offs


def time_setting(data, setting, reps):
    import torch

    from . import zcsd
    zcsd.set_tuning(**setting)
    a1, a2, sizes, offs = data
    for _ in range(2):
        zcsd.csd_batched_packed(a1, a2, sizes, offs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        zcsd.csd_batched_packed(a1, a2, sizes, offs)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def search(count=2048, lo=8, hi=256, seed=5, reps=3, workers=WORKERS, steps=STEPS, one_wg=ONE_WG,
           log=print):
    from . import zcsd
    data = workload(count, lo, hi, seed)
    start = zcsd.get_tuning()
    timings = []

    def run(setting):
        t = time_setting(data, setting, reps)
        timings.append({**setting, "seconds": round(t, 5)})
        log(f"{setting}: {t * 1e3:.2f} ms")
        return t

    base_steps = dict(class_step_small=start["class_step_small"], class_step_mid=start["class_step_mid"],
                      class_step_large=start["class_step_large"],
                      one_workgroup_max_n=start["one_workgroup_max_n"])
    best_w = min(workers, key=lambda w: run(dict(batched_workers=w, **base_steps)))
    best = None
    for st in steps:
        setting = dict(batched_workers=best_w, class_step_small=st[0], class_step_mid=st[1],
                       class_step_large=st[2], one_workgroup_max_n=start["one_workgroup_max_n"])
        t = run(setting)
        if best is None or t < best[1]:
            best = (setting, t)
    # then the largest size that runs as one-workgroup CSDs
    for lim in one_wg:
        if lim == best[0]["one_workgroup_max_n"]:
            continue
        setting = {**best[0], "one_workgroup_max_n": lim}
        t = run(setting)
        if t < best[1]:
            best = (setting, t)
    zcsd.set_tuning(**start)
    return {"workload": {"count": count, "lo": lo, "hi": hi, "seed": seed},
            "best": best[0], "best_seconds": round(best[1], 5), "timings": timings}


TILE128_MIN = (128, 256, 384, 512, 768, 1024)


def search_tiles(n, prec="fp64", seed=4, reps=2, candidates=TILE128_MIN, cache=None, log=print):
    """The GEMM tiling threshold (gemm_tile128_min: products with at least that
    many 128 x 128 output tiles use them, the others 64 x 64 tiles) for single
    CSDs of size n in precision `prec` ("fp64" or "mixed_fp32"): each
    candidate is timed on a uniform-angle problem of that size (one warm-up
    call, then the mean of `reps`), and the fastest is returned.  With `cache`
    (a JSON file) a result stored under "n=<n>,prec=<prec>" is reused, and a
    new one is stored there."""
    import os
    import torch

    from . import workloads as WL
    from . import zcsd
    key = f"n={n},prec={prec}"
    data = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            data = json.load(f)
        if key in data:
            return data[key]
    A1, A2, _ = WL.uniform_pair(n, seed)
    A1 = torch.tensor(A1, device="cuda:0")
    A2 = torch.tensor(A2, device="cuda:0")
    start = zcsd.get_tuning()
    timings = []
    try:
        for t in candidates:
            zcsd.set_tuning(gemm_tile128_min=t)
            zcsd.csd(A1, A2, prec=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                zcsd.csd(A1, A2, prec=prec)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / reps
            timings.append({"gemm_tile128_min": t, "seconds": round(sec, 5)})
            log(f"n={n} {prec} gemm_tile128_min={t}: {sec * 1e3:.2f} ms")
    finally:
        zcsd.set_tuning(**start)
    best = min(timings, key=lambda r: r["seconds"])
    res = {"n": n, "prec": prec, "gemm_tile128_min": best["gemm_tile128_min"],
           "seconds": best["seconds"], "timings": timings}
    if cache:
        data[key] = res
        with open(cache, "w") as f:
            json.dump(data, f, indent=1)
    return res


def apply_tiles(cache, n, prec="fp64", device=None):
    """Set the threshold a cache written by search_tiles holds for (n, prec) on
    the device's handle (the entry of the largest cached n <= n, else the
    smallest cached n, of that precision); returns the value set, or None if
    the cache has no entry of that precision."""
    from . import zcsd
    with open(cache) as f:
        data = json.load(f)
    rows = sorted((r["n"], r["gemm_tile128_min"]) for r in data.values() if r["prec"] == prec)
    if not rows:
        return None
    below = [v for m, v in rows if m <= n]
    value = below[-1] if below else rows[0][1]
    zcsd.set_tuning(device, gemm_tile128_min=value)
    return value


def apply(path, device=None):
    """Set the best setting of a file written by this tool on the device's handle."""
    from . import zcsd
    with open(path) as f:
        zcsd.set_tuning(device, **json.load(f)["best"])


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--count", type=int, default=2048)
    p.add_argument("--lo", type=int, default=8)
    p.add_argument("--hi", type=int, default=256)
    p.add_argument("--seed", type=int, default=5)
    p.add_argument("--reps", type=int, default=3)
    p.add_argument("--out", default=None)
    p.add_argument("--tiles", default=None,
                   help="comma-separated sizes n: search the GEMM tiling threshold of single CSDs instead")
    p.add_argument("--prec", default="fp64", choices=("fp64", "mixed_fp32"))
    p.add_argument("--cache", default=None, help="JSON cache of the tiling search")
    a = p.parse_args(argv)
    if a.tiles:
        for n in (int(x) for x in a.tiles.split(",")):
            r = search_tiles(n, a.prec, cache=a.cache)
            print(json.dumps({"n": n, "prec": a.prec, "gemm_tile128_min": r["gemm_tile128_min"],
                              "seconds": r["seconds"]}))
        return
    res = search(a.count, a.lo, a.hi, a.seed, a.reps)
    print(json.dumps({"best": res["best"], "best_seconds": res["best_seconds"]}))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
