"""Benchmark: one FP64 CS decomposition (Zolo-csd) of a 2n x n matrix, n = 4096.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 4096] [--no-cpu]

Workload (synthetic, seeded): A1 = U1 diag(cos t) V1^T, A2 = U2 diag(sin t) V1^T
with Haar U1, U2, V1 and 4096 angles uniform in [0, pi/2] (numpy PCG64 seed 4).
A step is one full call of zcsd_dcsd (rank test, two Zolo-pd, B, Zolo-eig,
assembly, sorting) on device-resident inputs.  Prints one JSON line with the
throughput (CSD/s), the roofline of the dominant kernel measured with HIP
events inside the timed steps, the accuracy of the result, and the CPU
oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "n=4096 CSD time & % MFMA peak; mixed/batched vs plain FP64 at equal error"
PEAKS = {"f64_mfma_tflops": 78.6, "f64_vector_tflops": 78.6, "hbm_gbs": 8000.0}

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this
# workload, scaled by the same counters on a copy of known size (the summaries
# with their commands are in profiles/).  A figure is reported only while the
# kernel's source file still has the hash it had when the counters were taken.
TRAFFIC = {
    "tsqr_tree": {"bytes": 1344081.2, "src": "paper_1804_09002_amd/csrc/qr_tsqr.hip",
                 "sha": "d3e3b36b44660cac", "summary": "profiles/tsqr_tree_kernel_csd4096_traffic.md"},
    "dgemm_128x128_NN": {"bytes": 584038177.2, "src": "paper_1804_09002_amd/csrc/gemm.hip",
                        "sha": "5a1f23a603ba3a83", "summary": "profiles/dgemm_kernel_128x128_NN_csd4096_traffic.md"},
    "dgemm_64x64_TN": {"bytes": 81413632.1, "src": "paper_1804_09002_amd/csrc/gemm.hip",
                      "sha": "5a1f23a603ba3a83", "summary": "profiles/dgemm_kernel_64x64_TN_csd4096_traffic.md"},
}
# kernels whose time is set by a dependent chain of small steps in one
# workgroup per problem, not by the matrix cores: their roofline is the FP64
# vector rate (256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s)
ALU_KERNELS = ("tsqr_local", "tsqr_tree", "tsqr_expand", "qr_panel")
# The mixed-precision leg: the mixed mode (FP32 products) and the FP64 path
# run with the same options (the Zolotarev target 1 - l_2 <= tol included) and
# are compared at the mixed mode's stated tolerance for every output measure.
MIXED_TOL = 2.0 ** -53
MIXED_TAU = 1e-5


def _traffic(kernel):
    import hashlib
    t = TRAFFIC.get(kernel)
    if not t:
        return None
    with open(os.path.join(ROOT, t["src"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != t["sha"]:
            return None
    return t["bytes"]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=4096)
    p.add_argument("--seed", type=int, default=4)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-n", type=int, default=2048)
    p.add_argument("--cpu-reps", type=int, default=2)
    p.add_argument("--no-extra", action="store_true",
                   help="skip the batched and forward+backward side measurements")
    p.add_argument("--batched-count", type=int, default=2048)
    p.add_argument("--single-sample", type=int, default=256,
                   help="problems of the batched workload timed one by one on the single path")
    p.add_argument("--leg", choices=("small_graph",), default=None,
                   help="run only this side measurement and print its JSON (for profiling)")
    return p.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _norm2_sym(E, iters=60):
    import torch
    x = torch.ones(E.shape[0], dtype=torch.float64, device=E.device) / E.shape[0] ** 0.5
    lam = 0.0
    for _ in range(iters):
        y = E @ x
        lam = float(torch.linalg.vector_norm(y))
        if lam == 0.0:
            break
        x = y / lam
    return lam


def accuracy(A1, A2, U1, U2, V1, th, theta_true):
    """The paper's measures (Sec. 6) on the device: ||A_hat - A||_2 / ||A||_2 and
    ||X^T X - I||_2 (2-norms by power iteration on symmetric products), plus Frobenius."""
    import torch
    n = A1.shape[0]
    c, s = torch.cos(th), torch.sin(th)
    R1 = (U1 * c) @ V1.T - A1
    R2 = (U2 * s) @ V1.T - A2
    res2 = (_norm2_sym(R1.T @ R1 + R2.T @ R2) / _norm2_sym(A1.T @ A1 + A2.T @ A2)) ** 0.5
    resF = float(torch.sqrt((R1 * R1).sum() + (R2 * R2).sum()) /
                 torch.sqrt((A1 * A1).sum() + (A2 * A2).sum()))
    I = torch.eye(n, dtype=torch.float64, device=A1.device)
    orth2, orthF = {}, {}
    for k, X in (("U1", U1), ("U2", U2), ("V1", V1)):
        E = X.T @ X - I
        orth2[k] = _norm2_sym(E)
        orthF[k] = float(torch.linalg.matrix_norm(E))
    dth = float((th - theta_true).abs().max())
    return {"backward_rel_2": res2, "backward_rel_fro": resF, "orth_2": orth2, "orth_fro": orthF,
            "max_abs_theta_err": dth}


def batched_leg(count, sample, seed=5):
    """2048 CSDs with n log-uniform in [8, 256] (uniform angles): one batched call
    vs the single path one problem at a time (timed on a sample, scaled)."""
    import numpy as np
    import torch
    from paper_1804_09002_amd import workloads as WL
    from paper_1804_09002_amd import zcsd
    sizes = [int(n) for n in WL.batched_sizes(count, seed)]
    rng = np.random.default_rng(seed)
    A1s, A2s = [], []
    for n in sizes:
        A1, A2, _ = WL.uniform_pair(n, int(rng.integers(1 << 31)))
        A1s.append(torch.tensor(A1, device="cuda:0"))
        A2s.append(torch.tensor(A2, device="cuda:0"))
    a1, sizes, offs = zcsd.pack_ragged(A1s)
    a2, _, _ = zcsd.pack_ragged(A2s)
    # warm-up: workspaces of the handle and of its worker streams, code objects
    # (measured on this workload: 0.163, 0.128, then 0.112 s per call)
    for _ in range(2):
        zcsd.csd_batched_packed(a1, a2, sizes, offs)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        U1, U2, V1, th, ranks, info = zcsd.csd_batched_packed(a1, a2, sizes, offs)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / reps
    idx = np.random.default_rng(seed + 1).choice(count, size=min(sample, count), replace=False)
    for k in idx[:4]:  # warm-up of the single path on a few sizes
        zcsd.csd(A1s[k], A2s[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in idx:
        zcsd.csd(A1s[k], A2s[k])
    torch.cuda.synchronize()
    t_s = (time.perf_counter() - t0) * count / len(idx)
    # accuracy of the batched outputs, Frobenius, over every problem
    worst_res = worst_orth = 0.0
    t_off = 0
    for k, n in enumerate(sizes):
        o = offs[k]
        u1 = U1[o:o + n * n].view(n, n).t()
        u2 = U2[o:o + n * n].view(n, n).t()
        v1 = V1[o:o + n * n].view(n, n).t()
        t = th[t_off:t_off + n]
        t_off += n
        R = torch.cat([(u1 * torch.cos(t)) @ v1.T - A1s[k], (u2 * torch.sin(t)) @ v1.T - A2s[k]])
        worst_res = max(worst_res, float(torch.linalg.norm(R) / torch.linalg.norm(torch.cat([A1s[k], A2s[k]]))))
        I = torch.eye(n, dtype=torch.float64, device="cuda:0")
        worst_orth = max(worst_orth, max(float(torch.linalg.norm(X.T @ X - I)) for X in (u1, u2, v1)))
    sum_n3 = float(sum(n ** 3 for n in sizes))
    return {"workload": f"csd_fp64_batched_{count}_n8to256_loguniform", "problems": count,
            "sum_n3": sum_n3, "batched_s": round(t_b, 4), "batched_csd_per_s": round(count / t_b, 2),
            "single_path_s_est": round(t_s, 3), "single_sample": int(len(idx)),
            "speedup_vs_single": round(t_s / t_b, 2),
            "model_tflops_batched": round(198.0 * sum_n3 / t_b / 1e12, 3),
            "worst_backward_rel_fro": worst_res, "worst_orth_fro": worst_orth}


def small_batched_leg(count=4096, lo=4, hi=64, seed=8):
    """4096 CSDs with n log-uniform in [4, 64] (uniform angles): one batched call
    with the handle's default one-workgroup limit (full-rank n <= 56 as whole
    CSDs in persistent launches, the rest through the size classes) against
    the same call with every problem in the classes (one_workgroup_max_n = 0),
    both steady state (two warm-up calls, mean of three)."""
    import numpy as np
    import torch
    from paper_1804_09002_amd import workloads as WL
    from paper_1804_09002_amd import zcsd
    sizes = [int(n) for n in WL.batched_sizes(count, seed, lo, hi)]
    rng = np.random.default_rng(seed)
    A1s, A2s = [], []
    for n in sizes:
        A1, A2, _ = WL.uniform_pair(n, int(rng.integers(1 << 31)))
        A1s.append(torch.tensor(A1, device="cuda:0"))
        A2s.append(torch.tensor(A2, device="cuda:0"))
    a1, sizes, offs = zcsd.pack_ragged(A1s)
    a2, _, _ = zcsd.pack_ragged(A2s)
    saved = zcsd.get_tuning()
    limit = saved["one_workgroup_max_n"]
    times = {}
    try:
        for lim in (0, limit):
            zcsd.set_tuning(one_workgroup_max_n=lim)
            for _ in range(2):
                zcsd.csd_batched_packed(a1, a2, sizes, offs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                U1, U2, V1, th, ranks, info = zcsd.csd_batched_packed(a1, a2, sizes, offs)
            torch.cuda.synchronize()
            times[lim] = (time.perf_counter() - t0) / 3
    finally:
        zcsd.set_tuning(**saved)
    worst_res = worst_orth = 0.0
    t_off = 0
    for k, n in enumerate(sizes):  # outputs of the last (one-workgroup) call
        o = offs[k]
        u1, u2, v1 = (X[o:o + n * n].view(n, n).t() for X in (U1, U2, V1))
        t = th[t_off:t_off + n]
        t_off += n
        R = torch.cat([(u1 * torch.cos(t)) @ v1.T - A1s[k], (u2 * torch.sin(t)) @ v1.T - A2s[k]])
        worst_res = max(worst_res, float(torch.linalg.norm(R) / torch.linalg.norm(torch.cat([A1s[k], A2s[k]]))))
        I = torch.eye(n, dtype=torch.float64, device="cuda:0")
        worst_orth = max(worst_orth, max(float(torch.linalg.norm(X.T @ X - I)) for X in (u1, u2, v1)))
    sum_n3 = float(sum(n ** 3 for n in sizes))
    return {"workload": f"csd_fp64_batched_{count}_n{lo}to{hi}_loguniform", "problems": count,
            "sum_n3": sum_n3, "one_workgroup_max_n": limit, "one_workgroup_s": round(times[limit], 5),
            "size_classes_s": round(times[0], 5),
            "speedup_vs_size_classes": round(times[0] / times[limit], 3),
            "one_workgroup_csd_per_s": round(count / times[limit], 1),
            "model_tflops_one_workgroup": round(198.0 * sum_n3 / times[limit] / 1e12, 4),
            "worst_backward_rel_fro": worst_res, "worst_orth_fro": worst_orth}


def small_graph_leg(count=4096, lo=4, hi=64, seed=8):
    """`count` CSDs with n log-uniform in [lo, hi] (uniform angles) through the
    device-routed entry point (zcsd_dcsd_batched_small: routing, persistent
    launches and table on the device), eager and as a captured HIP graph
    replay, against the host-routed batched call with every problem in the
    one-workgroup launches (one_workgroup_max_n = 64); outputs of the three
    compared bit for bit.  Each timing: two warm-up calls, mean of five."""
    import numpy as np
    import torch
    from paper_1804_09002_amd import workloads as WL
    from paper_1804_09002_amd import zcsd
    sizes = [int(n) for n in WL.batched_sizes(count, seed, lo, hi)]
    rng = np.random.default_rng(seed)
    A1s, A2s = [], []
    for n in sizes:
        A1, A2, _ = WL.uniform_pair(n, int(rng.integers(1 << 31)))
        A1s.append(torch.tensor(A1, device="cuda:0"))
        A2s.append(torch.tensor(A2, device="cuda:0"))
    a1, sizes, offs = zcsd.pack_ragged(A1s)
    a2, _, _ = zcsd.pack_ragged(A2s)
    dev = a1.device
    n_d = torch.tensor(sizes, dtype=torch.int32, device=dev)
    off_d = torch.tensor(offs, dtype=torch.int64, device=dev)
    toff_d = torch.tensor(np.concatenate([[0], np.cumsum(sizes)[:-1]]), dtype=torch.int64, device=dev)
    U1, U2, V1 = (torch.empty_like(a1) for _ in range(3))
    th = torch.empty(sum(sizes), dtype=torch.float64, device=dev)
    status = torch.empty(count, dtype=torch.int32, device=dev)
    ws = zcsd.small_batch_workspace(count)

    def call():
        zcsd.csd_batched_small(a1, a2, n_d, off_d, toff_d, U1, U2, V1, th, status, ws)

    def timed(fn, reps=5):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    saved = zcsd.get_tuning()
    try:
        zcsd.set_tuning(one_workgroup_max_n=64)
        t_host = timed(lambda: zcsd.csd_batched_packed(a1, a2, sizes, offs))
        ref = zcsd.csd_batched_packed(a1, a2, sizes, offs)
    finally:
        zcsd.set_tuning(**saved)
    t_eager = timed(call)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        call()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    torch.cuda.synchronize()
    eager_out = [X.clone() for X in (U1, U2, V1, th)]
    for X in (U1, U2, V1, th):
        X.zero_()
    t_graph = timed(g.replay)
    same_graph = all(torch.equal(x, y) for x, y in zip(eager_out, (U1, U2, V1, th)))
    same_host = all(torch.equal(x, y) for x, y in zip(ref[:4], (U1, U2, V1, th)))
    sum_n3 = float(sum(n ** 3 for n in sizes))
    return {"workload": f"csd_fp64_batched_{count}_n{lo}to{hi}_loguniform", "problems": count,
            "graph_replay_ms": round(t_graph * 1e3, 3), "device_routed_eager_ms": round(t_eager * 1e3, 3),
            "host_routed_one_workgroup_ms": round(t_host * 1e3, 3),
            "graph_csd_per_s": round(count / t_graph, 1),
            "model_tflops_graph": round(198.0 * sum_n3 / t_graph / 1e12, 4),
            "unwritten": int(((status & 255) != 0).sum()),
            "graph_equals_eager": same_graph, "equals_host_routed": same_host}


def backward_leg(count=64, n=512, seed=6):
    """Forward (one batched call) + hand-written backward of 64 CSDs at n = 512
    (uniform angles)."""
    import numpy as np
    import torch
    from paper_1804_09002_amd import workloads as WL
    from paper_1804_09002_amd import zcsd
    rng = np.random.default_rng(seed)
    A1s, A2s = [], []
    for _ in range(count):
        A1, A2, _ = WL.uniform_pair(n, int(rng.integers(1 << 31)))
        A1s.append(torch.tensor(A1, device="cuda:0"))
        A2s.append(torch.tensor(A2, device="cuda:0"))
    g = torch.tensor(rng.standard_normal((count, n)), device="cuda:0")
    G1 = torch.tensor(rng.standard_normal((count, n, n)), device="cuda:0")
    G2 = torch.tensor(rng.standard_normal((count, n, n)), device="cuda:0")

    a1, sizes, offs = zcsd.pack_ragged(A1s)
    a2, _, _ = zcsd.pack_ragged(A2s)

    def fwd():  # one batched call; the packed outputs are (count, n, n) column-major blocks
        U1, U2, V1, th, ranks, info = zcsd.csd_batched_packed(a1, a2, sizes, offs)
        cm = lambda X: X.view(count, n, n).transpose(1, 2)
        return cm(U1), cm(U2), cm(V1), th.view(count, n)

    U1, U2, V1, th = fwd()
    zcsd.csd_backward(U1, U2, V1, th, g, G1, G2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U1, U2, V1, th = fwd()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gA1, gA2 = zcsd.csd_backward(U1, U2, V1, th, g, G1, G2)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return {"workload": f"csd_fp64_fwd_bwd_{count}x_n{n}", "forward_s": round(t1 - t0, 4),
            "backward_s": round(t2 - t1, 4), "fwd_bwd_per_s": round(count / (t2 - t0), 2),
            "backward_tflops_16n3": round(16.0 * n ** 3 * count / (t2 - t1) / 1e12, 3)}


def complex_leg(n=2048, seed=7, reps=2):
    """The complex CSD (zcsd_zcsd) at n = 2048, uniform angles and Haar unitary
    factors: its real embedding has the size of the bench's real input."""
    import numpy as np
    import torch
    from paper_1804_09002_amd import workloads as WL
    from paper_1804_09002_amd import zcsd
    A1, A2, meta = WL.complex_pair(n, seed)
    a1 = torch.tensor(A1, dtype=torch.complex128, device="cuda:0")
    a2 = torch.tensor(A2, dtype=torch.complex128, device="cuda:0")
    zcsd.csd_complex(a1, a2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        U1, U2, V1, th, info = zcsd.csd_complex(a1, a2)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    truth = torch.tensor(np.sort(meta["theta"]), device="cuda:0")
    c = torch.cos(th).to(torch.complex128)
    s = torch.sin(th).to(torch.complex128)
    Vh = V1.conj().T.contiguous()
    R = torch.cat([(U1 * c) @ Vh - a1, (U2 * s) @ Vh - a2])
    I = torch.eye(n, dtype=torch.complex128, device="cuda:0")
    fro = lambda X: float(torch.linalg.vector_norm(X))
    return {"workload": f"csd_complex_fp64_n{n}_uniform_angles", "real_embedding_n": 2 * n,
            "ms_per_csd": round(ms, 3), "rank": info["rank"],
            "accuracy": {"max_abs_theta_err": float((th - truth).abs().max()),
                         "backward_rel_fro": fro(R) / fro(torch.cat([a1, a2])),
                         "orth_fro": {k: fro(X.conj().T.contiguous() @ X - I)
                                      for k, X in (("U1", U1), ("U2", U2), ("V1", V1))}}}


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or the platform string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(n, reps, seed):
    """The oracle (numpy/LAPACK FP64, test infrastructure) on a bounded sample."""
    import numpy as np
    from oracle import csd as O
    from paper_1804_09002_amd import workloads as WL
    A1, A2, _ = WL.uniform_pair(n, seed)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    for _ in range(reps):
        O.csd(A1, A2)
    dt = (time.perf_counter() - t0) / reps
    return dt, threads


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the path runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.leg == "small_graph":
        print(json.dumps([small_graph_leg(), small_graph_leg(256, 4, 16, seed=9)]), flush=True)
        return
    import numpy as np
    import torch
    from paper_1804_09002_amd import workloads as WL
    from paper_1804_09002_amd import zcsd

    n = args.n
    dev = torch.device("cuda:0")
    log(f"generating inputs n={n} seed={args.seed}")
    A1n, A2n, meta = WL.uniform_pair(n, args.seed)
    A1 = torch.tensor(A1n, device=dev)
    A2 = torch.tensor(A2n, device=dev)
    theta_true = torch.tensor(np.sort(meta["theta"]), device=dev)
    del A1n, A2n

    # warmup (first call also finds the dominant kernel by event time)
    dominant = None
    for w in range(args.warmup):
        log(f"warmup {w + 1}/{args.warmup}")
        if w == 0:
            with zcsd.profile() as p:
                out = zcsd.csd(A1, A2)
            st = p.stats()
            dominant = max(st, key=lambda k: st[k]["ms"]) if st else None
            kern_table = {k: {"ms": round(v["ms"], 3), "launches": v["launches"],
                              "tflops": (v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 else None}
                          for k, v in sorted(st.items(), key=lambda kv: -kv[1]["ms"])[:8]}
        else:
            out = zcsd.csd(A1, A2)
    torch.cuda.synchronize()

    log(f"timing {args.steps} steps (dominant kernel {dominant})")
    torch.cuda.synchronize()
    with zcsd.profile(only=dominant) as p:
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = zcsd.csd(A1, A2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    dstat = p.stats().get(dominant) if dominant else None
    ms_step = (t1 - t0) * 1e3 / args.steps
    U1, U2, V1, th, info = out
    acc = accuracy(A1, A2, U1, U2, V1, th, theta_true)

    roof = None
    if dstat and dstat["ms"] > 0:
        per_launch_flops = dstat["flops"] / dstat["launches"]
        avg_s = dstat["ms"] * 1e-3 / dstat["launches"]
        ach = per_launch_flops / avg_s / 1e12
        alu = dominant in ALU_KERNELS
        peak = PEAKS["f64_vector_tflops"] if alu else PEAKS["f64_mfma_tflops"]
        roof = {"kernel": dominant, "bound": "alu" if alu else "mfma", "achieved": round(ach, 4),
                "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 5),
                "traffic": _traffic(dominant),
                "launches_per_step": dstat["launches"] / args.steps,
                "avg_launch_us": round(avg_s * 1e6, 3),
                "algorithmic_flops_per_launch": per_launch_flops,
                "algorithmic_bytes_per_launch": dstat["bytes"] / dstat["launches"]}

    cpu = None
    if not args.no_cpu:
        log(f"cpu oracle sample: {args.cpu_reps} x n={args.cpu_n}")
        dt, threads = cpu_baseline(args.cpu_n, args.cpu_reps, args.seed)
        scale = (args.cpu_n / n) ** 3
        cpu = {"value": round(scale / dt, 6), "unit": "CSD/s", "cores": threads, "kind": "oracle",
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
               "sample": f"{args.cpu_reps} oracle CSDs at n={args.cpu_n} (same construction), "
                         f"{dt:.2f} s each, scaled by (n_sample/n)^3 to n={n}"}

    extra = None
    if not args.no_extra:
        log(f"mixed-precision leg: n={n}, Zolotarev target {MIXED_TOL:g} for both paths")
        legs = {}
        for prec in ("mixed_fp32", "fp64"):
            zcsd.csd(A1, A2, prec=prec, tol=MIXED_TOL)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                mo = zcsd.csd(A1, A2, prec=prec, tol=MIXED_TOL)
            torch.cuda.synchronize()
            ms_leg = (time.perf_counter() - t0) * 1e3 / args.steps
            mi = mo[4]
            legs[prec] = {"ms_per_csd": round(ms_leg, 3),
                          "accuracy": accuracy(A1, A2, mo[0], mo[1], mo[2], mo[3], theta_true),
                          "r": mi["r_used"][0], "eig_max_r": mi["eig_max_r"],
                          "lowp_products": mi["lowp_products"],
                          "phases_ms": {"polar": mi["time_ms"][0], "B": mi["time_ms"][1],
                                        "eig": mi["time_ms"][2], "assembly": mi["time_ms"][3]}}
            del mo
        mixed = {"workload": f"csd_mixed_fp32_n{n}_uniform_angles", "zolotarev_tol": MIXED_TOL,
                 "stated_tolerance": MIXED_TAU, "fp64_fallback": False,
                 "ms_per_csd": legs["mixed_fp32"]["ms_per_csd"],
                 "speedup_vs_fp64_same_tol": round(legs["fp64"]["ms_per_csd"] / legs["mixed_fp32"]["ms_per_csd"], 3),
                 "speedup_vs_fp64_full": round(ms_step / legs["mixed_fp32"]["ms_per_csd"], 3),
                 "mixed": legs["mixed_fp32"], "fp64_same_tol": legs["fp64"]}
        log(f"batched leg: {args.batched_count} problems")
        extra = {"mixed": mixed, "batched": batched_leg(args.batched_count, args.single_sample)}
        log("small batched leg: 4096 problems, n in [4, 64]")
        extra["batched_small"] = small_batched_leg()
        log("small batched leg, device-routed and as a captured graph")
        extra["batched_small_graph"] = [small_graph_leg(), small_graph_leg(256, 4, 16, seed=9)]
        log("forward+backward leg: 64 x n=512")
        extra["backward"] = backward_leg()
        log("complex leg: n=2048")
        extra["complex"] = complex_leg()

    flops_model = 198.0 * n ** 3  # 67(m1+m2)n^2 + 64n^3 with m1 = m2 = n (Remark (v))
    rec = {
        "metric": METRIC,
        "value": round(1000.0 / ms_step, 6),
        "unit": "CSD/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"csd_fp64_n{n}_uniform_angles", "n": n, "seed": args.seed,
                   "angles": "uniform[0,pi/2]", "factors": "Haar U1,U2,V1"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "model_flops_rate_tflops": round(flops_model / (ms_step * 1e-3) / 1e12, 3),
        "model_frac_f64_peak": round(flops_model / (ms_step * 1e-3) / 1e12 / PEAKS["f64_mfma_tflops"], 4),
        "accuracy": acc,
        "phases_ms": {"polar": info["time_ms"][0], "B": info["time_ms"][1],
                      "eig": info["time_ms"][2], "assembly": info["time_ms"][3]},
        "zolo": {"r": info["r_used"][0], "ell": info["ell"][0], "eig_levels": info["eig_levels"],
                 "eig_splits": info["eig_splits"], "eig_max_r": info["eig_max_r"],
                 "eig_offblock": info["eig_offblock"]},
        "kernels_warmup": kern_table if args.warmup > 0 else None,
        "extra": extra,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
