"""The accuracy study of Sec. 6 on the GPU path (real analogue).

    python -m paper_1804_09002_amd.accuracy_study [--jmax 9] [--seed 11]

For each test class (1-4 and the noisy 1'-4', ``workloads.paper_test_class``)
and n = nint(30 * 2^(j/2)), j = 0..jmax, one CS decomposition runs through the
C ABI on cuda:0 and the two measures the paper tabulates are printed as a
markdown table:

* the scaled residual ||A_hat - A||_2 / d(A), with A_hat = [U1 C V1^T; U2 S V1^T]
  on the computed (economical) factors and d(A) = max_i min(sigma_i,
  |1 - sigma_i|), the distance to the nearest partial isometry (Sec. 2.1);
* the scaled orthogonality ||X^T X - I||_2 / u, u = 2^-53, for X = U1, U2, V1.

The measures are evaluated on the host in FP64 (numpy); the decomposition
itself is the library's.
"""
from __future__ import annotations

import argparse
import sys

import numpy as np

U = 2.0 ** -53


def measures(A1, A2, U1, U2, V1, theta, r):
    A = np.vstack([A1, A2])
    U1, U2, V1, theta = U1[:, :r], U2[:, :r], V1[:, :r], theta[:r]
    Ahat = np.vstack([(U1 * np.cos(theta)) @ V1.T, (U2 * np.sin(theta)) @ V1.T])
    sig = np.linalg.svd(A, compute_uv=False)
    dA = float(np.max(np.minimum(sig, np.abs(1.0 - sig))))
    res = float(np.linalg.norm(Ahat - A, 2))
    orth = [float(np.linalg.norm(X.T @ X - np.eye(r), 2)) / U for X in (U1, U2, V1)]
    return {"dA": dA, "res": res, "res_dA": res / dA, "orth_u": orth}


def run(jmax=9, seed=11, classes=None):
    import torch

    from . import workloads as WL
    from . import zcsd

    dev = torch.device("cuda:0")
    rows = []
    for cls in classes or WL.PAPER_CLASSES:
        for n in WL.paper_sizes(jmax):
            rng = np.random.default_rng(seed * 100003 + n)
            A1, A2 = WL.paper_test_class(cls, n, rng)
            U1, U2, V1, th, info = zcsd.csd(torch.tensor(A1, device=dev), torch.tensor(A2, device=dev))
            U1, U2, V1, th = (x.cpu().numpy() for x in (U1, U2, V1, th))
            m = measures(A1, A2, U1, U2, V1, th, info["rank"])
            m.update({"cls": cls, "n": n, "rank": info["rank"]})
            rows.append(m)
    return rows


def load_paper(path):
    """The Zolo-csd (Z) columns of Tables 1 and 2 (Sec. 6), keyed by (class, n)."""
    import json
    with open(path) as f:
        d = json.load(f)
    return {(r["class"], r["n"]): r for r in d["rows"]}


def table(rows, paper=None):
    """Markdown table; with `paper` (load_paper) each measure is followed by the
    paper's figures for the same class and n in parentheses: Zolo-csd's, and
    LAPACK's csd after a slash where Table 1 has them."""
    out = ["| class | n | rank | d(A) | ‖Â−A‖₂/d(A) | ‖U1ᵀU1−I‖₂/u | ‖U2ᵀU2−I‖₂/u | ‖V1ᵀV1−I‖₂/u |",
           "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for m in rows:
        o = m["orth_u"]
        p = paper.get((m["cls"], m["n"])) if paper else None

        def z(k, f):
            if not p:
                return ""
            lap = p.get("lapack")
            return f" ({p[k]:{f}} / {lap[k]:{f}})" if lap else f" ({p[k]:{f}})"
        out.append(f"| {m['cls']} | {m['n']} | {m['rank']} | {m['dA']:.1e} | {m['res_dA']:.2f}{z('res', '.2f')} | "
                   f"{o[0]:.1f}{z('U1', '.1f')} | {o[1]:.1f}{z('U2', '.1f')} | {o[2]:.1f}{z('V1', '.1f')} |")
    return "\n".join(out)


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--jmax", type=int, default=9)
    p.add_argument("--seed", type=int, default=11)
    p.add_argument("--paper", default=None,
                   help="JSON of the paper's Zolo-csd and LAPACK columns (tests/golden/paper_tables_sec6.json)"
                        " to print beside the measured values")
    a = p.parse_args(argv)
    rows = run(a.jmax, a.seed)
    print(table(rows, load_paper(a.paper) if a.paper else None), flush=True)
    worst_res = max(m["res_dA"] for m in rows)
    worst_orth = max(max(m["orth_u"]) for m in rows)
    print(f"\nworst scaled residual {worst_res:.2f}, worst scaled orthogonality {worst_orth:.1f}",
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
