"""Writes c4_tiny512_fd.json: central finite differences of the FP64 oracle's
image loss (the differentiable workload of tests/differentiable.py) for 64
seeded leaf heights and 64 seeded leaf widths, each drawn among the leaves
whose analytic oracle gradient is non-zero (above 1e-3 of the largest);
probes whose +/- eps renders change a hit cell are skipped and the next
leaf is drawn.  eps = 1e-4 m for heights and 1e-5 sigma_j for widths.
Calls only the oracle (and the seeded input generators).

    python tests/golden/make_c4_fd.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from tests import differentiable as D  # noqa: E402

COUNT = 64


def main():
    P = D.build_problem()
    s = P["s"]
    out = {"workload": "tiny heightfield, 512x512, target = oracle depth of v + N(0, 2 m) (seed 1003), "
                       "L2 over pixels where both hit", "loss": P["loss0"]}
    for which, g in (("v", P["gv"]), ("sigma", P["gs"])):
        cand = np.nonzero(np.abs(g) > 1e-3 * np.abs(g).max())[0]
        rng = np.random.default_rng(1003 + (which == "sigma"))
        rng.shuffle(cand)
        leaf, fd, eps_l, ana = [], [], [], []
        for j in cand:
            eps = 1e-4 if which == "v" else 1e-5 * float(s.leaves["sigma"][j])
            f = D.fd(P, int(j), which, eps)
            if f is None:
                continue
            leaf.append(int(j))
            fd.append(float(f))
            eps_l.append(eps)
            ana.append(float(g[j]))
            if len(leaf) == COUNT:
                break
        out[which] = {"leaf": leaf, "eps": eps_l, "fd": fd, "oracle_analytic": ana,
                      "grad_inf_norm": float(np.abs(g).max())}
        print(which, len(leaf), "leaves", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_tiny512_fd.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
