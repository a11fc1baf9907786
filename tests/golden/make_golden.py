"""Writes the stored oracle results used by the full-size GPU parity tests.

Calls only the oracle (oracle/) and the seeded input generators; run from the
repository root:  python -m tests.golden.make_golden [name ...]
Each entry: the workload, the start (restart index), the stopping rule and the
oracle's final fit, sweep count and per-sweep fit history head.
"""
import json
import os
import sys
import time

import numpy as np

from oracle import cp
from paper_1111_6091_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def als_reference(name, max_sweeps=10000, fit_tol=1e-12, restart=0):
    Z, _, spec = synth.workload(name)
    A0 = synth.uniform_start(Z.shape, spec["R"], spec["seed"], restart)
    t = time.time()
    A, h = cp.als(Z, A0, max_sweeps=max_sweeps, fit_tol=fit_tol, record="fused")
    el = time.time() - t
    return {
        "workload": name, "restart": restart, "fit_tol": fit_tol, "max_sweeps": max_sweeps,
        "sweeps": h["sweeps"], "final_fit_fused": h["fit"][-1], "final_fit_exact": cp.fit(Z, A),
        "fit_head": h["fit"][:20], "oracle_seconds": el,
        "lambda": [float(x) for x in cp.weights(A)],
    }


def main(names):
    for name in names:
        ref = als_reference(name)
        path = os.path.join(HERE, f"als_{name}.json")
        with open(path, "w") as f:
            json.dump(ref, f, indent=1)
        print(name, ref["sweeps"], ref["final_fit_exact"], f"{ref['oracle_seconds']:.1f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1_20cube_r3"])
