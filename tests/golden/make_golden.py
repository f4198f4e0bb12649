"""Write the full-size oracle results the GPU parity tests compare against.

    python tests/golden/make_golden.py [name ...]

For each workload (the 8-D Gaussian, 10 x 1e7 events; the LO 2->2 toy,
10 x 1e8; massless 2->4 RAMBO, 10 x 5e7; all seed 0, 1.5 refinement
exponent, refinement after every iteration but the last) this runs the FP64
CPU oracle's whole run (oracle.run: the steps of the method as the paper's
Sec. 3.1 example drives them, iteration by iteration from the uniform grid)
and stores its per-iteration (I_t, sigma_t), the final grid and the
non-finite count in tests/golden/<name>_fp64_seed0.json. Only the oracle is
called; nothing here runs on, or reads anything from, the GPU path.
The workloads run in parallel processes (about two minutes in all, the RAMBO
run being the longest).
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NAMES = ("gauss8d", "lo_toy", "rambo24")


def path_of(name: str) -> str:
    return os.path.join(HERE, f"{name}_fp64_seed0.json")


def make(name: str) -> str:
    import oracle
    from paper_2010_09341_amd import workloads as W
    wl = W.WORKLOADS[name]
    t0 = time.perf_counter()
    I_t, s_t, edges, bad = oracle.run(wl.dim, wl.nb, wl.fid, wl.params, wl.n_events, wl.seed,
                                      wl.n_iter, wl.alpha)
    dt = time.perf_counter() - t0
    rec = {
        "what": f"FP64 oracle run of {wl.note}; seed {wl.seed}, refinement exponent {wl.alpha}",
        "written_by": "tests/golden/make_golden.py (calls oracle.run only)",
        "workload": name, "dim": wl.dim, "n_bins": wl.nb, "integrand_id": wl.fid,
        "params": wl.params, "n_events": wl.n_events, "n_iter": wl.n_iter, "seed": wl.seed,
        "alpha": wl.alpha, "oracle_seconds": round(dt, 1), "n_nonfinite": int(bad),
        # repr() of a binary64 value reads back bitwise
        "I_t": [repr(float(v)) for v in I_t],
        "sigma_t": [repr(float(v)) for v in s_t],
        "edges": [[repr(float(v)) for v in row] for row in edges],
    }
    with open(path_of(name), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return f"{name}: {dt:.1f} s"


def load(name: str):
    """(record, I_t, sigma_t, edges) with the arrays as binary64 numpy arrays."""
    import numpy as np
    with open(path_of(name)) as f:
        rec = json.load(f)
    I_t = np.array([float(v) for v in rec["I_t"]])
    s_t = np.array([float(v) for v in rec["sigma_t"]])
    edges = np.array([[float(v) for v in row] for row in rec["edges"]])
    return rec, I_t, s_t, edges


if __name__ == "__main__":
    names = sys.argv[1:] or list(NAMES)
    with mp.get_context("fork").Pool(len(names)) as pool:
        for line in pool.imap_unordered(make, names):
            print(line, flush=True)
