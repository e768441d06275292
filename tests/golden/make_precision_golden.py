"""Writes the oracle's reference values for the precision-form sizes.

For the dipole workload (gamma = 0.75, dt = 5e-4, D^2 = 1e-4, c^2 = 50, PCG
relative tolerance 1e-10) on the 4096^2 grid and on the 256^3 grid, one time
step of Algorithm 1 from m0 with a cold pressure start is taken by the CPU
oracle (oracle/nf_oracle.py, FP64).  The full fields are too large to store,
so the file keeps, for m^1 (every component) and p[m^0]:
  * the full discrete L2 norms sum f^2 (for relative errors),
  * the values at 4096 node indices drawn with numpy default_rng(20260) from
    the flattened [z][y][x] layout (the same indices for every field),
  * the PCG iteration count.
Only the oracle and the seeded input generators are called.

Usage: python tests/golden/make_precision_golden.py {4096x2|256x3}
writes tests/golden/precision_<case>.json.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2606_06720_amd import workloads as W  # noqa: E402

NSAMPLE = 4096
SEED = 20260


def make(case):
    N, ndim = (int(v) for v in case.split("x"))
    w = W.dipole_workload(N, 0.75, ndim=ndim)
    t0 = time.time()
    m1, p0, info = O.step(w["m0"], None, w["r"], w["S"], w["c2"], w["D2"], w["gamma"], w["dt"], w["rtol"], 1000)
    elapsed = time.time() - t0
    npts = N ** ndim
    idx = np.sort(np.random.default_rng(SEED).choice(npts, size=NSAMPLE, replace=False))
    out = {
        "what": "oracle FP64: one time step of the dipole workload from m0 (cold pressure start)",
        "grid": [N] * ndim,
        "params": {"gamma": w["gamma"], "c2": w["c2"], "D2": w["D2"], "dt": w["dt"], "rtol": w["rtol"]},
        "pcg_iters": info.iters,
        "oracle_seconds": elapsed,
        "sample_seed": SEED,
        "index": idx.tolist(),
        "fields": {},
    }
    fields = {("m%d" % c): m1[c] for c in range(ndim)}
    fields["p"] = p0
    for k, f in fields.items():
        flat = f.ravel()
        out["fields"][k] = {"sum_sq": float(np.sum(flat * flat)), "sample": [float(v) for v in flat[idx]]}
    path = os.path.join(HERE, "precision_%s.json" % case)
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(path, "iters", info.iters, "%.0f s" % elapsed, flush=True)


if __name__ == "__main__":
    for c in sys.argv[1:] or ["4096x2", "256x3"]:
        make(c)
