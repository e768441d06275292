"""The precision form at its own sizes against the FP64 oracle: one time step of
the dipole workload (gamma 0.75) from m0 on the 4096^2 grid and on the 256^3
grid, FP64 and FP32-refined handles, compared with the oracle's values stored
by tests/golden/make_precision_golden.py (4096 sampled nodes per field; the
relative L2 error over the samples, per field).  Bars: 1e-10 for FP64, 1e-6
for the FP32 form with FP64 refinement."""

import json
import os

import numpy as np
import pytest

from paper_2606_06720_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def sampled_errors(gold, m, p):
    idx = np.asarray(gold["index"])
    out = {}
    for k, v in gold["fields"].items():
        f = p if k == "p" else m[int(k[1:])]
        got = f.reshape(-1)[idx]
        want = np.asarray(v["sample"])
        out[k] = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    return out


@pytest.mark.parametrize("case", ["4096x2", "256x3"])
def test_precision_form_one_step_matches_oracle(case):
    import torch

    from paper_2606_06720_amd import nf as NF

    with open(os.path.join(GOLDEN, "precision_%s.json" % case)) as fh:
        gold = json.load(fh)
    N, ndim = (int(v) for v in case.split("x"))
    w = W.dipole_workload(N, 0.75, ndim=ndim)
    assert gold["grid"] == [N] * ndim and gold["params"]["dt"] == w["dt"] and gold["params"]["c2"] == w["c2"]
    dev = torch.device("cuda:0")
    r, S = torch.from_numpy(w["r"]).to(dev), torch.from_numpy(w["S"]).to(dev)
    for dtype, bar in ((NF.NF_F64, 1e-10), (NF.NF_F32_REFINED, 1e-6)):
        print("precision case", case, "dtype", dtype, flush=True)
        m = torch.from_numpy(w["m0"]).to(dev)
        p = torch.zeros_like(r)
        with NF.Grid(w["n"], w["L"], dtype=dtype) as g:
            rc, si = g.step(w["c2"], w["D2"], w["gamma"], w["dt"], m, p, r, S, rtol=w["rtol"])
        err = sampled_errors(gold, m.cpu().numpy(), p.cpu().numpy())
        print(case, "dtype", dtype, "iters", si.solve.iters, "oracle iters", gold["pcg_iters"], err, flush=True)
        for k, e in err.items():
            assert e <= bar, (k, e)
        if dtype == NF.NF_F64:
            assert abs(si.solve.iters - gold["pcg_iters"]) <= 1
        del m, p
        torch.cuda.empty_cache()
