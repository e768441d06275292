"""The benchmark's launch configuration: the three 1024^2 dipole instances
(gamma 0.5, 0.75, 1.0), each with its own handle, HIP stream and host thread,
run concurrently through nf_run.  The states must be bitwise those of the same
runs one after another on one stream (the kernels and their reductions are
deterministic and the handles share nothing), and the gamma = 0.75 instance
is checked against the oracle after one step."""

import threading

import numpy as np
import pytest

import oracle as O
from paper_2606_06720_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

GAMMAS = (0.5, 0.75, 1.0)


def test_three_stream_instances_bitwise_equal_to_sequential_runs():
    import torch

    from paper_2606_06720_amd import nf as NF

    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    N, steps = 1024, 4
    ws = [W.dipole_workload(N, g) for g in GAMMAS]
    grids = [NF.Grid(w["n"], w["L"]) for w in ws]
    r = [T(w["r"]) for w in ws]
    S = [T(w["S"]) for w in ws]

    def fresh():
        return [T(w["m0"]) for w in ws], [torch.zeros((N, N), dtype=torch.float64, device=dev) for _ in ws]

    # concurrent: one stream and one host thread per instance
    mc, pc = fresh()
    streams = [torch.cuda.Stream(device=dev) for _ in ws]
    torch.cuda.synchronize()
    infos = [None] * 3

    def go(k):
        w = ws[k]
        with torch.cuda.stream(streams[k]):
            infos[k] = grids[k].run(w["c2"], w["D2"], w["gamma"], w["dt"], steps, mc[k], pc[k], r[k], S[k],
                                    rtol=w["rtol"], max_iter=1000)

    th = [threading.Thread(target=go, args=(k,)) for k in range(3)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    assert all(i is not None for i in infos)
    # one after another on the default stream
    ms, ps = fresh()
    for k, w in enumerate(ws):
        grids[k].run(w["c2"], w["D2"], w["gamma"], w["dt"], steps, ms[k], ps[k], r[k], S[k], rtol=w["rtol"],
                     max_iter=1000)
    torch.cuda.synchronize()
    for k in range(3):
        assert torch.equal(mc[k], ms[k]) and torch.equal(pc[k], ps[k]), GAMMAS[k]
    # one concurrent step of the gamma = 0.75 instance against the oracle
    m1, p1 = fresh()
    th = []
    for k in range(3):
        w = ws[k]

        def one(k=k, w=w):
            with torch.cuda.stream(streams[k]):
                grids[k].step(w["c2"], w["D2"], w["gamma"], w["dt"], m1[k], p1[k], r[k], S[k], rtol=w["rtol"])

        th.append(threading.Thread(target=one))
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    w = ws[1]
    mo, po, _ = O.step(w["m0"], None, w["r"], w["S"], w["c2"], w["D2"], w["gamma"], w["dt"], w["rtol"])
    rel = lambda a, b: float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))
    assert rel(m1[1].cpu().numpy(), mo) <= 1e-10
    assert rel(p1[1].cpu().numpy(), po) <= 1e-10
    for g in grids:
        g.close()
