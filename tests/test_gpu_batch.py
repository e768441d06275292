"""GPU tests of the ensemble entry points (nf_batch_create / nf_batch_run):
every instance of a batch must produce bitwise the fields and counters of
nf_run on its own handle (same kernel bodies, deterministic reductions), and
the oracle's time loop within the FP64 bar."""

import numpy as np
import pytest

import oracle as O
from paper_2606_06720_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2606_06720_amd import nf as NF

    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return NF, T, torch


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _instances(mix, seed0):
    """Ensemble-type instances (per-instance r, m0 and (c2, D2, gamma) draws)."""
    out = W.ensemble_workload(mix, seed0)
    for w in out:
        w["prm"] = (w["c2"], w["D2"], w["gamma"])
    return out


def _key(info):
    # the counters nf_batch_run reports (energies are NaN: no energy stopping)
    return (info.steps, info.stop_reason, info.last_dm, info.total_cg_iters, info.unconverged_solves)


def _run_batch(env, inst, dtype, steps, dt, rtol):
    NF, T, torch = env
    ms = [T(w["m0"]) for w in inst]
    ps = [torch.zeros_like(T(w["r"])) for w in inst]
    rs = [T(w["r"]) for w in inst]
    Ss = [T(w["S"]) for w in inst]
    with NF.Batch([w["n"] for w in inst], dtype=dtype) as b:
        infos = b.run([w["prm"] for w in inst], dt, steps, ms, ps, rs, Ss, rtol=rtol)
    return ms, ps, infos


def _run_single(env, w, dtype, steps, dt, rtol):
    NF, T, torch = env
    m, r, S = T(w["m0"]), T(w["r"]), T(w["S"])
    p = torch.zeros_like(r)
    with NF.Grid(w["n"], dtype=dtype) as g:
        info = g.run(*w["prm"], dt, steps, m, p, r, S, rtol=rtol)
    return m, p, info


@pytest.mark.parametrize("dtype_name", ["NF_F64", "NF_F32_REFINED"])
def test_batch_is_bitwise_the_single_instance_run(env, dtype_name):
    NF, T, torch = env
    dtype = getattr(NF, dtype_name)
    inst = _instances(((64, 3), (32, 1), (128, 1), (16, 1)), 1000)
    ms, ps, infos = _run_batch(env, inst, dtype, 6, 5e-4, 1e-10)
    for i, w in enumerate(inst):
        m1, p1, info1 = _run_single(env, w, dtype, 6, 5e-4, 1e-10)
        assert torch.equal(ms[i], m1) and torch.equal(ps[i], p1), i
        assert _key(infos[i]) == _key(info1), (i, infos[i], info1)


def test_batch_matches_oracle(env):
    NF, T, torch = env
    inst = _instances(((32, 2), (64, 1)), 2000)
    ms, ps, infos = _run_batch(env, inst, NF.NF_F64, 5, 5e-4, 1e-12)
    for i, w in enumerate(inst):
        mo, po, rio = O.run(w["m0"], None, w["r"], w["S"], *w["prm"], 5e-4, 5, rtol=1e-12)
        assert infos[i].steps == 5 and infos[i].unconverged_solves == 0
        assert abs(infos[i].total_cg_iters - rio.total_cg_iters) <= 6
        assert rel(ms[i].cpu().numpy(), mo) <= 1e-10
        assert rel(ps[i].cpu().numpy(), po) <= 1e-10
        assert abs(infos[i].last_dm - rio.last_dm) <= 1e-9 * rio.last_dm


def test_batch_ensemble_shape_mix(env):
    # the ensemble's grid mix at reduced counts: 256^2, 512^2 and 1024^2
    # instances in one batch, against single-instance runs of three of them
    NF, T, torch = env
    inst = _instances(((256, 3), (512, 2), (1024, 1)), 3000)
    ms, ps, infos = _run_batch(env, inst, NF.NF_F64, 4, 5e-4, 1e-10)
    for i in (0, 3, 5):
        m1, p1, info1 = _run_single(env, inst[i], NF.NF_F64, 4, 5e-4, 1e-10)
        assert torch.equal(ms[i], m1) and torch.equal(ps[i], p1), i
        assert _key(infos[i]) == _key(info1)


def test_batch_failure_paths(env):
    NF, T, torch = env
    inst = _instances(((32, 2),), 4000)
    inst[1]["S"] = inst[1]["S"] + 1e-3
    with pytest.raises(NF.NfError) as e:
        _run_batch(env, inst, NF.NF_F64, 2, 5e-4, 1e-10)
    assert e.value.code == NF.NF_EINCOMPAT
    inst = _instances(((32, 1),), 4001)
    inst[0]["prm"] = (1.0, 1e-3, 0.0)
    with pytest.raises(NF.NfError) as e:
        _run_batch(env, inst, NF.NF_F64, 2, 5e-4, 1e-10)
    assert e.value.code == NF.NF_EINVAL
    with pytest.raises(NF.NfError) as e:
        NF.Batch([(32, 33)])
    assert e.value.code == NF.NF_EINVAL
