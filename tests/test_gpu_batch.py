"""GPU tests of the ensemble entry points (nf_batch_create / nf_batch_run):
every instance of a batch must produce bitwise the fields and counters of
nf_run on its own handle (same kernel bodies, deterministic reductions),
whatever the partition count (fixed or tuned), and the oracle's time loop
within the FP64 bar.  A stop in one partition ends all of them at the same
point."""

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


def _run_batch(env, inst, dtype, steps, dt, rtol, parts=None, out=None, max_iter=1000):
    NF, T, torch = env
    ms = [T(w["m0"]) for w in inst]
    ps = [torch.zeros_like(T(w["r"])) for w in inst]
    rs = [T(w["r"]) for w in inst]
    Ss = [T(w["S"]) for w in inst]
    if out is not None:
        out.update(m=ms, p=ps)
    with NF.Batch([w["n"] for w in inst], dtype=dtype) as b:
        if parts is not None:
            b.set_partitions(parts)
        infos = b.run([w["prm"] for w in inst], dt, steps, ms, ps, rs, Ss, rtol=rtol, max_iter=max_iter)
        if out is not None:
            out["parts"] = b.partitions()
    return ms, ps, infos


def _run_single(env, w, dtype, steps, dt, rtol, max_iter=1000):
    NF, T, torch = env
    m, r, S = T(w["m0"]), T(w["r"]), T(w["S"])
    p = torch.zeros_like(r)
    with NF.Grid(w["n"], dtype=dtype) as g:
        info = g.run(*w["prm"], dt, steps, m, p, r, S, rtol=rtol, max_iter=max_iter)
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


@pytest.mark.parametrize("dtype_name", ["NF_F64", "NF_F32_REFINED"])
def test_batch_capped_solves_match_single_runs(env, dtype_name):
    # max_iter below what the solves need: every solve stops at the cap, takes
    # the final residual test there and counts as unconverged, as in nf_run;
    # a looser cap lets the instances that converge fast finish while the
    # others are capped in the same launches
    NF, T, torch = env
    dtype = getattr(NF, dtype_name)
    inst = _instances(((64, 2), (32, 2)), 1500)
    for max_iter in (3, 12):
        for parts in (1, 2):
            ms, ps, infos = _run_batch(env, inst, dtype, 3, 5e-4, 1e-10, parts=parts, max_iter=max_iter)
            for i, w in enumerate(inst):
                m1, p1, info1 = _run_single(env, w, dtype, 3, 5e-4, 1e-10, max_iter=max_iter)
                assert torch.equal(ms[i], m1) and torch.equal(ps[i], p1), (max_iter, parts, i)
                assert _key(infos[i]) == _key(info1), (max_iter, parts, i, infos[i], info1)
        if max_iter == 3:
            assert all(x.unconverged_solves == 4 for x in infos), [x.unconverged_solves for x in infos]


def _rect_instance(n, L, seed):
    """An ensemble-type instance on an Nx x Ny grid over an Lx x Ly box."""
    rng = np.random.default_rng(seed)
    X = W.grid_coords(n, L)
    S = W.gaussian(X, (0.25 * L[0], 0.5 * L[1]), 0.05 * L[1]) - W.gaussian(X, (0.75 * L[0], 0.5 * L[1]), 0.05 * L[1])
    return dict(n=n, L=L, r=np.ascontiguousarray(0.05 + 0.05 * W.smooth_random_field(rng, n, L)),
                S=np.ascontiguousarray(S - S.mean()), m0=np.ascontiguousarray(rng.random((2, n[1], n[0]))),
                prm=(float(rng.uniform(5.0, 50.0)), float(rng.uniform(1e-5, 1e-3)), float(rng.uniform(0.5, 1.25))))


@pytest.mark.parametrize("dtype_name", ["NF_F64", "NF_F32_REFINED"])
def test_batch_paper_grids_and_boxes(env, dtype_name):
    # launch groups keyed by grid and box: the paper's 50 * 2^k grids (radix-5
    # stages, square and rectangular) next to power-of-two rectangular grids
    # over non-square boxes, two partitions; every instance bitwise its own
    # nf_run on a handle of that box, and the FP64 fields against the oracle's
    # time loop
    NF, T, torch = env
    dtype = getattr(NF, dtype_name)
    inst = _instances(((50, 2), (100, 1)), 8000)
    inst += [_rect_instance((64, 32), (2.0, 1.0), 8100), _rect_instance((64, 32), (2.0, 1.0), 8101),
             _rect_instance((32, 64), (1.0, 0.5), 8102), _rect_instance((100, 50), (2.0, 1.0), 8103),
             _rect_instance((100, 50), (2.0, 1.0), 8104)]
    steps, dt = 3, 5e-4
    ms = [T(w["m0"]) for w in inst]
    ps = [torch.zeros_like(T(w["r"])) for w in inst]
    rs = [T(w["r"]) for w in inst]
    Ss = [T(w["S"]) for w in inst]
    with NF.Batch([w["n"] for w in inst], [w["L"] for w in inst], dtype=dtype) as b:
        b.set_partitions(2)
        infos = b.run([w["prm"] for w in inst], dt, steps, ms, ps, rs, Ss, rtol=1e-12)
    for i, w in enumerate(inst):
        m1, r1, S1 = T(w["m0"]), T(w["r"]), T(w["S"])
        p1 = torch.zeros_like(r1)
        with NF.Grid(w["n"], w["L"], dtype=dtype) as g:
            info1 = g.run(*w["prm"], dt, steps, m1, p1, r1, S1, rtol=1e-12)
        assert torch.equal(ms[i], m1) and torch.equal(ps[i], p1), (dtype_name, i)
        assert _key(infos[i]) == _key(info1), (dtype_name, i)
        if dtype_name == "NF_F64":
            mo, po, _ = O.run(w["m0"], None, w["r"], w["S"], *w["prm"], dt, steps, rtol=1e-12, L=w["L"])
            assert rel(ms[i].cpu().numpy(), mo) <= 1e-10, i
            assert rel(ps[i].cpu().numpy(), po) <= 1e-10, i


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


@pytest.mark.parametrize("dtype_name", ["NF_F64", "NF_F32_REFINED"])
def test_batch_partition_count_does_not_change_results(env, dtype_name):
    NF, T, torch = env
    dtype = getattr(NF, dtype_name)
    inst = _instances(((64, 3), (128, 2), (32, 2)), 5000)
    ref = _run_batch(env, inst, dtype, 4, 5e-4, 1e-10, parts=1)
    for parts in (2, 3, 4, 0):
        got = {}
        ms, ps, infos = _run_batch(env, inst, dtype, 4, 5e-4, 1e-10, parts=parts, out=got)
        k, tune_ms = got["parts"]
        print("parts", parts, "in use", k, "tuning ms", tune_ms)
        assert k == parts if parts else 1 <= k <= 4
        if parts == 0:
            # the tuner timed every count up to min(4, count) and kept the fastest
            assert all(t > 0 for t in tune_ms) and tune_ms[k - 1] == min(tune_ms)
        for i in range(len(inst)):
            assert torch.equal(ms[i], ref[0][i]) and torch.equal(ps[i], ref[1][i]), (parts, i)
            assert _key(infos[i]) == _key(ref[2][i]), (parts, i)


def test_batch_partitions_stop_together(env):
    NF, T, torch = env
    # incompatible S in one partition: nothing is advanced in any partition
    inst = _instances(((32, 4),), 6000)
    inst[3]["S"] = inst[3]["S"] + 1e-3
    got = {}
    with pytest.raises(NF.NfError) as e:
        _run_batch(env, inst, NF.NF_F64, 2, 5e-4, 1e-10, parts=2, out=got)
    assert e.value.code == NF.NF_EINCOMPAT
    for i, w in enumerate(inst):
        assert np.array_equal(got["m"][i].cpu().numpy(), w["m0"]), i
    # activation overflow in one partition at the first step: every partition
    # stops after that step, as with a single partition
    inst = _instances(((32, 4),), 6001)
    for w in inst:
        w["prm"] = (1.0, 1e-3, 0.75)
    inst[2]["prm"] = (1e6, 1e-3, 0.75)
    inst[2]["S"] = 1e3 * inst[2]["S"]
    runs = []
    for parts in (1, 2):
        got = {}
        with pytest.raises(NF.NfError) as e:
            _run_batch(env, inst, NF.NF_F64, 3, 1.0, 1e-10, parts=parts, out=got)
        assert e.value.code == NF.NF_ENONFINITE
        runs.append(got)
    for i in (0, 1, 3):
        assert torch.equal(runs[0]["m"][i], runs[1]["m"][i]), i
        assert not np.array_equal(runs[1]["m"][i].cpu().numpy(), inst[i]["m0"]), i
    with NF.Batch([(32, 32)] * 2) as b:
        for bad in (-1, 3, 5):
            with pytest.raises(NF.NfError) as e:
                b.set_partitions(bad)
            assert e.value.code == NF.NF_EINVAL


@pytest.mark.parametrize("dtype_name", ["NF_F64", "NF_F32_REFINED"])
def test_batch_graph_replays_match_eager_launches(env, dtype_name):
    # the same handle runs several times (recorded chunks replayed, with the
    # eager passes of the time step and host synchronisation in between); every
    # run must be bitwise the run of a handle that launches kernel by kernel
    NF, T, torch = env
    dtype = getattr(NF, dtype_name)
    inst = _instances(((32, 3), (64, 2)), 7000)
    states = []
    for graphs in (True, False):
        ms = [T(w["m0"]) for w in inst]
        ps = [torch.zeros_like(T(w["r"])) for w in inst]
        rs = [T(w["r"]) for w in inst]
        Ss = [T(w["S"]) for w in inst]
        seq = []
        with NF.Batch([w["n"] for w in inst], dtype=dtype) as b:
            b.set_partitions(2)
            b.set_graphs(graphs)
            for rep in range(4):
                infos = b.run([w["prm"] for w in inst], 5e-4, 3, ms, ps, rs, Ss, rtol=1e-10)
                torch.cuda.synchronize()
                seq.append(([x.clone() for x in ms], [x.clone() for x in ps], [_key(i) for i in infos]))
        states.append(seq)
    for rep in range(4):
        g, e = states[0][rep], states[1][rep]
        for i in range(len(inst)):
            assert torch.equal(g[0][i], e[0][i]) and torch.equal(g[1][i], e[1][i]), (rep, i)
        assert g[2] == e[2], rep


def test_batch_wide_rows(env):
    # rows of 2048 and 4096 points: the split update writes p in a pass of its
    # own and runs activation and relaxation in the two-row tile, in the batch
    # as on a single handle (bitwise), and within the FP64 bar of the oracle
    NF, T, torch = env
    rng = np.random.default_rng(5000)
    inst = []
    for n, gamma in (((2048, 16), 0.75), ((4096, 8), 1.0), ((4096, 8), 0.5)):
        sh = n[::-1]
        S = rng.standard_normal(sh)
        inst.append(dict(n=n, L=(1.0, n[1] / n[0]), m0=rng.uniform(-1.0, 1.0, (2,) + sh),
                         r=rng.uniform(0.05, 0.15, sh), S=S - S.mean(), prm=(50.0, 1e-4, gamma)))
    steps, dt = 3, 5e-4
    ms = [T(w["m0"]) for w in inst]
    ps = [torch.zeros_like(T(w["r"])) for w in inst]
    with NF.Batch([w["n"] for w in inst], L=[w["L"] for w in inst]) as b:
        infos = b.run([w["prm"] for w in inst], dt, steps, ms, ps, [T(w["r"]) for w in inst],
                      [T(w["S"]) for w in inst], rtol=1e-12)
    for i, w in enumerate(inst):
        m1, p1 = T(w["m0"]), torch.zeros_like(T(w["r"]))
        with NF.Grid(w["n"], w["L"]) as g:
            info1 = g.run(*w["prm"], dt, steps, m1, p1, T(w["r"]), T(w["S"]), rtol=1e-12)
        assert torch.equal(ms[i], m1) and torch.equal(ps[i], p1), i
        assert _key(infos[i]) == _key(info1), i
    w = inst[2]
    mo, po, _ = O.run(w["m0"], None, w["r"], w["S"], *w["prm"], dt, steps, rtol=1e-12, L=w["L"])
    assert rel(ms[2].cpu().numpy(), mo) <= 1e-10
    assert rel(ps[2].cpu().numpy(), po) <= 1e-10
