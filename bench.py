"""Throughput benchmark of the spectral network-formation hot path on one GPU.

Workload: the 2D periodic 1024 x 1024 FP64 case -- r = 0.05 + 0.05 f (f a
smooth random field of 16 low-wavenumber modes), a Gaussian source/sink pair
(sigma 0.02), m0 uniform[0,1]^2, D^2 = 1e-4, c^2 = 50, dt = 5e-4, PCG relative
tolerance 1e-10 -- run for the three metabolic exponents gamma = 0.5, 0.75, 1.0.
One benchmark step advances all three instances by one time step (PCG solve +
split update), so a step processes 3 * 1024^2 grid points.  All inputs are
resident in device memory before the timed region.

Prints one JSON line (metric: grid-point-steps/s) with a roofline entry for the
dominant kernel (average execution span of its launches in the timed region,
stamped by the kernel itself on the device wall clock: first workgroup start
to last workgroup end) and a CPU-oracle baseline on a bounded sample.
"""

import argparse
import hashlib
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GAMMAS = (0.5, 0.75, 1.0)
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, public spec

# algorithmic bytes per grid point of one launch of each PCG-loop kernel (FP64):
#   row_flux : reads grad_x, grad_y (2 x 8), m (16), r (8); writes F_x, F_y (2 x 8)
#   col_div  : reads F_x, F_y (16), d, r (16); writes q (8)
#   col_update: reads x, d, r, q (32); writes x, r, d (24) and grad_x, grad_y (16)
KERNEL_BYTES_PER_POINT = {"row_flux": 56.0, "col_div": 40.0, "col_update": 72.0}
KERNEL_IDS = {"row_flux": 0, "col_div": 1, "col_update": 2}
# algorithmic bytes per grid point of the passes of one time step outside the
# PCG loop: gradient of the warm start (24), initial operator apply (56 + 32),
# first update (32), split: p and gradient (16 + 24), activation/relaxation
# pass (64), heat multiplier (32), final row pass with Delta m (48)
STEP_BYTES_PER_POINT = 328.0
KERNEL_SOURCES = ("paper_2606_06720_amd/csrc/nf_kernels.hip", "paper_2606_06720_amd/csrc/nf_fft.hpp",
                  "paper_2606_06720_amd/csrc/nf_tiles.hpp", "paper_2606_06720_amd/csrc/nf_internal.h")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, n):
    """Counter-derived HBM bytes per launch from the committed profile summary,
    or None if absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%d.json" % (kernel, n))
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def load_rocprof_duration(kernel, n):
    """Working-dispatch average duration (us) of the kernel in the committed
    rocprofv3 trace of the default bench command, or None if absent or taken
    on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "duration_%s_%d.json" % (kernel, n))
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("concurrent_working_avg_us")


def _oracle_steps(N, gamma, steps, barrier=None):
    """Worker of the CPU baseline: `steps` oracle time steps of the dipole case
    from m0 (the start of the GPU line's window); returns (seconds, PCG iterations)."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import oracle as O
    from paper_2606_06720_amd import workloads as W

    w = W.dipole_workload(N, gamma)
    m, p = w["m0"], None
    if barrier is not None:
        barrier.wait()
    iters = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        m, p, info = O.step(m, p, w["r"], w["S"], w["c2"], w["D2"], w["gamma"], w["dt"], w["rtol"])
        iters += info.iters
    return time.perf_counter() - t0, iters


def _pool_worker(args):
    return _oracle_steps(*args, barrier=_POOL_BARRIER)


_POOL_BARRIER = None


def _pool_init(b):
    global _POOL_BARRIER
    _POOL_BARRIER = b


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(N, steps, max_workers=16):
    """The oracle (numpy FP64, single-threaded FFTs) on the host cores, on a bounded
    sample of the GPU line's window: its first `steps` time steps from m0.
    One thread: the gamma = 0.75 instance in this process.  All cores: one
    worker process per available core (at most `max_workers`, the CPU share of
    one GPU), each running one instance (the three gamma values in turn) for
    the same steps, started together; the aggregate rate is the sum of the
    workers' rates.  Runs before anything touches the GPU."""
    import multiprocessing as mp

    t1, it1 = _oracle_steps(N, 0.75, steps)
    cores = max(1, min(len(os.sched_getaffinity(0)), max_workers))
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(cores)
    jobs = [(N, GAMMAS[k % len(GAMMAS)], steps) for k in range(cores)]
    with ctx.Pool(cores, initializer=_pool_init, initargs=(barrier,)) as pool:
        res = pool.map(_pool_worker, jobs, chunksize=1)
    rate_all = sum(N * N * steps / t for t, _ in res)
    iters_all = sum(i for _, i in res)
    t_all = max(t for t, _ in res)
    return {
        "value": rate_all,
        "unit": "grid-point-steps/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "first %d time step(s) from m0 of the %d^2 dipole instances (the start of the GPU line's window); "
                  "one thread: gamma 0.75, %d PCG iterations, %.1f s; all cores: %d worker processes (one instance "
                  "each, gammas in turn, started together), %d PCG iterations, slowest %.1f s; numpy FFT"
                  % (steps, N, it1, t1, cores, iters_all, t_all),
        "value_1": N * N * steps / t1,
        "value_all": rate_all,
        "cores_all": cores,
        "cpu_model": cpu_model(),
        "pcg_iters_per_step": it1 / steps,
        # like-for-like across windows with different iteration counts: grid points
        # times PCG iterations per second
        "grid_point_iters_per_s_1": N * N * it1 / t1,
        "grid_point_iters_per_s_all": sum(N * N * i / t for t, i in res),
    }


def adjoint_cost(N, steps, fd_dirs=32):
    """Cost of reverse mode at N^2 (gamma = 0.75, the 1024^2 dipole case): one
    nf_step_adjoint against one nf_step (both from the same state), and the
    sqrt(T)-checkpointed gradient of the misfit of the final |m| after `steps`
    steps against the forward run of those steps."""
    import numpy as np
    import torch

    from paper_2606_06720_amd import adjoint as A
    from paper_2606_06720_amd import nf as NF
    from paper_2606_06720_amd import workloads as W

    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    w = W.dipole_workload(N, 0.75)
    prm = (w["c2"], w["D2"], w["gamma"])
    r, S, m0 = T(w["r"]), T(w["S"]), T(w["m0"])
    f2 = W.smooth_random_field(np.random.default_rng(6), (N, N), 1.0)
    rtol = 1e-10
    with NF.Grid(w["n"], w["L"]) as g:
        m_tgt, _ = A.forward_states(g, prm, w["dt"], steps, m0, T(w["r"] * (1 + 0.1 * f2)), S, rtol, 1000, steps)
        # warm state after a few steps
        m = m0.clone()
        p = torch.zeros_like(r)
        for _ in range(5):
            g.step(*prm, w["dt"], m, p, r, S, rtol=rtol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m_T, ckpt = A.forward_states(g, prm, w["dt"], steps, m0, r, S, rtol, 1000, steps + 1)
        torch.cuda.synchronize()
        t_run = time.perf_counter() - t0
        stride = int(np.ceil(np.sqrt(steps)))
        # one untimed gradient first, so that the checkpoint buffers come from
        # the caching allocator in the timed one
        m_T, ckpt = A.forward_states(g, prm, w["dt"], steps, m0, r, S, rtol, 1000, stride)
        _, lam_T = A.misfit_loss(m_T, m_tgt)
        A.adjoint_sweep(g, prm, w["dt"], steps, r, S, ckpt, lam_T, rtol, 1000, stride)
        del ckpt
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m_T, ckpt = A.forward_states(g, prm, w["dt"], steps, m0, r, S, rtol, 1000, stride)
        _, lam_T = A.misfit_loss(m_T, m_tgt)
        torch.cuda.synchronize()
        t_ckpt = time.perf_counter() - t0
        st = {}
        t0 = time.perf_counter()
        A.adjoint_sweep(g, prm, w["dt"], steps, r, S, ckpt, lam_T, rtol, 1000, stride, st)
        torch.cuda.synchronize()
        t_sweep = time.perf_counter() - t0
        # the same sweep with the recomputation in line (one handle, one stream),
        # for the cost of the adjoint steps themselves
        t0 = time.perf_counter()
        A.adjoint_sweep(g, prm, w["dt"], steps, r, S, ckpt, lam_T, rtol, 1000, stride, overlap=False)
        torch.cuda.synchronize()
        t_sweep_seq = time.perf_counter() - t0
        # the sweep recomputes every segment: time that part alone
        t0 = time.perf_counter()
        for c in sorted(ckpt):
            mm, pp = ckpt[c][0].clone(), ckpt[c][1].clone()
            for k in range(c, min(c + stride, steps)):
                g.step(*prm, w["dt"], mm, pp, r, S, rtol=rtol, max_iter=1000)
        torch.cuda.synchronize()
        t_rec = time.perf_counter() - t0
        fd = None
        if fd_dirs > 0:
            # central differences of the misfit along random directions, half
            # in r and half in S (S directions made mean-free), against the
            # checkpointed gradient; both at a tight PCG tolerance, since the
            # noise of a difference quotient is about rtol / h relative to the loss
            rtol_fd, h = 1e-12, 1e-6
            l0, gr, gS = A.run_gradient(g, prm, w["dt"], steps, m0, r, S, m_tgt, rtol=rtol_fd, max_iter=2000)

            def L(r_, S_):
                m_T, _ = A.forward_states(g, prm, w["dt"], steps, m0, r_, S_, rtol_fd, 2000, steps)
                return A.misfit_loss(m_T, m_tgt)[0]

            rng = np.random.default_rng(7)
            err_r, err_S = [], []
            for k in range(fd_dirs):
                if k % 8 == 0:
                    progress("adjoint finite differences: direction %d of %d" % (k, fd_dirs))
                v = rng.standard_normal((N, N))
                if k % 2 == 0:
                    vt = T(v)
                    fdv = (L(r + h * vt, S) - L(r - h * vt, S)) / (2 * h)
                    err_r.append(abs(fdv - float((gr * vt).sum())) / abs(float((gr * vt).sum())))
                else:
                    vt = T(v - v.mean())
                    fdv = (L(r, S + h * vt) - L(r, S - h * vt)) / (2 * h)
                    err_S.append(abs(fdv - float((gS * vt).sum())) / abs(float((gS * vt).sum())))
            fd = {"directions": fd_dirs, "h": h, "rtol": rtol_fd, "loss": l0,
                  "directions_r": len(err_r), "directions_S": len(err_S),
                  "max_rel_err_r": max(err_r) if err_r else None, "max_rel_err_S": max(err_S) if err_S else None,
                  "median_rel_err_r": float(np.median(err_r)) if err_r else None,
                  "median_rel_err_S": float(np.median(err_S)) if err_S else None}
    t_adj = t_sweep_seq - t_rec
    t_fwd = t_run / steps
    return {
        "fd_check": fd,
        "workload": "%d^2 dipole case, gamma 0.75, PCG rtol 1e-10, misfit of the final |m|" % N,
        "gradient_steps": steps,
        "checkpoint_stride": stride,
        "forward_step_ms": 1e3 * t_fwd,
        "adjoint_step_ms": 1e3 * t_adj / steps,
        "adjoint_over_forward_step": (t_adj / steps) / t_fwd,
        "forward_pcg_iters_per_step": st.get("recompute_iters", 0) / steps,
        "adjoint_pcg_iters_per_step": st.get("adjoint_iters", 0) / steps,
        "forward_run_ms": 1e3 * t_run,
        # the sweep recomputes segment j - 1 on a second handle and stream while the
        # adjoint steps of segment j run (adjoint.adjoint_sweep); sequential: in line
        "checkpointed_gradient_ms": 1e3 * (t_ckpt + t_sweep),
        "gradient_over_forward_run": (t_ckpt + t_sweep) / t_run,
        "checkpointed_gradient_sequential_ms": 1e3 * (t_ckpt + t_sweep_seq),
        "gradient_sequential_over_forward_run": (t_ckpt + t_sweep_seq) / t_run,
    }


def oracle_sample(case):
    """The oracle's stored one-step reference for the precision-form sizes
    (tests/golden/make_precision_golden.py), or None."""
    path = os.path.join(ROOT, "tests", "golden", "precision_%s.json" % case)
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return None


def sampled_errors(gold, m, p):
    """Relative L2 error over the stored sample nodes, per field (m components, p)."""
    import numpy as np

    idx = np.asarray(gold["index"])
    out = {}
    for k, v in gold["fields"].items():
        f = p if k == "p" else m[int(k[1:])]
        got = f.reshape(-1)[idx]
        want = np.asarray(v["sample"])
        out[k] = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    return out


def loop_pass_spans(g, w, m, p, r, S, N, real_bytes, steps=10):
    """Average execution span of each PCG-loop pass of handle g (stamped by the
    kernel on the device wall clock) over `steps` further time steps, with the
    algorithmic bandwidth it gives (bytes per point scaled by real_bytes / 8)."""
    out = {}
    for kname, kid in sorted(KERNEL_IDS.items(), key=lambda kv: kv[1]):
        g.time_kernel(kid)
        g.run(w["c2"], w["D2"], w["gamma"], w["dt"], steps, m, p, r, S, rtol=w["rtol"])
        ms, cnt = g.time_kernel_read()
        g.time_kernel(-1)
        if not cnt:
            continue
        us = 1e3 * ms / cnt
        gbs = KERNEL_BYTES_PER_POINT[kname] * real_bytes / 8.0 * N * N / (us * 1e-6) / 1e9
        out[kname] = {"avg_launch_us": us, "launches": cnt, "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


def precision_form(sizes, steps, warmup=3):
    """FP64 and FP32-refined pressure solves on the same GPU: ms per time step
    of the dipole case (gamma 0.75) at each (N, ndim), the relative L2
    difference of m and p between the forms after the same steps from the same
    state, and, where the oracle's reference is stored, the error of one step
    from m0 of each form against the FP64 oracle per field."""
    import numpy as np
    import torch

    from paper_2606_06720_amd import nf as NF
    from paper_2606_06720_amd import workloads as W

    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    out = {}
    for N, ndim in sizes:
        w = W.dipole_workload(N, 0.75, ndim=ndim)
        gold = oracle_sample("%dx%d" % (N, ndim))
        res = {}
        for dt_, name in ((NF.NF_F64, "f64"), (NF.NF_F32_REFINED, "f32_refined")):
            r, S = T(w["r"]), T(w["S"])
            with NF.Grid(w["n"], w["L"], dtype=dt_) as g:
                err = None
                if gold is not None:
                    m, p = T(w["m0"]), torch.zeros_like(r)
                    g.step(w["c2"], w["D2"], w["gamma"], w["dt"], m, p, r, S, rtol=w["rtol"])
                    err = sampled_errors(gold, m.cpu().numpy(), p.cpu().numpy())
                    del m, p
                m, p = T(w["m0"]), torch.zeros_like(r)
                g.run(w["c2"], w["D2"], w["gamma"], w["dt"], warmup, m, p, r, S, rtol=w["rtol"])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = g.run(w["c2"], w["D2"], w["gamma"], w["dt"], steps, m, p, r, S, rtol=w["rtol"])
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                res[name] = dict(ms_per_step=1e3 * t / steps, pcg_iters_per_step=info.total_cg_iters / steps,
                                 m=m.cpu().numpy(), p=p.cpu().numpy(), err=err)
                if ndim == 2:
                    # the PCG-loop passes of this form, one at a time, over a few more steps:
                    # average execution span per launch (in-kernel stamps) against the
                    # algorithmic bytes of the pass (half in the FP32 inner solve)
                    res[name]["passes"] = loop_pass_spans(g, w, m, p, r, S, N, 8 if dt_ == NF.NF_F64 else 4)
            progress("precision %d^%d %s: %.3f ms per step, vs oracle %s" % (N, ndim, name, 1e3 * t / steps, err))
            del m, r, S, p
            torch.cuda.empty_cache()
        a, b = res["f32_refined"], res["f64"]
        npts = float(N) ** ndim
        out["%d^%d" % (N, ndim)] = {
            "f64_grid_point_steps_per_s": npts / (1e-3 * b["ms_per_step"]),
            "f32_refined_grid_point_steps_per_s": npts / (1e-3 * a["ms_per_step"]),
            "f64_ms_per_step": b["ms_per_step"],
            "f32_refined_ms_per_step": a["ms_per_step"],
            "speedup": b["ms_per_step"] / a["ms_per_step"],
            "f64_pcg_iters_per_step": b["pcg_iters_per_step"],
            "f32_inner_iters_per_step": a["pcg_iters_per_step"],
            "rel_diff_m": float(np.linalg.norm(a["m"] - b["m"]) / np.linalg.norm(b["m"])),
            "rel_diff_p": float(np.linalg.norm(a["p"] - b["p"]) / np.linalg.norm(b["p"])),
            # one step from m0 against the FP64 oracle (relative L2 over 4096 sampled nodes per field)
            "f64_vs_oracle": b["err"],
            "f32_refined_vs_oracle": a["err"],
        }
        if ndim == 2:
            out["%d^%d" % (N, ndim)]["loop_passes"] = {"f64": b["passes"], "f32_refined": a["passes"]}
    return {"workload": "dipole case, gamma 0.75, PCG rtol 1e-10, %d steps after %d; vs_oracle: one step from m0 "
                        "against the oracle's stored values at sampled nodes" % (steps, warmup),
            "sizes": out}


def ensemble_cost(steps, check_steps=20, mix=None):
    """The ensemble of independent instances (grid mix as given) advanced by one
    batch (nf_batch_run), FP64 and FP32-refined: `steps` timed steps from m0,
    and, over the first `check_steps` steps from m0, the batch against the same
    instances run one after another (nf_run): rates and bitwise equality."""
    import numpy as np
    import torch

    from paper_2606_06720_amd import nf as NF
    from paper_2606_06720_amd import workloads as W

    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    inst = W.ensemble_workload(mix or W.ENSEMBLE_MIX)
    npts = sum(w["n"][0] * w["n"][1] for w in inst)
    prm = [(w["c2"], w["D2"], w["gamma"]) for w in inst]
    dt = W.ENSEMBLE_RUN["dt"]
    rtol = W.ENSEMBLE_RUN["rtol"]
    out = {"workload": "%d instances %s, per-instance (c2, D2, gamma) draws, dt %g, rtol %g; batch: %d steps from "
                       "m0 after tuning; comparison with one-by-one runs: the first %d steps from m0"
                       % (len(inst), [list(x) for x in (mix or W.ENSEMBLE_MIX)], dt, rtol, steps, check_steps)}
    rs = [T(w["r"]) for w in inst]
    Ss = [T(w["S"]) for w in inst]
    for dt_, name in ((NF.NF_F64, "f64"), (NF.NF_F32_REFINED, "f32_refined")):
        with NF.Batch([w["n"] for w in inst], dtype=dt_) as b:
            ms = [T(w["m0"]) for w in inst]
            ps = [torch.zeros_like(x) for x in rs]
            # the first run tunes the partition count (not timed)
            b.run(prm, dt, 2, ms, ps, rs, Ss, rtol=rtol)
            parts, tune_ms = b.partitions()
            for i, w in enumerate(inst):
                ms[i].copy_(T(w["m0"]))
                ps[i].zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos = b.run(prm, dt, steps, ms, ps, rs, Ss, rtol=rtol)
            torch.cuda.synchronize()
            tb = time.perf_counter() - t0
            finite = all(bool(torch.isfinite(x).all()) for x in ms)
            del ms, ps
            mc = [T(w["m0"]) for w in inst]
            pc = [torch.zeros_like(x) for x in rs]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.run(prm, dt, check_steps, mc, pc, rs, Ss, rtol=rtol)
            torch.cuda.synchronize()
            tbc = time.perf_counter() - t0
        ms2 = [T(w["m0"]) for w in inst]
        ps2 = [torch.zeros_like(x) for x in rs]
        gs = [NF.Grid(w["n"], dtype=dt_) for w in inst]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, g in enumerate(gs):
            g.run(*prm[i], dt, check_steps, ms2[i], ps2[i], rs[i], Ss[i], rtol=rtol)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        for g in gs:
            g.close()
        # the tile variants the tuner chose for each grid shape (a handle of an
        # already tuned shape reads them from the process-wide choice)
        variants = {}
        for N_, _ in (mix or W.ENSEMBLE_MIX):
            with NF.Grid((N_, N_), dtype=dt_) as gq:
                variants["%d^2" % N_] = gq.tuning()
        progress("ensemble %s: batch %.3g grid-point-steps/s" % (name, npts * steps / tb))
        out[name] = {
            "batch_grid_point_steps_per_s": npts * steps / tb,
            "batch_steps": steps,
            "finite": finite,
            "pcg_iters_per_solve": sum(i.total_cg_iters for i in infos) / (len(inst) * steps),
            "first_steps_batch_grid_point_steps_per_s": npts * check_steps / tbc,
            "first_steps_one_by_one_grid_point_steps_per_s": npts * check_steps / ts,
            "first_steps_batch_speedup": ts / tbc,
            "first_steps_bitwise_equal_to_one_by_one": all(torch.equal(a, c) for a, c in zip(mc, ms2)),
            "partitions": parts,
            "tuning_ms_two_steps_by_partition_count": [round(t, 2) for t in tune_ms],
            "tile_variants": variants,
        }
        del mc, pc, ms2, ps2
        torch.cuda.empty_cache()
    return out


def profile_case(spec):
    """N:form:steps:ndim -- run `steps` time steps of the dipole case (gamma
    0.75, rtol 1e-10) at N^ndim with form f64 or f32r through nf_step, for
    kernel traces of the precision form."""
    import numpy as np
    import torch

    from paper_2606_06720_amd import nf as NF
    from paper_2606_06720_amd import workloads as W

    N, form, steps, ndim = spec.split(":")
    N, steps, ndim = int(N), int(steps), int(ndim)
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    w = W.dipole_workload(N, 0.75, ndim=ndim)
    m, r, S = T(w["m0"]), T(w["r"]), T(w["S"])
    p = torch.zeros_like(r)
    with NF.Grid(w["n"], w["L"], dtype=NF.NF_F64 if form == "f64" else NF.NF_F32_REFINED) as g:
        for k in range(steps):
            _, si = g.step(w["c2"], w["D2"], w["gamma"], w["dt"], m, p, r, S, rtol=w["rtol"])
            print(json.dumps({"case": spec, "step": k, "pcg_iters": si.solve.iters}), flush=True)
    torch.cuda.synchronize()


def copy_calibration(nbytes):
    """A plain device-to-device copy of known size, for scaling HBM counters."""
    import torch

    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 5}), flush=True)


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--kernel", default="row_flux", choices=sorted(KERNEL_IDS))
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=200, help="steps of the reverse-mode cost run (0 = skip)")
    ap.add_argument("--sequential", action="store_true", help="run the instances one after another on one stream")
    ap.add_argument("--precision-steps", type=int, default=200, help="steps per form of the precision comparison (0 = skip)")
    ap.add_argument("--ensemble-steps", type=int, default=500, help="steps of the batched ensemble run (0 = skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, help="only run a copy of this many bytes")
    ap.add_argument("--profile-case", default="", help="only run N:form:steps:ndim time steps (for kernel traces)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: one GPU only (--gpus %d requested); sharding a grid or an ensemble across GPUs "
              "is not implemented" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.profile_case:
        profile_case(args.profile_case)
        return

    N = args.n
    # the CPU baseline runs first, in worker processes started before anything
    # touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(N, args.cpu_steps)
    if cpu is not None:
        progress("cpu baseline done: %.3g grid-point-steps/s on %d cores" % (cpu["value"], cpu["cores"]))

    import numpy as np
    import torch

    from paper_2606_06720_amd import nf as NF
    from paper_2606_06720_amd import workloads as W

    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    inst = []
    for gam in GAMMAS:
        w = W.dipole_workload(N, gam)
        g = NF.Grid(w["n"], w["L"])
        inst.append(dict(w=w, g=g, m0=T(w["m0"]), m=T(w["m0"]), p=torch.zeros((N, N), dtype=torch.float64, device=dev),
                         r=T(w["r"]), S=T(w["S"])))

    # The instances are independent: each runs on its own HIP stream (default
    # priority) from its own host thread, so that one instance's transform phase
    # overlaps another's memory phase on the GPU.
    for it in inst:
        it["stream"] = torch.cuda.Stream(device=dev)

    def run_one(it, steps, out, k):
        w = it["w"]
        with torch.cuda.stream(it["stream"]):
            out[k] = it["g"].run(w["c2"], w["D2"], w["gamma"], w["dt"], steps, it["m"], it["p"], it["r"], it["S"],
                                 rtol=w["rtol"], max_iter=1000)

    def run_all(steps):
        infos = [None] * len(inst)
        if args.sequential:
            for k, it in enumerate(inst):
                run_one(it, steps, infos, k)
        else:
            th = [threading.Thread(target=run_one, args=(it, steps, infos, k)) for k, it in enumerate(inst)]
            for t in th:
                t.start()
            for t in th:
                t.join()
        for k, i in enumerate(infos):
            if i is None:
                raise RuntimeError("instance %d failed" % k)
        return infos

    # the kernel's span stamps are on during the warmup too, so that their
    # first-use costs (buffer set-up, first launches) fall outside the timed
    # region; switching them on again clears the counts
    for it in inst:
        it["g"].time_kernel(KERNEL_IDS[args.kernel])
    if args.warmup > 0:
        run_all(args.warmup)
    for it in inst:
        it["m"].copy_(it["m0"])
        it["p"].zero_()
        it["g"].time_kernel(KERNEL_IDS[args.kernel])
    torch.cuda.synchronize()
    # the per-instance state copies above ran on the default stream

    t0 = time.perf_counter()
    infos = run_all(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    kms, kcount = 0.0, 0
    for it in inst:
        ms, c = it["g"].time_kernel_read()
        kms += ms
        kcount += c
        it["g"].time_kernel(-1)
    total_points = len(GAMMAS) * N * N
    value = total_points * args.steps / elapsed
    cg_iters = sum(i.total_cg_iters for i in infos)

    avg_s = (kms / 1e3) / max(kcount, 1)
    alg_bytes = KERNEL_BYTES_PER_POINT[args.kernel] * N * N
    achieved = alg_bytes / avg_s / 1e9 if kcount else None
    traffic = load_traffic(args.kernel, N)
    step_bytes = (sum(KERNEL_BYTES_PER_POINT.values()) * cg_iters + STEP_BYTES_PER_POINT * len(GAMMAS) * args.steps) * N * N
    rp_us = load_rocprof_duration(args.kernel, N) if not args.sequential else None
    roofline = {
        "bound": "hbm",
        "kernel": args.kernel,
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
        "traffic": traffic,
        "algorithmic_bytes_per_launch": alg_bytes,
        "avg_launch_us": avg_s * 1e6,
        "launches": kcount,
        "duration_source": "kernel execution span (device wall clock, first workgroup start to last end)",
        # the same kernel's working-dispatch average in the committed rocprofv3 trace of this
        # command (dispatch to completion signal, so it includes launch setup and end-of-kernel
        # release), and the fraction that duration gives
        "rocprof_avg_launch_us": rp_us,
        "frac_rocprof": (alg_bytes / (rp_us * 1e-6) / 1e9 / HBM_PEAK_GBS) if rp_us else None,
        # all passes of the timed steps: algorithmic bytes over the wall time
        "step_achieved": step_bytes / elapsed / 1e9,
        "step_frac": step_bytes / elapsed / 1e9 / HBM_PEAK_GBS,
    }
    # context: the tuner's throughput of the chosen operator-middle tile, one launch per
    # interval when three run concurrently on separate buffers (as the three streams do)
    tun = inst[0]["g"].tuning()
    if args.kernel == "row_flux" and tun.get("tuned") and tun["us"][0] > 0:
        roofline["three_stream_throughput_us"] = tun["us"][0]
        roofline["frac_three_stream_throughput"] = alg_bytes / (tun["us"][0] * 1e-6) / 1e9 / HBM_PEAK_GBS
    finite = all(torch.isfinite(it["m"]).all().item() for it in inst)

    # context: the gamma = 0.75 instance alone on one stream over the same steps
    solo = inst[1]
    solo["m"].copy_(solo["m0"])
    solo["p"].zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ws = solo["w"]
    si = solo["g"].run(ws["c2"], ws["D2"], ws["gamma"], ws["dt"], args.steps, solo["m"], solo["p"], solo["r"],
                       solo["S"], rtol=ws["rtol"], max_iter=1000)
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    single = {"gamma": ws["gamma"], "grid_point_steps_per_s": N * N * args.steps / t_solo,
              "ms_per_step": 1e3 * t_solo / args.steps, "pcg_iters_per_time_step": si.total_cg_iters / args.steps}

    out = {
        "metric": "grid-point-steps/s at 2D 1024^2 (PCG incl.)",
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "2D periodic %dx%d FP64 dipole source/sink, smooth random r, gamma in %s, dt=5e-4, "
                        "PCG rtol 1e-10; one step = one time step of each gamma instance" % (N, N, list(GAMMAS)),
            "concurrency": "sequential, one stream" if args.sequential else "one stream per instance",
            "grid": [N, N],
            "instances": len(GAMMAS),
            "grid_points_per_step": total_points,
            "pcg_iters_per_time_step": cg_iters / (len(GAMMAS) * args.steps),
            "grid_point_iters_per_s": N * N * cg_iters / elapsed,
            "finite": bool(finite),
        },
        "roofline": roofline,
        "single_instance": single,
        # tile variants of the PCG loop chosen by the tuner for the 1024^2 FP64 handles
        "tile_variants": inst[0]["g"].tuning(),
    }
    progress("headline done: %.4g grid-point-steps/s, %.3f ms per step" % (value, 1e3 * elapsed / args.steps))
    if args.adjoint_steps > 0:
        out["adjoint_cost"] = adjoint_cost(N, args.adjoint_steps)
        progress("adjoint block done")
    if args.precision_steps > 0:
        out["precision_form"] = precision_form(((N, 2), (4096, 2), (256, 3)), args.precision_steps)
        progress("precision block done")
    if args.ensemble_steps > 0:
        out["ensemble"] = ensemble_cost(args.ensemble_steps)
        progress("ensemble block done")
    if cpu is not None:
        out["cpu_baseline"] = cpu
    for it in inst:
        it["g"].close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
