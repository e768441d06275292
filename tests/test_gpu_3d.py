"""GPU parity of the 3D path (ndim = 3 handles): transforms against numpy,
operator apply, pressure solves, time steps and runs against the CPU oracle
(FP64 bar 1e-10 relative L2), the discrete energy of Sec. 2.5 and the run's
energy stopping against the oracle, the mixed-precision form against the
oracle and against the FP64 form at 256^3, and the 3D error paths."""

import numpy as np
import pytest

import oracle as O
from paper_2606_06720_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

TOL = 1e-10


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2606_06720_amd import nf as NF

    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    Z = lambda shape: torch.zeros(shape, dtype=torch.float64, device=dev)
    return NF, T, Z, torch


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def rand_fields(n, seed):
    rng = np.random.default_rng(seed)
    shape = n[::-1]
    m = rng.uniform(-1.0, 1.0, (3,) + shape)
    r = rng.uniform(0.05, 0.15, shape)
    S = rng.standard_normal(shape)
    S -= S.mean()
    return m, r, S


def packed(F, nx):
    """numpy fftn of f[z][y][x] (F[kz][ky][kx]) -> packed [kx][ky][kz] with
    slot 0 = F(kx=0) + i F(kx=Nx/2)."""
    H = nx // 2
    P = np.transpose(F[:, :, :H], (2, 1, 0)).copy()
    P[0] = F[:, :, 0].T + 1j * F[:, :, H].T
    return np.stack([P.real, P.imag], axis=-1)


@pytest.mark.parametrize("n", [(8, 8, 8), (16, 8, 32), (32, 16, 8), (64, 64, 64), (8, 128, 16)])
def test_transforms_match_numpy(env, n):
    NF, T, Z, torch = env
    f = np.random.default_rng(3).standard_normal(n[::-1])
    want = packed(np.fft.fftn(f), n[0])
    with NF.Grid(n) as g:
        out = Z(g.spec_shape)
        g.transform_forward(T(f), out)
        back = Z(n[::-1])
        g.transform_inverse(out, back)
    assert rel(out.cpu().numpy(), want) <= 1e-13
    assert rel(back.cpu().numpy(), f) <= 1e-13


@pytest.mark.parametrize("n,L", [((8, 8, 8), (1.0, 1.0, 1.0)), ((16, 32, 8), (2.0, 0.5, 1.5))])
def test_operator_apply_matches_oracle(env, n, L):
    NF, T, Z, torch = env
    m, r, S = rand_fields(n, 5)
    p = np.random.default_rng(6).standard_normal(n[::-1])
    want = O.apply_A(p, m, r, L)
    with NF.Grid(n, L) as g:
        out = Z(n[::-1])
        g.apply_operator(T(m), T(r), T(p), out)
    assert rel(out.cpu().numpy(), want) <= 1e-12


@pytest.mark.parametrize("n,rtol", [((8, 8, 8), 1e-12), ((16, 16, 16), 1e-12), ((32, 16, 8), 1e-10),
                                    ((8, 32, 64), 1e-12)])
def test_pressure_solve_matches_oracle(env, n, rtol):
    NF, T, Z, torch = env
    m, r, S = rand_fields(n, 7)
    p_or, info_or = O.pressure_pcg(m, r, S, None, rtol, 3000)
    with NF.Grid(n) as g:
        p = Z(n[::-1])
        rc, info = g.pressure_solve(T(m), T(r), T(S), p, rtol=rtol, max_iter=3000)
    assert info.converged and abs(info.iters - info_or.iters) <= 1
    assert rel(p.cpu().numpy(), p_or) <= TOL
    assert info.true_rel_res <= 2 * rtol
    assert abs(p.cpu().numpy().mean()) <= 1e-14 * np.abs(p_or).max()


def test_pressure_constant_coefficients_closed_form(env):
    NF, T, Z, torch = env
    n = (16, 32, 8)
    X, Y, Zc = W.grid_coords(n, 1.0)
    mc, rc_ = np.array([0.6, 0.3, -0.4]), 0.15
    K = np.outer(mc, mc) + rc_ * np.eye(3)
    S = np.zeros_like(X)
    p_want = np.zeros_like(X)
    for k, a in (((3, 1, 2), 1.0), ((-2, 5, 1), 0.4), ((6, -7, 3), 0.1)):
        arg = 2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Zc)
        S += a * np.cos(arg)
        p_want += a * np.cos(arg) / (4 * np.pi ** 2 * (np.array(k) @ K @ np.array(k)))
    m = np.broadcast_to(mc[:, None, None, None], (3,) + X.shape).copy()
    with NF.Grid(n) as g:
        p = Z(n[::-1])
        rc, info = g.pressure_solve(T(m), T(np.full(X.shape, rc_)), T(S), p, rtol=1e-12)
    assert info.iters == 1
    assert rel(p.cpu().numpy(), p_want) <= 1e-13


@pytest.mark.parametrize("gamma", [0.5, 0.75, 1.0])
def test_dipole_steps_match_oracle_32(env, gamma):
    NF, T, Z, torch = env
    w = W.dipole_workload(32, gamma, ndim=3)
    m, p, r, S = T(w["m0"]), Z(w["r"].shape), T(w["r"]), T(w["S"])
    mo, po = w["m0"], None
    with NF.Grid(w["n"], w["L"]) as g:
        for _ in range(3):
            rc, si = g.step(w["c2"], w["D2"], w["gamma"], w["dt"], m, p, r, S, rtol=w["rtol"])
            mo, po, io = O.step(mo, po, w["r"], w["S"], w["c2"], w["D2"], w["gamma"], w["dt"], w["rtol"])
            assert abs(si.solve.iters - io.iters) <= 1
            assert rel(p.cpu().numpy(), po) <= TOL
            assert rel(m.cpu().numpy(), mo) <= TOL


def test_bump_run_matches_oracle_16(env):
    NF, T, Z, torch = env
    w = W.bump_workload(16, ndim=3)
    m, p, r, S = T(w["m0"]), Z(w["r"].shape), T(w["r"]), T(w["S"])
    with NF.Grid(w["n"], w["L"]) as g:
        ri = g.run(w["c2"], w["D2"], w["gamma"], w["dt"], 12, m, p, r, S, rtol=1e-12)
    mo, po, rio = O.run(w["m0"], None, w["r"], w["S"], w["c2"], w["D2"], w["gamma"], w["dt"], 12, rtol=1e-12)
    assert ri.steps == 12 and abs(ri.total_cg_iters - rio.total_cg_iters) <= 3
    assert rel(m.cpu().numpy(), mo) <= TOL
    assert rel(p.cpu().numpy(), po) <= TOL
    assert abs(ri.last_dm - rio.last_dm) <= 1e-9 * rio.last_dm


def test_non_cubic_box_steps_match_oracle(env):
    NF, T, Z, torch = env
    n, L = (16, 8, 32), (1.0, 0.5, 2.0)
    m, r, S = rand_fields(n, 13)
    m = np.abs(m)
    prm = dict(c2=20.0, D2=2e-3, gamma=0.8, dt=1e-3)
    mt, pt = T(m), Z(n[::-1])
    mo, po = m, None
    with NF.Grid(n, L) as g:
        for _ in range(3):
            g.step(prm["c2"], prm["D2"], prm["gamma"], prm["dt"], mt, pt, T(r), T(S), rtol=1e-11)
            mo, po, _ = O.step(mo, po, r, S, prm["c2"], prm["D2"], prm["gamma"], prm["dt"], 1e-11, L=L)
    assert rel(mt.cpu().numpy(), mo) <= TOL
    assert rel(pt.cpu().numpy(), po) <= TOL


def test_refined_solve_and_steps_match_oracle(env):
    NF, T, Z, torch = env
    w = W.dipole_workload(32, 0.75, ndim=3)
    m, p, r, S = T(w["m0"]), Z(w["r"].shape), T(w["r"]), T(w["S"])
    mo, po = w["m0"], None
    with NF.Grid(w["n"], w["L"], dtype=NF.NF_F32_REFINED) as g:
        for _ in range(3):
            rc, si = g.step(w["c2"], w["D2"], w["gamma"], w["dt"], m, p, r, S, rtol=1e-12)
            mo, po, _ = O.step(mo, po, w["r"], w["S"], w["c2"], w["D2"], w["gamma"], w["dt"], 1e-13)
            assert si.solve.converged
            assert rel(p.cpu().numpy(), po) <= TOL
            assert rel(m.cpu().numpy(), mo) <= TOL
        # at the workload's rtol the precision form's 1e-6 bar
        m2, p2 = T(w["m0"]), Z(w["r"].shape)
        g.run(w["c2"], w["D2"], w["gamma"], w["dt"], 5, m2, p2, r, S, rtol=w["rtol"])
    mo5, po5, _ = O.run(w["m0"], None, w["r"], w["S"], w["c2"], w["D2"], w["gamma"], w["dt"], 5, rtol=w["rtol"])
    em, ep = rel(m2.cpu().numpy(), mo5), rel(p2.cpu().numpy(), po5)
    print("3D 32^3 f32-refined, rtol 1e-10, 5 steps: rel err m %.2e  p %.2e" % (em, ep))
    assert em <= 1e-6 and ep <= 1e-6


def test_precision_form_256_against_fp64(env):
    # the precision case's 3D grid: 256^3, fields built as in the dipole case
    # (3D analogue), gamma 0.75; FP32-refined against the FP64 form (held to
    # the oracle above) after two steps, both at rtol 1e-12
    NF, T, Z, torch = env
    w = W.dipole_workload(256, 0.75, ndim=3)
    out = {}
    for dt_ in (NF.NF_F64, NF.NF_F32_REFINED):
        m, p, r, S = T(w["m0"]), Z(w["r"].shape), T(w["r"]), T(w["S"])
        with NF.Grid(w["n"], w["L"], dtype=dt_) as g:
            for _ in range(2):
                rc, si = g.step(w["c2"], w["D2"], w["gamma"], w["dt"], m, p, r, S, rtol=1e-12)
                assert si.solve.converged
            out[dt_] = (m.cpu().numpy(), p.cpu().numpy())
        del m, p, r, S
        torch.cuda.empty_cache()
    em = rel(out[NF.NF_F32_REFINED][0], out[NF.NF_F64][0])
    ep = rel(out[NF.NF_F32_REFINED][1], out[NF.NF_F64][1])
    print("256^3 f32-refined vs f64 after 2 steps: rel diff m %.2e  p %.2e" % (em, ep))
    assert em <= TOL and ep <= TOL


def test_3d_error_paths(env):
    NF, T, Z, torch = env
    n = (16, 16, 8)
    m, r, S = rand_fields(n, 11)
    with NF.Grid(n) as g:
        p = Z(n[::-1])
        with pytest.raises(NF.NfError) as e:
            g.pressure_solve(T(m), T(r), T(S + 1e-3), p)
        assert e.value.code == NF.NF_EINCOMPAT
        rc, info = g.pressure_solve(T(m), T(r), T(S), p, rtol=1e-10, max_iter=1, allow_notconv=True)
        assert rc == NF.NF_ENOTCONV and info.iters == 1 and not info.converged
        _, info_or = O.pressure_pcg(m, r, S, None, 1e-10, 1)
        assert abs(info.rel_res - info_or.rel_res) <= 1e-12 * info_or.rel_res
        with pytest.raises(NF.NfError) as e:
            lam = Z((3,) + n[::-1])
            g.step_adjoint(1.0, 1e-3, 0.75, -1e-3, T(m), p, T(r), T(S), lam, Z((3,) + n[::-1]), Z(n[::-1]),
                           Z(n[::-1]), Z(n[::-1]))
        assert e.value.code == NF.NF_EINVAL
        with pytest.raises(NF.NfError) as e:
            g.step(1e6, 1e-3, 0.75, 1.0, T(m), Z(n[::-1]), T(r), T(1e3 * S))
        assert e.value.code == NF.NF_ENONFINITE
        rc, info = g.pressure_solve(T(m), T(r), T(S), p, rtol=1e-10)
        assert info.converged
    with pytest.raises(NF.NfError) as e:
        NF.Grid((16, 16, 2048))
    assert e.value.code == NF.NF_EINVAL


@pytest.mark.parametrize("n,L", [((16, 32, 8), (1.0, 2.0, 0.5)), ((32, 32, 32), (1.0, 1.0, 1.0))])
def test_energy_matches_oracle_3d(env, n, L):
    NF, T, Z, torch = env
    m, r, S = rand_fields(n, 23)
    prm = (12.0, 3e-3, 0.7)
    p_or, _ = O.pressure_pcg(m, r, S, None, 1e-13, 4000, L)
    want = O.energy(m, p_or, r, *prm, L)
    for dtype in (NF.NF_F64, NF.NF_F32_REFINED):
        with NF.Grid(n, L, dtype=dtype) as g:
            e_given = g.energy(*prm, T(m), T(r), T(S), p=T(p_or))
            e_solve = g.energy(*prm, T(m), T(r), T(S))
        for got in (e_given, e_solve):
            for a, b in zip(got, want):
                assert abs(a - b) <= 1e-11 * abs(want[0])


def test_energy_stopping_run_matches_oracle_3d(env):
    NF, T, Z, torch = env
    w = W.bump_workload(16, ndim=3)
    m, p, r, S = T(w["m0"]), Z(w["r"].shape), T(w["r"]), T(w["S"])
    with NF.Grid(w["n"], w["L"]) as g:
        ri = g.run(w["c2"], w["D2"], w["gamma"], w["dt"], 6, m, p, r, S, stop_on_energy_increase=True, rtol=1e-12,
                   max_iter=4000)
    mo, po, rio = O.run(w["m0"], None, w["r"], w["S"], w["c2"], w["D2"], w["gamma"], w["dt"], 6, stop_on_energy=True,
                        rtol=1e-12, max_iter=4000)
    assert ri.steps == rio.steps == 6 and ri.stop_reason == NF.NF_STOP_MAX_STEPS == rio.stop_reason
    assert ri.last_energy < ri.prev_energy
    assert abs(ri.last_energy - rio.energies[-1]) <= 1e-10 * abs(rio.energies[-1])
    assert abs(ri.prev_energy - rio.energies[-2]) <= 1e-10 * abs(rio.energies[-2])
    assert rel(m.cpu().numpy(), mo) <= TOL
    assert rel(p.cpu().numpy(), po) <= TOL
    # a step that raises the energy stops the run (a large activation step)
    with NF.Grid(w["n"], w["L"]) as g:
        m2, p2 = T(w["m0"]), Z(w["r"].shape)
        ri = g.run(100.0, 1e-4, 0.75, 0.05, 10, m2, p2, r, T(14 * w["S"]), stop_on_energy_increase=True)
    _, _, rio = O.run(w["m0"], None, w["r"], 14 * w["S"], 100.0, 1e-4, 0.75, 0.05, 10, stop_on_energy=True)
    assert rio.unconverged_solves == 0 and ri.unconverged_solves == 0
    assert ri.stop_reason == NF.NF_STOP_ENERGY_INCREASE == rio.stop_reason
    assert ri.steps == rio.steps == 1
    assert abs(ri.last_energy - rio.energies[-1]) <= 1e-9 * abs(rio.energies[-1])


def test_step_energy_3d_matches_oracle(env):
    """nf_step on a 3D handle with the step energy on: E_h(m^k) with p[m^k]."""
    NF, T, Z, torch = env
    n, L = (16, 8, 32), (1.0, 0.5, 2.0)
    m, r, S = rand_fields(n, 29)
    c2, D2, gamma, dt = 12.0, 3e-3, 0.7, 2e-3
    mo = m.copy()
    with NF.Grid(n, L) as g:
        g.set_step_energy(True)
        mg, pg = T(m), Z(n[::-1])
        for k in range(2):
            _, si = g.step(c2, D2, gamma, dt, mg, pg, T(r), T(S), rtol=1e-12, max_iter=4000)
            p_k, _ = O.pressure_pcg(mo, r, S, None, 1e-13, 4000, L)
            want = O.energy(mo, p_k, r, c2, D2, gamma, L)[0]
            assert si.energy_valid and abs(si.energy - want) <= 1e-10 * abs(want), (k, si.energy, want)
            mo, _, _ = O.step(mo, p_k, r, S, c2, D2, gamma, dt, 1e-12, 4000, L)


@pytest.mark.parametrize("gamma", [0.75, 1.0, 1.25])
def test_step_adjoint_3d_matches_oracle(env, gamma):
    """nf_step_adjoint on a 3D handle (non-cubic grid and box) against the
    oracle's adjoint of one step, which is written for any dimension."""
    NF, T, Z, torch = env
    n, L = (16, 8, 32), (1.0, 0.5, 2.0)
    rng = np.random.default_rng(67)
    sh = n[::-1]
    m = rng.uniform(0.2, 1.0, (3,) + sh)
    r = rng.uniform(0.05, 0.15, sh)
    S = rng.standard_normal(sh)
    S -= S.mean()
    lam = rng.standard_normal((3,) + sh)
    c2, D2, dt = 30.0, 2e-3, 2e-3
    p, _ = O.pressure_pcg(m, r, S, None, 1e-13, 4000, L)
    lk, dr, dS, mu, _ = O.step_adjoint(m, p, r, S, c2, D2, gamma, dt, lam, rtol=1e-13, max_iter=4000, L=L)
    with NF.Grid(n, L) as g:
        lam_k = Z((3,) + sh)
        gr = torch.full(sh, 0.5, dtype=torch.float64, device="cuda:0")   # accumulated into
        gS, mug = Z(sh), Z(sh)
        rc, info = g.step_adjoint(c2, D2, gamma, dt, T(m), T(p), T(r), T(S), T(lam), lam_k, gr, gS, mug,
                                  rtol=1e-13, max_iter=4000)
    assert info.converged
    assert rel(lam_k.cpu().numpy(), lk) <= 1e-9
    assert rel(gr.cpu().numpy() - 0.5, dr) <= 1e-9
    assert rel(gS.cpu().numpy(), dS) <= 1e-9
    assert rel(mug.cpu().numpy(), mu) <= 1e-9


def test_checkpointed_gradient_3d_matches_oracle(env):
    """The checkpointed reverse sweep (adjoint.run_gradient) on a 3D handle
    against the oracle's stored-state sweep."""
    from paper_2606_06720_amd import adjoint as A

    NF, T, Z, torch = env
    w = W.bump_workload(16, ndim=3)
    prm = (w["c2"], w["D2"], w["gamma"])
    steps = 5
    m_tgt = O.run(w["m0"], None, w["r"] * 1.5, 1.2 * w["S"], *prm, w["dt"], max_steps=steps, rtol=1e-13,
                  max_iter=4000, L=w["L"])[0]
    l_or, gr_or, gS_or = O.run_gradient(w["m0"], w["r"], w["S"], *prm, w["dt"], steps, m_tgt, rtol=1e-13,
                                        max_iter=4000, L=w["L"])
    with NF.Grid(w["n"], w["L"]) as g:
        loss, gr, gS = A.run_gradient(g, prm, w["dt"], steps, T(w["m0"]), T(w["r"]), T(w["S"]), T(m_tgt),
                                      rtol=1e-13, max_iter=4000, stride=2)
    assert abs(loss - l_or) <= 1e-8 * l_or
    assert rel(gr.cpu().numpy(), gr_or) <= 1e-7
    assert rel(gS.cpu().numpy(), gS_or) <= 1e-7
