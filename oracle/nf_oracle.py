"""Plain FP64 CPU oracle for one time step of the Fourier spectral scheme for the
periodic Hu-Cai network-formation system.

TEST INFRASTRUCTURE ONLY.  This module is the checker the GPU path is compared
against.  Only the test suite, the package smoke check and the benchmark's CPU
baseline leg may import or run it.  It shares no code with the HIP library or its
Python binding (no kernels, tables, helpers or pre/post-processing), and the
product path never calls it.

It is written to be read against the paper (Aceves-Sanchez, Degond,
Merino-Aceituno, Wytrzens, "A Spectral-Based Method for Network-Formation PDEs"):
every routine cites the section / equation it implements.  All arithmetic is
float64 with numpy's FFT as the transform primitive; there is no blocking,
fusion or reordering beyond what the cited definitions state.

Conventions
-----------
* grid ``n = (Nx, Ny[, Nz])``, lengths ``L = (Lx, Ly[, Lz])``; scalar fields are
  arrays of shape ``n[::-1]`` (x fastest), vector fields ``v[c]`` with c = 0 the
  x component; spatial direction c lives on array axis ``d-1-c``.
* nodes ``x_i = i L / N`` for ``i < N`` (periodic grid, Sec. 2.2).
* forward DFT ``e^{-i ...}`` unnormalised, inverse with ``1/n`` (numpy's
  convention).  Every operator below is independent of that choice.

Readings of points the paper leaves open:
* first-derivative multipliers use the discrete Fourier variable with the
  Nyquist entry set to zero (``xi_tilde``); the heat kernel keeps it;
* the discrete pressure is the minimum-norm solution: the 2^d Fourier modes whose
  first-derivative wavenumbers all vanish are projected out of S and of p;
* the CG of Sec. 2.4 is the textbook preconditioned CG with the constant-
  coefficient preconditioner built from the grid mean of K = m m^T + r I, warm
  started from the previous pressure, stopped on the recurrence residual
  ``||r_k||_2 <= rtol ||Pi S||_2``;
* activation for d = 3 replaces the 2D projector ``g_perp g_perp^T / |g|^2`` by
  ``I - g g^T / |g|^2`` (identical in 2D);
* the energy of Sec. 2.5 uses the same spectral gradient, the variable ``r``
  inside the ``||grad p||^2`` term, and ``p = p[m]`` for the same ``m``.

Pins (tests/test_oracle_pins.py; each is something other than this code)
------------------------------------------------------------------------
* wavenumbers, first_derivative_wavenumbers: hand-worked example (golden file),
  Nyquist checkerboards annihilated;
* grad, neg_div, apply_K, apply_A: exact derivatives of trigonometric modes,
  symbolic (sympy) divergence of manufactured 2D/3D solutions, adjointness,
  eigenpairs of K;
* null_mode_mask, project, assemble_A, pressure_dense: symmetry, positive
  semi-definiteness and exact nullity 2^d with the checkerboard basis;
* kbar, apply_Minv, pressure_pcg: closed-form Fourier solution for constant
  coefficients (one iteration), SVD minimum-norm solves, the energy identity,
  invariance to the preconditioner's scale, warm start and failure paths;
* activation: scipy.linalg.expm, RK4 of the ODE, special directions, semigroup;
* relaxation: closed forms at gamma = 1 and 1/2, RK4, semigroup, extinction;
* diffusion: heat-kernel decay per Fourier mode (Nyquist included), mean,
  semigroup;
* split_update: order of the sub-steps (activation before relaxation by the
  closed forms at gamma = 1/2; diffusion last by mean preservation), axis-swap
  and reflection equivariance;
* energy: single-mode closed form of the diffusion term, two-valued fields for
  the relaxation term at three gamma, constant-coefficient closed forms of both
  pressure terms, the pressure energy identity, and the gradient-flow identity
  (its directional derivative is minus the flow's right-hand side);
* dm_rel: hand-worked example (golden file) and the closed form |a - 1| / dt
  for m^k = a m^{k-1};
* run: stopping criteria, energy decrease for small dt;
* step_adjoint, run_gradient: central differences of the forward map (step_adjoint
  in 2D and 3D).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Incompatible",
    "SolveInfo",
    "RunInfo",
    "STOP_MAX_STEPS",
    "STOP_DM_BELOW_EPS",
    "STOP_ENERGY_INCREASE",
    "wavenumbers",
    "first_derivative_wavenumbers",
    "grad",
    "neg_div",
    "apply_K",
    "apply_A",
    "null_mode_mask",
    "project",
    "check_compatible",
    "kbar",
    "apply_Minv",
    "pressure_pcg",
    "pressure_dense",
    "assemble_A",
    "activation",
    "relaxation",
    "diffusion",
    "split_update",
    "step",
    "energy",
    "dm_rel",
    "run",
    "step_adjoint",
    "misfit_loss",
    "run_gradient",
]

STOP_MAX_STEPS = 0
STOP_DM_BELOW_EPS = 1
STOP_ENERGY_INCREASE = 2


class Incompatible(ValueError):
    """S violates the solvability condition int S = 0 (Sec. 1.1, below eq. m)."""


@dataclass
class SolveInfo:
    iters: int = 0
    rel_res: float = 0.0        # recurrence residual / ||Pi S||
    true_rel_res: float = 0.0   # ||Pi S - A p|| / ||Pi S||
    converged: bool = True
    history: list = field(default_factory=list)


@dataclass
class RunInfo:
    steps: int = 0
    stop_reason: int = STOP_MAX_STEPS
    last_dm: float = float("nan")
    last_energy: float = float("nan")
    total_cg_iters: int = 0
    unconverged_solves: int = 0
    energies: list = field(default_factory=list)
    dms: list = field(default_factory=list)


# ---------------------------------------------------------------------------------
# Discrete Fourier variables (Sec. 2.3.3, definition of xi_hat)
# ---------------------------------------------------------------------------------

def wavenumbers(N, L):
    """xi_hat(l) = 2 pi l / L for 0 <= l <= N/2 and 2 pi (l - N) / L for N/2 < l < N."""
    ell = np.arange(N, dtype=np.float64)
    return np.where(ell <= N / 2, 2.0 * np.pi * ell / L, 2.0 * np.pi * (ell - N) / L)


def first_derivative_wavenumbers(N, L):
    """xi_hat with the Nyquist entry (l = N/2, N even) set to zero.

    A first derivative of a real periodic grid function must map it to a real
    grid function; keeping +pi N / L at the Nyquist index would add a purely
    imaginary component.  Zeroing it equals taking the real part of the complex
    inverse transform.
    """
    xi = wavenumbers(N, L).copy()
    if N % 2 == 0:
        xi[N // 2] = 0.0
    return xi


def _dims(f_shape):
    return len(f_shape)


def _xi_along(c, shape, L, tilde):
    """Wavenumber array for direction c broadcast over a field of ``shape``."""
    d = len(shape)
    axis = d - 1 - c
    N = shape[axis]
    xi = first_derivative_wavenumbers(N, L[c]) if tilde else wavenumbers(N, L[c])
    bshape = [1] * d
    bshape[axis] = N
    return xi.reshape(bshape)


def _L(L, d):
    if np.isscalar(L):
        return (float(L),) * d
    return tuple(float(v) for v in L)


# ---------------------------------------------------------------------------------
# Spectral differential operators (Sec. 2.4, eq. p_discrete)
# ---------------------------------------------------------------------------------

def grad(f, L=1.0):
    """Spectral gradient G f: component c is Re F^-1[ i xi_tilde_c F f ]."""
    d = f.ndim
    L = _L(L, d)
    fh = np.fft.fftn(f)
    out = np.empty((d,) + f.shape)
    for c in range(d):
        out[c] = np.fft.ifftn(1j * _xi_along(c, f.shape, L, True) * fh).real
    return out


def neg_div(v, L=1.0):
    """-div_h v = -Re F^-1[ i xi_tilde . F v ]  (the transpose G^T of ``grad``)."""
    d = v.shape[0]
    L = _L(L, d)
    acc = np.zeros(v.shape[1:], dtype=np.complex128)
    for c in range(d):
        acc += 1j * _xi_along(c, v.shape[1:], L, True) * np.fft.fftn(v[c])
    return -np.fft.ifftn(acc).real


def apply_K(m, r, v):
    """K v with the permeability tensor K = m (x) m + r I (eq. p): (m.v) m + r v."""
    mv = np.sum(m * v, axis=0)
    return mv[None] * m + r[None] * v


def apply_A(p, m, r, L=1.0):
    """Left-hand side of eq. p_discrete: -F^-1[i xi . F(K F^-1[i xi F p])]."""
    return neg_div(apply_K(m, r, grad(p, L)), L)


# ---------------------------------------------------------------------------------
# Null space, compatibility, preconditioner (Sec. 1.1 solvability, Sec. 2.4, Sec. 5)
# ---------------------------------------------------------------------------------

def null_mode_mask(shape, L=1.0):
    """True on the 2^d Fourier modes where every first-derivative wavenumber is 0."""
    d = len(shape)
    L = _L(L, d)
    mask = np.ones(shape, dtype=bool)
    for c in range(d):
        mask = mask & (_xi_along(c, shape, L, True) == 0.0)
    return mask


def project(f, L=1.0):
    """Pi f: remove the components of f on the discrete null space of the operator."""
    fh = np.fft.fftn(f)
    fh[null_mode_mask(f.shape, L)] = 0.0
    return np.fft.ifftn(fh).real


def check_compatible(S, tol=1e-12):
    """Discrete form of the solvability condition int S = 0."""
    if abs(np.sum(S)) > tol * np.sum(np.abs(S)):
        raise Incompatible("sum(S) = %.3e exceeds %.1e * sum|S|" % (np.sum(S), tol))


def kbar(m, r):
    """Grid mean of K = m m^T + r I, the constant-coefficient preconditioner tensor."""
    d = m.shape[0]
    K = np.empty((d, d))
    for a in range(d):
        for b in range(d):
            K[a, b] = np.mean(m[a] * m[b]) + (np.mean(r) if a == b else 0.0)
    return K


def apply_Minv(f, Kb, L=1.0):
    """Inverse of the constant-coefficient operator -div(Kbar grad): multiply by
    1 / (xi_tilde^T Kbar xi_tilde) in Fourier space, 0 on the null modes."""
    d = f.ndim
    L = _L(L, d)
    sym = np.zeros(f.shape)
    for a in range(d):
        for b in range(d):
            sym = sym + Kb[a, b] * _xi_along(a, f.shape, L, True) * _xi_along(b, f.shape, L, True)
    inv = np.zeros_like(sym)
    nz = sym != 0.0
    inv[nz] = 1.0 / sym[nz]
    return np.fft.ifftn(inv * np.fft.fftn(f)).real


# ---------------------------------------------------------------------------------
# Pressure solve (Sec. 2.4): CG on eq. p_discrete, warm started from p^k
# ---------------------------------------------------------------------------------

def pressure_pcg(m, r, S, p0=None, rtol=1e-10, max_iter=1000, L=1.0, check=True,
                 precond_scale=1.0, keep_history=False):
    """Textbook preconditioned CG for A p = Pi S (A from eq. p_discrete).

    Returns (p, SolveInfo).  p is the minimum-norm solution (Pi p = p) to the
    tolerance.  ``precond_scale`` multiplies Kbar (a test hook: CG iterates do not
    depend on the preconditioner's scale).
    """
    d = m.shape[0]
    L = _L(L, d)
    if check:
        check_compatible(S)
    b = project(S, L)
    bnorm = math.sqrt(float(np.vdot(b, b)))
    info = SolveInfo()
    if bnorm == 0.0:
        info.true_rel_res = 0.0
        return np.zeros_like(S), info
    x = np.zeros_like(S) if p0 is None else project(np.asarray(p0, dtype=np.float64), L)
    Kb = precond_scale * kbar(m, r)
    res = b - apply_A(x, m, r, L)
    z = apply_Minv(res, Kb, L)
    dvec = z.copy()
    rho = float(np.vdot(res, z))
    rnorm = math.sqrt(float(np.vdot(res, res)))
    it = 0
    if keep_history:
        info.history.append(rnorm / bnorm)
    while rnorm > rtol * bnorm and it < max_iter:
        q = apply_A(dvec, m, r, L)
        alpha = rho / float(np.vdot(dvec, q))
        x = x + alpha * dvec
        res = res - alpha * q
        it += 1
        rnorm = math.sqrt(float(np.vdot(res, res)))
        if keep_history:
            info.history.append(rnorm / bnorm)
        if rnorm <= rtol * bnorm:
            break
        z = apply_Minv(res, Kb, L)
        rho_new = float(np.vdot(res, z))
        beta = rho_new / rho
        dvec = z + beta * dvec
        rho = rho_new
    info.iters = it
    info.rel_res = rnorm / bnorm
    info.converged = rnorm <= rtol * bnorm
    tr = b - apply_A(x, m, r, L)
    info.true_rel_res = math.sqrt(float(np.vdot(tr, tr))) / bnorm
    return x, info


def assemble_A(m, r, L=1.0):
    """Dense matrix of eq. p_discrete's operator, column j = A e_j (tiny grids only)."""
    shape = m.shape[1:]
    n = int(np.prod(shape))
    A = np.empty((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        A[:, j] = apply_A(e.reshape(shape), m, r, L).ravel()
    return A


def pressure_dense(m, r, S, L=1.0):
    """Minimum-norm least-squares solution of A p = Pi S with a dense SVD solve."""
    d = m.shape[0]
    L = _L(L, d)
    check_compatible(S)
    A = assemble_A(m, r, L)
    b = project(S, L).ravel()
    p, *_ = np.linalg.lstsq(A, b, rcond=1e-10)
    return p.reshape(S.shape)


# ---------------------------------------------------------------------------------
# Splitting for the conductivity equation (Sec. 2.3)
# ---------------------------------------------------------------------------------

def activation(m, g, c2, dt):
    """Exact activation sub-step, eq. m_activation_discrete.

    m <- |g|^-2 [ g_perp g_perp^T + g g^T exp(c^2 |g|^2 dt) ] m, and m unchanged
    where |g|^2 = 0.  In 3D the projector g_perp g_perp^T is |g|^2 I - g g^T.
    """
    d = m.shape[0]
    g2 = np.sum(g * g, axis=0)
    gm = np.sum(g * m, axis=0)
    E = np.exp(c2 * g2 * dt)
    if d == 2:
        gperp = np.stack([-g[1], g[0]])
        gpm = np.sum(gperp * m, axis=0)
        num = gperp * gpm[None] + g * (gm * E)[None]
    else:
        num = g2[None] * m - g * gm[None] + g * (gm * E)[None]
    with np.errstate(invalid="ignore", divide="ignore"):
        out = num / g2[None]
    return np.where((g2 == 0.0)[None], m, out)


def relaxation(m, gamma, dt):
    """Exact relaxation sub-step, eq. m_relaxation_discrete.

    gamma = 1: m e^{-dt}; else m unchanged where |m| = 0; else
    a = m/|m| (|m|^{2(1-gamma)} - 2(1-gamma) dt)^{1/(2(1-gamma))} kept where
    b = |m|^{2(1-gamma)} - 2(1-gamma) dt >= 0 and 0 where b < 0.
    """
    if gamma == 1.0:
        return m * math.exp(-dt)
    s = np.sqrt(np.sum(m * m, axis=0))
    e = 1.0 - gamma
    with np.errstate(invalid="ignore", divide="ignore"):
        b = s ** (2.0 * e) - 2.0 * e * dt
        a = (m / s[None]) * (np.maximum(b, 0.0) ** (1.0 / (2.0 * e)))[None]
    out = np.where((b >= 0.0)[None], a, 0.0)
    return np.where((s == 0.0)[None], m, out)


def diffusion(m, D2, dt, L=1.0):
    """Exact diffusion sub-step, eq. diffusion_space_discrete, per component:
    m_c <- F^-1[ exp(-D^2 |xi_hat|^2 dt) F m_c ]."""
    d = m.shape[0]
    L = _L(L, d)
    shape = m.shape[1:]
    xi2 = np.zeros(shape)
    for c in range(d):
        xi2 = xi2 + _xi_along(c, shape, L, False) ** 2
    H = np.exp(-D2 * xi2 * dt)
    out = np.empty_like(m)
    for c in range(d):
        out[c] = np.fft.ifftn(H * np.fft.fftn(m[c])).real
    return out


def split_update(m, p, c2, D2, gamma, dt, L=1.0):
    """Step 2 of Algorithm 1: activation with grad p, then relaxation, then diffusion."""
    g = grad(p, L)
    m1 = activation(m, g, c2, dt)
    m2 = relaxation(m1, gamma, dt)
    return diffusion(m2, D2, dt, L)


def step(m, p, r, S, c2, D2, gamma, dt, rtol=1e-10, max_iter=1000, L=1.0):
    """One pass of the time loop of Algorithm 1.

    Step 1 solves p = p[m^k] (warm start from the given p), Step 2 applies the
    split update.  Returns (m^{k+1}, p[m^k], SolveInfo).
    """
    p_new, info = pressure_pcg(m, r, S, p, rtol, max_iter, L)
    return split_update(m, p_new, c2, D2, gamma, dt, L), p_new, info


# ---------------------------------------------------------------------------------
# Stopping criteria and energy (Sec. 2.5)
# ---------------------------------------------------------------------------------

def energy(m, p, r, c2, D2, gamma, L=1.0):
    """Discrete energy E_h of Sec. 2.5 (eq. energy discretised on the grid).

    Returns (total, D^2/2 ||grad m||^2, ||  |m|^gamma ||^2/(2 gamma),
             c^2/2 ||m . grad p||^2, c^2/2 sum r |grad p|^2), each with the
    discrete L2 norm ||f||^2 = h_1...h_d sum f^2.  p must be p[m].
    """
    d = m.shape[0]
    L = _L(L, d)
    shape = m.shape[1:]
    hvol = 1.0
    for c in range(d):
        hvol *= L[c] / shape[d - 1 - c]
    gm2 = 0.0
    for c in range(d):
        gmc = grad(m[c], L)
        gm2 += float(np.sum(gmc * gmc))
    gp = grad(p, L)
    e_diff = 0.5 * D2 * hvol * gm2
    mabs = np.sqrt(np.sum(m * m, axis=0))
    e_relax = hvol * float(np.sum(mabs ** (2.0 * gamma))) / (2.0 * gamma)
    mgp = np.sum(m * gp, axis=0)
    e_act = 0.5 * c2 * hvol * float(np.sum(mgp * mgp))
    e_flow = 0.5 * c2 * hvol * float(np.sum(r * np.sum(gp * gp, axis=0)))
    total = e_diff + e_relax + e_act + e_flow
    return (total, e_diff, e_relax, e_act, e_flow)


def dm_rel(m_new, m_old, dt):
    """Delta m^k = ||m^k - m^{k-1}||_2 / (dt ||m^{k-1}||_2) (Sec. 2.5)."""
    num = math.sqrt(float(np.sum((m_new - m_old) ** 2)))
    den = math.sqrt(float(np.sum(m_old ** 2)))
    if den == 0.0:
        return 0.0 if num == 0.0 else math.inf
    return num / (dt * den)


def run(m0, p0, r, S, c2, D2, gamma, dt, max_steps, eps_dm=0.0, stop_on_energy=False,
        rtol=1e-10, max_iter=1000, L=1.0):
    """Time loop of Algorithm 1 with its two stopping criteria (Sec. 2.5).

    p[m^0] is solved first; each pass then applies the split update to m^k with
    p[m^k] and solves p[m^{k+1}] (warm start).  After each pass it stops if
    E_h(m^{k+1}) >= E_h(m^k) (when enabled) or Delta m <= eps_dm.  At least one
    pass is taken.  A solve that reaches max_iter does not stop the run (its
    last iterate is used and counted).  Returns (m_final, p[m_final], RunInfo).
    """
    m = np.array(m0, dtype=np.float64, copy=True)
    p, info = pressure_pcg(m, r, S, p0, rtol, max_iter, L)
    ri = RunInfo(total_cg_iters=info.iters, unconverged_solves=int(not info.converged))
    e_prev = energy(m, p, r, c2, D2, gamma, L)[0] if stop_on_energy else None
    if stop_on_energy:
        ri.energies.append(e_prev)
    while ri.steps < max_steps:
        m_new = split_update(m, p, c2, D2, gamma, dt, L)
        p, info = pressure_pcg(m_new, r, S, p, rtol, max_iter, L)
        ri.total_cg_iters += info.iters
        ri.unconverged_solves += int(not info.converged)
        dm = dm_rel(m_new, m, dt)
        m = m_new
        ri.steps += 1
        ri.last_dm = dm
        ri.dms.append(dm)
        if stop_on_energy:
            e = energy(m, p, r, c2, D2, gamma, L)[0]
            ri.energies.append(e)
            ri.last_energy = e
            if e >= e_prev:
                ri.stop_reason = STOP_ENERGY_INCREASE
                break
            e_prev = e
        if dm <= eps_dm:
            ri.stop_reason = STOP_DM_BELOW_EPS
            break
    return m, p, ri


# ---------------------------------------------------------------------------------
# Discrete adjoint of one time step (reverse mode of the step above)
# ---------------------------------------------------------------------------------
#
# The step maps (m, r, S) to m' = H Rel(Act(m, G p)), p = A(m, r)^+ Pi S.  Given
# lam = dL/dm', the adjoint returns dL/dm, dL/dr, dL/dS.  Each stage below is the
# transpose of the corresponding forward stage, written out from its formula:
#   diffusion H = F^-1 diag(h) F is real symmetric, so H^T = H;
#   relaxation m** = rho(s) m*/s has Jacobian (rho/s)(I - u u^T) + rho' u u^T;
#   activation m* = m + kappa(z) (g.m) g, kappa = c2 dt phi1(z), z = c2 dt |g|^2;
#   g = G p has transpose G^T = neg_div;
#   the pressure satisfies A p = Pi S with A = G^T K G, K = m m^T + r I, so for
#   lam_p = dL/dp the adjoint pressure mu solves A mu = Pi lam_p and
#   dL/dS = Pi mu, dL/dr = -(G mu . G p), dL/dm gains -[(m.Gp) G mu + (m.G mu) G p].

def _relaxation_jacobian_apply(mstar, lam, gamma, dt):
    """J^T lam for the relaxation map at m* (J is symmetric)."""
    if gamma == 1.0:
        return lam * math.exp(-dt)
    s = np.sqrt(np.sum(mstar * mstar, axis=0))
    e = 1.0 - gamma
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        b = s ** (2.0 * e) - 2.0 * e * dt
        rho = np.maximum(b, 0.0) ** (1.0 / (2.0 * e))
        drho = (s / rho) ** (2.0 * e - 1.0)          # d rho / d s where b > 0
        u = mstar / s[None]
        ul = np.sum(u * lam, axis=0)
        out = (rho / s)[None] * (lam - u * ul[None]) + (drho * ul)[None] * u
    alive = (b > 0.0) & (s > 0.0)
    out = np.where(alive[None], out, 0.0)
    # at |m*| = 0 the map is the identity for gamma > 1 (s^{-2e} -> 0) and
    # extinct for gamma < 1
    if gamma > 1.0:
        out = np.where((s == 0.0)[None], lam, out)
    return out


def _phi1(z):
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(z == 0.0, 1.0, np.expm1(z) / np.where(z == 0.0, 1.0, z))


def _dphi1(z):
    """phi1'(z) = (e^z (z - 1) + 1) / z^2, by its Taylor series near 0."""
    zs = np.where(np.abs(z) < 1e-3, 0.0, z)
    with np.errstate(invalid="ignore", divide="ignore"):
        closed = (np.expm1(zs) * (zs - 1.0) + zs) / np.where(zs == 0.0, 1.0, zs * zs)
    series = 0.5 + z / 3.0 + z * z / 8.0 + z ** 3 / 30.0
    return np.where(np.abs(z) < 1e-3, series, closed)


def step_adjoint(m, p, r, S, c2, D2, gamma, dt, lam_next, rtol=1e-12, max_iter=2000, L=1.0, mu0=None):
    """Reverse of ``step``: given m = m^k, p = p[m^k] and lam = dL/dm^{k+1},
    return (dL/dm^k, dL/dr, dL/dS, mu, SolveInfo) for this step alone."""
    d = m.shape[0]
    L = _L(L, d)
    g = grad(p, L)
    # forward intermediates
    g2 = np.sum(g * g, axis=0)
    z = c2 * dt * g2
    kappa = c2 * dt * _phi1(z)
    gm = np.sum(g * m, axis=0)
    mstar = m + (kappa * gm)[None] * g
    # diffusion (symmetric)
    lam2 = diffusion(lam_next, D2, dt, L)
    # relaxation
    lam1 = _relaxation_jacobian_apply(mstar, lam2, gamma, dt)
    # activation: w.r.t. m and w.r.t. g
    gl = np.sum(g * lam1, axis=0)
    lam_m = lam1 + (kappa * gl)[None] * g
    dkappa = c2 * dt * _dphi1(z)
    lam_g = (2.0 * c2 * dt * dkappa * gm * gl)[None] * g + (kappa * gl)[None] * m + (kappa * gm)[None] * lam1
    # g = G p
    lam_p = neg_div(lam_g, L)
    # adjoint pressure: A mu = Pi lam_p (A symmetric); S = 0 trick: solve with lam_p as source
    mu, info = pressure_pcg(m, r, project(lam_p, L), mu0, rtol, max_iter, L, check=False)
    gmu = grad(mu, L)
    dS = project(mu, L)
    dr = -np.sum(gmu * g, axis=0)
    mg = np.sum(m * g, axis=0)
    mgmu = np.sum(m * gmu, axis=0)
    lam_k = lam_m - (mg[None] * gmu + mgmu[None] * g)
    return lam_k, dr, dS, mu, info


def misfit_loss(m, m_target):
    """L = 1/2 sum (|m| - |m_target|)^2 and dL/dm (zero where |m| = 0)."""
    a = np.sqrt(np.sum(m * m, axis=0))
    at = np.sqrt(np.sum(m_target * m_target, axis=0))
    diff = a - at
    with np.errstate(invalid="ignore", divide="ignore"):
        lam = np.where((a > 0.0)[None], (diff / a)[None] * m, 0.0)
    return 0.5 * float(np.sum(diff * diff)), lam


def run_gradient(m0, r, S, c2, D2, gamma, dt, steps, m_target, rtol=1e-12, max_iter=2000, L=1.0):
    """Loss of the final state after `steps` time steps (Algorithm 1 without the
    stopping tests) and its gradients w.r.t. r and S, by storing every state and
    sweeping the step adjoints backwards.  Returns (loss, dL/dr, dL/dS)."""
    ms, ps = [], []
    m = np.array(m0, dtype=np.float64, copy=True)
    p = None
    for _ in range(steps):
        p, _ = pressure_pcg(m, r, S, p, rtol, max_iter, L)
        ms.append(m)
        ps.append(p)
        m = split_update(m, p, c2, D2, gamma, dt, L)
    loss, lam = misfit_loss(m, m_target)
    gr = np.zeros_like(r)
    gS = np.zeros_like(S)
    mu = None
    for k in range(steps - 1, -1, -1):
        lam, dr, dS, mu, _ = step_adjoint(ms[k], ps[k], r, S, c2, D2, gamma, dt, lam, rtol, max_iter, L, mu)
        gr += dr
        gS += dS
    return loss, gr, gS
