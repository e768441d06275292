"""Seeded synthetic inputs shaped like the paper's workloads.

This module only *builds input fields* (the background permeability ``r``, the
source/sink term ``S`` and the initial conductivity ``m0``).  It contains none of
the numerical method's arithmetic, so both the GPU path and the CPU checker can
consume the same arrays without sharing any solver code.

Array conventions (shared by every consumer):

* grid sizes are given as ``n = (Nx, Ny)`` or ``(Nx, Ny, Nz)`` and domain lengths
  as ``L = (Lx, Ly[, Lz])``;
* scalar fields are C-contiguous ``float64`` arrays of shape ``n[::-1]``
  (``[y][x]`` in 2D, ``[z][y][x]`` in 3D, x fastest);
* vector fields are ``[component][...]`` with component 0 = x, 1 = y, 2 = z;
* node ``i`` along an axis of length ``L`` with ``N`` nodes sits at ``i*L/N``
  (the periodic grid of Sec. 2.2, node ``N`` identified with node 0).

Recipes (all fields periodic on the box):

* ``bump_workload``     -- r = 0.1, S = unit-peak Gaussian bump (sigma 0.05) at the
  box centre minus its grid mean, m0 i.i.d. uniform[0,1] per component;
* ``dipole_workload``   -- r = 0.05 + 0.05 f with f a smooth random field (16
  random low-wavenumber cosine modes, |f| <= 0.9), S = a Gaussian source at
  (0.25, 0.5) and a Gaussian sink at (0.75, 0.5) (sigma 0.02, amplitude 1),
  m0 i.i.d. uniform[0,1];
* the paper's own analytic data of Sec. 3: the initial conductivities m^A, m^B,
  m^const (eqs. m_ini_normal, m_ini_symm, m_ini_const), the one-source/four-sink
  term S_4 (eqs. S_4sinks...) and the internal-sink term S_int (eq. SinternalSink).
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "grid_coords",
    "gaussian",
    "smooth_random_field",
    "bump_workload",
    "dipole_workload",
    "paper_m_A",
    "paper_m_B",
    "paper_m_const",
    "paper_S4",
    "paper_Sint",
]


def _as_tuple(v, d):
    if np.isscalar(v):
        return (float(v),) * d
    v = tuple(float(x) for x in v)
    if len(v) != d:
        raise ValueError("length mismatch")
    return v


def grid_coords(n, L=1.0):
    """Node coordinates as a list [X, Y(, Z)] of arrays of shape ``n[::-1]``."""
    n = tuple(int(v) for v in n)
    d = len(n)
    L = _as_tuple(L, d)
    axes = [np.arange(n[c], dtype=np.float64) * (L[c] / n[c]) for c in range(d)]
    # meshgrid with 'ij' on the reversed axis order gives arrays indexed [z][y][x]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")
    return mesh[::-1]


def gaussian(coords, center, sigma):
    """exp(-|x - center|^2 / (2 sigma^2)) with plain Euclidean distance."""
    r2 = np.zeros_like(coords[0])
    for X, c in zip(coords, center):
        r2 += (X - c) ** 2
    return np.exp(-r2 / (2.0 * sigma * sigma))


def smooth_random_field(rng, n, L=1.0, n_modes=16, kmax=4):
    """f = 0.9 * g / sum|a_j|, g = sum_j a_j cos(2 pi k_j . x / L + phi_j).

    Draw order per mode j: the integer wavevector k_j (uniform in
    {-kmax..kmax}^d, rejecting 0), then a_j ~ N(0,1), then phi_j ~ U[0, 2 pi).
    |f| <= 0.9 everywhere by construction.
    """
    n = tuple(int(v) for v in n)
    d = len(n)
    L = _as_tuple(L, d)
    X = grid_coords(n, L)
    g = np.zeros(n[::-1])
    total = 0.0
    for _ in range(n_modes):
        while True:
            k = rng.integers(-kmax, kmax + 1, size=d)
            if np.any(k != 0):
                break
        a = rng.standard_normal()
        phi = rng.uniform(0.0, 2.0 * np.pi)
        arg = np.full(n[::-1], phi)
        for c in range(d):
            arg += 2.0 * np.pi * k[c] * X[c] / L[c]
        g += a * np.cos(arg)
        total += abs(a)
    return 0.9 * g / total


def _uniform_m0(rng, n):
    d = len(n)
    return np.ascontiguousarray(rng.random((d,) + tuple(n[::-1])))


def bump_workload(N=64, seed_m0=0, ndim=2):
    """Small 2D/3D case: r = 0.1, centred Gaussian bump source, uniform m0.

    Parameters D^2 = 1e-3, c^2 = 25, gamma = 0.75, dt = 1e-3, 100 steps,
    relative PCG tolerance 1e-10.
    """
    n = (N,) * ndim
    X = grid_coords(n, 1.0)
    S = gaussian(X, (0.5,) * ndim, 0.05)
    S = S - S.mean()
    r = np.full(n[::-1], 0.1)
    m0 = _uniform_m0(np.random.default_rng(seed_m0), n)
    return dict(
        n=n, L=(1.0,) * ndim, r=r, S=np.ascontiguousarray(S), m0=m0,
        c2=25.0, D2=1e-3, gamma=0.75, dt=1e-3, steps=100, rtol=1e-10,
    )


def dipole_workload(N=1024, gamma=0.75, seed_r=1, seed_m0=2, ndim=2):
    """Large case: smooth random r, Gaussian source/sink pair, uniform m0.

    Parameters D^2 = 1e-4, c^2 = 50, gamma as given (0.5, 0.75 or 1.0),
    dt = 5e-4, 1000 steps, relative PCG tolerance 1e-10.
    """
    n = (N,) * ndim
    X = grid_coords(n, 1.0)
    f = smooth_random_field(np.random.default_rng(seed_r), n, 1.0)
    r = 0.05 + 0.05 * f
    centre_src = (0.25,) + (0.5,) * (ndim - 1)
    centre_snk = (0.75,) + (0.5,) * (ndim - 1)
    S = gaussian(X, centre_src, 0.02) - gaussian(X, centre_snk, 0.02)
    S = S - S.mean()  # removes only rounding: the pair cancels by half-period symmetry
    m0 = _uniform_m0(np.random.default_rng(seed_m0), n)
    return dict(
        n=n, L=(1.0,) * ndim, r=np.ascontiguousarray(r), S=np.ascontiguousarray(S), m0=m0,
        c2=50.0, D2=1e-4, gamma=float(gamma), dt=5e-4, steps=1000, rtol=1e-10,
    )


ENSEMBLE_MIX = ((256, 16), (512, 32), (1024, 16))


def ensemble_workload(mix=ENSEMBLE_MIX, seed0=1000):
    """Ensemble of independent instances: for each (N, count) in `mix`, `count`
    instances on an N x N grid, instance i (numbered across the mix) drawing
    from default_rng(seed0 + i): first the smooth random field of r (as in
    dipole_workload), then m0, then c^2 log-uniform in [5, 100], D^2
    log-uniform in [1e-5, 1e-3] and gamma uniform in [0.5, 1.25].  S is the
    Gaussian source/sink pair of dipole_workload.  dt = 5e-4, 500 steps,
    relative PCG tolerance 1e-10.  Returns a list of per-instance dicts with
    keys n, L, r, S, m0, c2, D2, gamma.
    """
    out = []
    i = 0
    for N, count in mix:
        n = (N, N)
        X = grid_coords(n, 1.0)
        S = gaussian(X, (0.25, 0.5), 0.02) - gaussian(X, (0.75, 0.5), 0.02)
        S = np.ascontiguousarray(S - S.mean())
        for _ in range(count):
            rng = np.random.default_rng(seed0 + i)
            r = 0.05 + 0.05 * smooth_random_field(rng, n, 1.0)
            m0 = _uniform_m0(rng, n)
            c2 = float(np.exp(rng.uniform(np.log(5.0), np.log(100.0))))
            D2 = float(np.exp(rng.uniform(np.log(1e-5), np.log(1e-3))))
            gamma = float(rng.uniform(0.5, 1.25))
            out.append(dict(n=n, L=(1.0, 1.0), r=np.ascontiguousarray(r), S=S, m0=m0, c2=c2, D2=D2, gamma=gamma))
            i += 1
    return out


ENSEMBLE_RUN = dict(dt=5e-4, steps=500, rtol=1e-10)


# ---- analytic data printed in the paper (Sec. 3.1-3.3) --------------------------------

def paper_m_A(N, factor=1.0e4):
    """m^A = (exp(-factor (y-0.5)^2 - 50 (x-0.5)^2), 0) on [0,1)^2 (eq. m_ini_normal)."""
    X, Y = grid_coords((N, N), 1.0)
    m = np.zeros((2, N, N))
    m[0] = np.exp(-factor * (Y - 0.5) ** 2 - 50.0 * (X - 0.5) ** 2)
    return m


def paper_m_B(N):
    """m^B = (exp(-50 (y-0.5)^2 - 50 (x-0.5)^2), 0) (eq. m_ini_symm)."""
    X, Y = grid_coords((N, N), 1.0)
    m = np.zeros((2, N, N))
    m[0] = np.exp(-50.0 * (Y - 0.5) ** 2 - 50.0 * (X - 0.5) ** 2)
    return m


def paper_m_const(N):
    """m^const = (1, 1) (eq. m_ini_const)."""
    return np.ones((2, N, N))


def paper_S4(N):
    """One source at the centre and four quarter-weight sinks (eqs. S_4sinks...)."""
    X, Y = grid_coords((N, N), 1.0)
    src = np.exp(-1000.0 * ((Y - 0.5) ** 2 + (X - 0.5) ** 2))
    snk = np.zeros_like(src)
    for (xi, yi) in ((0.2, 0.2), (0.2, 0.8), (0.8, 0.2), (0.8, 0.8)):
        snk += 0.25 * np.exp(-1000.0 * ((Y - yi) ** 2 + (X - xi) ** 2))
    return src - snk


def paper_Sint(N):
    """Internal sink: exp(-1000 |x - (0.5,0.5)|^2) - pi/1000 (eq. SinternalSink)."""
    X, Y = grid_coords((N, N), 1.0)
    return np.exp(-1000.0 * ((Y - 0.5) ** 2 + (X - 0.5) ** 2)) - np.pi / 1000.0
