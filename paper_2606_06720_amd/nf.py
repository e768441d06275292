"""Python binding of the C ABI in ``include/nf.h`` (argument marshalling only).

Every call goes straight to ``libnf.so``; all arithmetic of the time step runs in
the library's HIP kernels.  Fields are torch tensors on the current HIP device
(float64, C-contiguous): scalars ``[Ny, Nx]``, the conductivity ``m`` as
``[2, Ny, Nx]`` with component 0 = m_x.  The handle enqueues on torch's current
stream at each call.

If the library is missing this module raises on import: there is no fallback.
"""

from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnf.so")

NF_OK = 0
NF_EINVAL = -1
NF_ENOMEM = -2
NF_EDEVICE = -3
NF_ENOTCONV = -4
NF_EINCOMPAT = -5
NF_ENONFINITE = -6
NF_F64 = 0
NF_F32_REFINED = 1
NF_STOP_MAX_STEPS = 0
NF_STOP_DM_BELOW_EPS = 1
NF_STOP_ENERGY_INCREASE = 2
NF_STOP_ERROR = 3
NF_KERNEL_ROW_FLUX = 0
NF_KERNEL_COL_DIV = 1
NF_KERNEL_COL_UPDATE = 2

_CODES = {
    NF_EINVAL: "NF_EINVAL",
    NF_ENOMEM: "NF_ENOMEM",
    NF_EDEVICE: "NF_EDEVICE",
    NF_ENOTCONV: "NF_ENOTCONV",
    NF_EINCOMPAT: "NF_EINCOMPAT",
    NF_ENONFINITE: "NF_ENONFINITE",
}


class NfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_CODES.get(code, "NF_?"), code, msg))
        self.code = code


class nf_params(ctypes.Structure):
    _fields_ = [("c2", ctypes.c_double), ("D2", ctypes.c_double), ("gamma", ctypes.c_double)]


class nf_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("true_rel_res", ctypes.c_double)]


class nf_step_info(ctypes.Structure):
    _fields_ = [("solve", nf_solve_info), ("dm_rel", ctypes.c_double), ("energy", ctypes.c_double),
                ("energy_valid", ctypes.c_int)]


class nf_run_info(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("stop_reason", ctypes.c_int), ("last_dm", ctypes.c_double),
                ("last_energy", ctypes.c_double), ("prev_energy", ctypes.c_double),
                ("total_cg_iters", ctypes.c_int64), ("unconverged_solves", ctypes.c_int64)]


class nf_tuning_info(ctypes.Structure):
    _fields_ = [("tuned", ctypes.c_int), ("flux_rows", ctypes.c_int), ("flux_plan", ctypes.c_int),
                ("div_cols", ctypes.c_int), ("div_plan", ctypes.c_int), ("div_threads", ctypes.c_int),
                ("update_cols", ctypes.c_int), ("update_plan", ctypes.c_int), ("update_threads", ctypes.c_int),
                ("candidates", ctypes.c_int * 3), ("us", ctypes.c_double * 3),
                ("us_default", ctypes.c_double * 3), ("flux_threads", ctypes.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libnf.so is not built (run __graft_entry__.build()): " + LIB_PATH)
    # torch brings its own HIP runtime; it must be the one in the process before
    # the library is loaded, or two runtimes end up fighting over the device
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    vp, dp, i64p = ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(ctypes.c_int64)
    lib.nf_create_grid.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64p, ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_int, vp]
    lib.nf_destroy_grid.argtypes = [vp]
    lib.nf_set_stream.argtypes = [vp, vp]
    lib.nf_pressure_solve.argtypes = [vp, vp, vp, vp, vp, dp, ctypes.c_int, ctypes.POINTER(nf_solve_info)]
    lib.nf_pressure_solve_noalloc.argtypes = [i64p, ctypes.POINTER(ctypes.c_double), vp, vp, vp, vp, vp, dp,
                                              ctypes.c_int, ctypes.POINTER(nf_solve_info)]
    lib.nf_step.argtypes = [vp, ctypes.POINTER(nf_params), dp, vp, vp, vp, vp, dp, ctypes.c_int,
                            ctypes.POINTER(nf_step_info)]
    lib.nf_set_step_energy.argtypes = [vp, ctypes.c_int]
    lib.nf_run.argtypes = [vp, ctypes.POINTER(nf_params), dp, ctypes.c_int64, dp, ctypes.c_int, vp, vp, vp, vp,
                           dp, ctypes.c_int, ctypes.POINTER(nf_run_info)]
    lib.nf_energy.argtypes = [vp, ctypes.POINTER(nf_params), vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double)]
    lib.nf_step_adjoint.argtypes = [vp, ctypes.POINTER(nf_params), dp, vp, vp, vp, vp, vp, vp, vp, vp, vp, dp,
                                     ctypes.c_int, ctypes.POINTER(nf_solve_info)]
    lib.nf_transform_forward.argtypes = [vp, vp, vp]
    lib.nf_transform_inverse.argtypes = [vp, vp, vp]
    lib.nf_apply_operator.argtypes = [vp, vp, vp, vp, vp]
    lib.nf_gradient.argtypes = [vp, vp, vp]
    lib.nf_set_inner_tolerance.argtypes = [vp, dp]
    lib.nf_set_autotune.argtypes = [ctypes.c_int]
    lib.nf_tuning.argtypes = [vp, ctypes.POINTER(nf_tuning_info)]
    lib.nf_set_tiles.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.nf_time_kernel.argtypes = [vp, ctypes.c_int]
    lib.nf_time_kernel_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.nf_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64p, ctypes.POINTER(ctypes.c_double),
                                    ctypes.c_int, vp]
    lib.nf_batch_destroy.argtypes = [vp]
    lib.nf_batch_set_stream.argtypes = [vp, vp]
    lib.nf_batch_run.argtypes = [vp, ctypes.POINTER(nf_params), dp, ctypes.c_int64, ctypes.POINTER(vp),
                                 ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), dp, ctypes.c_int,
                                 ctypes.POINTER(nf_run_info)]
    lib.nf_batch_set_partitions.argtypes = [vp, ctypes.c_int]
    lib.nf_batch_partitions.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.nf_batch_set_graphs.argtypes = [vp, ctypes.c_int]
    lib.nf_batch_last_error.argtypes = [vp]
    lib.nf_batch_last_error.restype = ctypes.c_char_p
    lib.nf_last_error.argtypes = [vp]
    lib.nf_last_error.restype = ctypes.c_char_p
    lib.nf_version.restype = ctypes.c_char_p
    for f in ("nf_create_grid", "nf_destroy_grid", "nf_set_stream", "nf_pressure_solve", "nf_pressure_solve_noalloc",
              "nf_step", "nf_set_step_energy", "nf_run",
              "nf_energy", "nf_step_adjoint", "nf_transform_forward", "nf_transform_inverse", "nf_apply_operator",
              "nf_gradient", "nf_time_kernel",
              "nf_time_kernel_read", "nf_set_inner_tolerance", "nf_set_autotune", "nf_tuning", "nf_set_tiles",
              "nf_batch_create", "nf_batch_destroy",
              "nf_batch_set_stream", "nf_batch_run", "nf_batch_set_partitions", "nf_batch_partitions",
              "nf_batch_set_graphs"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


_lib = _load()


def version():
    return _lib.nf_version().decode()


@dataclass
class SolveInfo:
    iters: int
    converged: bool
    rel_res: float
    true_rel_res: float


@dataclass
class StepInfo:
    solve: SolveInfo
    dm_rel: float
    energy: float = float("nan")  # E_h(m^k) when the handle evaluates it (set_step_energy)
    energy_valid: bool = False


@dataclass
class RunInfo:
    steps: int
    stop_reason: int
    last_dm: float
    last_energy: float
    prev_energy: float
    total_cg_iters: int
    unconverged_solves: int


def _si(s):
    return SolveInfo(int(s.iters), bool(s.converged), float(s.rel_res), float(s.true_rel_res))


def _ptr(t, shape, name):
    import torch

    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError("%s must be a contiguous float64 device tensor of shape %s (got %s %s %s)"
                         % (name, tuple(shape), t.dtype, t.device, tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


def _current_stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Grid:
    """A solver handle (``nf_create_grid``) for an Nx x Ny (x Nz) periodic box."""

    def __init__(self, n, L=None, dtype=NF_F64):
        n = tuple(int(v) for v in n)
        if len(n) not in (2, 3):
            raise ValueError("2D or 3D grids only")
        self.n = n
        self.dim = len(n)
        self.dtype = int(dtype)
        self.L = tuple(float(v) for v in (L if L is not None else (1.0,) * self.dim))
        if len(self.L) != self.dim:
            raise ValueError("one box length per axis")
        self._h = ctypes.c_void_p()
        nn = (ctypes.c_int64 * 3)(*(n + (1,) * (3 - self.dim)))
        LL = (ctypes.c_double * 3)(*(self.L + (1.0,) * (3 - self.dim)))
        rc = _lib.nf_create_grid(ctypes.byref(self._h), self.dim, nn, LL, int(dtype), _current_stream())
        if rc != NF_OK:
            raise NfError(rc, "nf_create_grid failed for n=%s L=%s: %s"
                          % (n, self.L, _lib.nf_last_error(None).decode()))

    # shapes
    @property
    def sshape(self):
        return tuple(self.n[::-1])

    @property
    def vshape(self):
        return (self.dim,) + tuple(self.n[::-1])

    def _check(self, rc, allow=()):
        if rc != NF_OK and rc not in allow:
            raise NfError(rc, _lib.nf_last_error(self._h).decode())
        return rc

    def _sync_stream(self):
        _lib.nf_set_stream(self._h, _current_stream())

    def close(self):
        if self._h:
            _lib.nf_destroy_grid(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def pressure_solve(self, m, r, S, p, rtol=1e-10, max_iter=1000, allow_notconv=False):
        """nf_pressure_solve: p (in: warm start, out: solution). Returns (rc, SolveInfo)."""
        self._sync_stream()
        info = nf_solve_info()
        rc = _lib.nf_pressure_solve(self._h, _ptr(m, self.vshape, "m"), _ptr(r, self.sshape, "r"),
                                    _ptr(S, self.sshape, "S"), _ptr(p, self.sshape, "p"), float(rtol),
                                    int(max_iter), ctypes.byref(info))
        self._check(rc, (NF_ENOTCONV,) if allow_notconv else ())
        return rc, _si(info)

    def step(self, c2, D2, gamma, dt, m, p, r, S, rtol=1e-10, max_iter=1000, allow_notconv=False):
        """nf_step: m^k -> m^{k+1} in place, p <- p[m^k]. Returns (rc, StepInfo)."""
        self._sync_stream()
        prm = nf_params(float(c2), float(D2), float(gamma))
        info = nf_step_info()
        rc = _lib.nf_step(self._h, ctypes.byref(prm), float(dt), _ptr(m, self.vshape, "m"),
                          _ptr(p, self.sshape, "p"), _ptr(r, self.sshape, "r"), _ptr(S, self.sshape, "S"),
                          float(rtol), int(max_iter), ctypes.byref(info))
        self._check(rc, (NF_ENOTCONV,) if allow_notconv else ())
        return rc, StepInfo(_si(info.solve), float(info.dm_rel), float(info.energy), bool(info.energy_valid))

    def set_step_energy(self, on):
        """nf_set_step_energy: whether step() also evaluates E_h of the state it starts from."""
        self._check(_lib.nf_set_step_energy(self._h, 1 if on else 0))

    def run(self, c2, D2, gamma, dt, max_steps, m, p, r, S, eps_dm=0.0, stop_on_energy_increase=False,
            rtol=1e-10, max_iter=1000):
        """nf_run: time loop with the stopping criteria. Returns RunInfo."""
        self._sync_stream()
        prm = nf_params(float(c2), float(D2), float(gamma))
        info = nf_run_info()
        rc = _lib.nf_run(self._h, ctypes.byref(prm), float(dt), int(max_steps), float(eps_dm),
                         int(bool(stop_on_energy_increase)), _ptr(m, self.vshape, "m"), _ptr(p, self.sshape, "p"),
                         _ptr(r, self.sshape, "r"), _ptr(S, self.sshape, "S"), float(rtol), int(max_iter),
                         ctypes.byref(info))
        self._check(rc)
        return RunInfo(int(info.steps), int(info.stop_reason), float(info.last_dm), float(info.last_energy),
                       float(info.prev_energy), int(info.total_cg_iters), int(info.unconverged_solves))

    def step_adjoint(self, c2, D2, gamma, dt, m, p, r, S, lam_next, lam_k, grad_r, grad_S, mu, rtol=1e-12,
                     max_iter=2000, allow_notconv=False):
        """nf_step_adjoint: lam_k <- dL/dm^k; grad_r, grad_S += this step's gradients; mu inout."""
        self._sync_stream()
        prm = nf_params(float(c2), float(D2), float(gamma))
        info = nf_solve_info()
        rc = _lib.nf_step_adjoint(self._h, ctypes.byref(prm), float(dt), _ptr(m, self.vshape, "m"),
                                  _ptr(p, self.sshape, "p"), _ptr(r, self.sshape, "r"), _ptr(S, self.sshape, "S"),
                                  _ptr(lam_next, self.vshape, "lam_next"), _ptr(lam_k, self.vshape, "lam_k"),
                                  _ptr(grad_r, self.sshape, "grad_r"), _ptr(grad_S, self.sshape, "grad_S"),
                                  _ptr(mu, self.sshape, "mu"), float(rtol), int(max_iter), ctypes.byref(info))
        self._check(rc, (NF_ENOTCONV,) if allow_notconv else ())
        return rc, _si(info)

    def energy(self, c2, D2, gamma, m, r, S, p=None):
        """nf_energy: (total, D^2/2|grad m|^2, relaxation, c^2/2|m.grad p|^2, c^2/2 r|grad p|^2)."""
        self._sync_stream()
        prm = nf_params(float(c2), float(D2), float(gamma))
        out = (ctypes.c_double * 5)()
        rc = _lib.nf_energy(self._h, ctypes.byref(prm), _ptr(m, self.vshape, "m"), _ptr(p, self.sshape, "p"),
                            _ptr(r, self.sshape, "r"), _ptr(S, self.sshape, "S"), out)
        self._check(rc)
        return tuple(float(v) for v in out)


    # diagnostics -----------------------------------------------------------
    def tuning(self):
        """nf_tuning: the tile variants of the PCG loop of this handle, as a dict."""
        t = nf_tuning_info()
        self._check(_lib.nf_tuning(self._h, ctypes.byref(t)))
        return {"tuned": bool(t.tuned), "flux_rows": t.flux_rows, "flux_plan": t.flux_plan,
                "flux_threads": t.flux_threads, "div_cols": t.div_cols,
                "div_plan": t.div_plan, "div_threads": t.div_threads, "update_cols": t.update_cols,
                "update_plan": t.update_plan, "update_threads": t.update_threads,
                "candidates": list(t.candidates), "us": list(t.us), "us_default": list(t.us_default)}

    def set_tiles(self, flux_var=-1, div_var=-1, update_var=-1):
        """nf_set_tiles: fix this handle's tile variants (operator middle 0..8, others 0..11; -1 keeps)."""
        self._check(_lib.nf_set_tiles(self._h, int(flux_var), int(div_var), int(update_var)))

    def set_inner_tolerance(self, floor_rtol):
        self._check(_lib.nf_set_inner_tolerance(self._h, float(floor_rtol)))

    def time_kernel(self, which):
        """nf_time_kernel: time launches of one PCG-loop kernel (-1 = off)."""
        self._check(_lib.nf_time_kernel(self._h, int(which)))

    def time_kernel_read(self):
        """nf_time_kernel_read: (total ms, launches counted)."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        self._check(_lib.nf_time_kernel_read(self._h, ctypes.byref(ms), ctypes.byref(cnt)))
        return float(ms.value), int(cnt.value)

    @property
    def spec_shape(self):
        return (self.n[0] // 2,) + tuple(self.n[1:]) + (2,)

    def transform_forward(self, f, out):
        """nf_transform_forward: packed half spectrum [Nx/2][Ny]([Nz]) (re, im) of f."""
        self._sync_stream()
        self._check(_lib.nf_transform_forward(self._h, _ptr(f, self.sshape, "f"), _ptr(out, self.spec_shape, "out")))

    def transform_inverse(self, spec, f):
        """nf_transform_inverse: normalised inverse of a packed half spectrum."""
        self._sync_stream()
        self._check(_lib.nf_transform_inverse(self._h, _ptr(spec, self.spec_shape, "spec"), _ptr(f, self.sshape, "f")))

    def apply_operator(self, m, r, p, out):
        """nf_apply_operator: out = A p (left-hand side of the discrete pressure equation)."""
        self._sync_stream()
        self._check(_lib.nf_apply_operator(self._h, _ptr(m, self.vshape, "m"), _ptr(r, self.sshape, "r"),
                                           _ptr(p, self.sshape, "p"), _ptr(out, self.sshape, "out")))

    def gradient(self, f, grad):
        """nf_gradient: grad [2][Ny][Nx] = spectral gradient of f [Ny][Nx] (2D)."""
        self._sync_stream()
        self._check(_lib.nf_gradient(self._h, _ptr(f, self.sshape, "f"), _ptr(grad, self.vshape, "grad")))


def _ri(x):
    return RunInfo(int(x.steps), int(x.stop_reason), float(x.last_dm), float(x.last_energy), float(x.prev_energy),
                   int(x.total_cg_iters), int(x.unconverged_solves))


class Batch:
    """An ensemble handle (``nf_batch_create``): independent instances with
    their own grid sizes (Nx, Ny) and boxes, advanced together by
    ``nf_batch_run``."""

    def __init__(self, shapes, L=None, dtype=NF_F64):
        shapes = [tuple(int(v) for v in n) for n in shapes]
        if not shapes or any(len(n) != 2 for n in shapes):
            raise ValueError("a non-empty list of 2D grid shapes is required")
        L = [(1.0, 1.0)] * len(shapes) if L is None else [tuple(float(v) for v in l) for l in L]
        if len(L) != len(shapes):
            raise ValueError("one box per instance")
        self.shapes, self.L, self.count = shapes, L, len(shapes)
        nn = (ctypes.c_int64 * (2 * self.count))(*[v for n in shapes for v in n])
        LL = (ctypes.c_double * (2 * self.count))(*[v for l in L for v in l])
        self._h = ctypes.c_void_p()
        rc = _lib.nf_batch_create(ctypes.byref(self._h), self.count, nn, LL, int(dtype), _current_stream())
        if rc != NF_OK:
            raise NfError(rc, "nf_batch_create failed: %s" % _lib.nf_batch_last_error(None).decode())

    def close(self):
        if self._h:
            _lib.nf_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_partitions(self, parts):
        """nf_batch_set_partitions: 0 tunes the count at the next run."""
        rc = _lib.nf_batch_set_partitions(self._h, int(parts))
        if rc != NF_OK:
            raise NfError(rc, _lib.nf_batch_last_error(self._h).decode())

    def set_graphs(self, on):
        """nf_batch_set_graphs: replay recorded PCG chunks (True) or launch one by one."""
        rc = _lib.nf_batch_set_graphs(self._h, 1 if on else 0)
        if rc != NF_OK:
            raise NfError(rc, "nf_batch_set_graphs failed")

    def partitions(self):
        """nf_batch_partitions: (count in use, tuning ms per candidate count)."""
        t = (ctypes.c_double * 4)()
        k = _lib.nf_batch_partitions(self._h, t)
        if k < 0:
            raise NfError(k, "nf_batch_partitions failed")
        return k, [v for v in t]

    def run(self, params, dt, steps, m, p, r, S, rtol=1e-10, max_iter=1000):
        """nf_batch_run: params is a list of (c2, D2, gamma); m, p, r, S lists of
        device tensors (one per instance, shapes as for Grid.run).  Returns the
        list of RunInfo."""
        c = self.count
        if not (len(params) == len(m) == len(p) == len(r) == len(S) == c):
            raise ValueError("one entry per instance is required")
        _lib.nf_batch_set_stream(self._h, _current_stream())
        prm = (nf_params * c)(*[nf_params(float(a), float(b), float(g)) for a, b, g in params])
        ptrs = []
        for name, lst, vec in (("m", m, True), ("p", p, False), ("r", r, False), ("S", S, False)):
            arr = (ctypes.c_void_p * c)()
            for i, t in enumerate(lst):
                nx, ny = self.shapes[i]
                arr[i] = _ptr(t, (2, ny, nx) if vec else (ny, nx), "%s[%d]" % (name, i)).value
            ptrs.append(arr)
        info = (nf_run_info * c)()
        rc = _lib.nf_batch_run(self._h, prm, float(dt), int(steps), ptrs[0], ptrs[1], ptrs[2], ptrs[3], float(rtol),
                               int(max_iter), info)
        if rc != NF_OK:
            raise NfError(rc, _lib.nf_batch_last_error(self._h).decode())
        return [_ri(x) for x in info]


# C-ABI-named aliases ------------------------------------------------------------
def nf_create_grid(n, L=None, dtype=NF_F64):
    return Grid(n, L, dtype)


def nf_destroy_grid(g):
    g.close()


def nf_pressure_solve(g, m, r, S, p, rtol=1e-10, max_iter=1000):
    return g.pressure_solve(m, r, S, p, rtol, max_iter)


def nf_pressure_solve_noalloc(n, L, m, r, S, p, rtol=1e-10, max_iter=1000, allow_notconv=False):
    """nf_pressure_solve_noalloc on the current torch stream: the handle-free
    solve whose workspace is the library's fixed device array (2D FP64,
    power-of-two sides, Nx * Ny <= 65536).  Returns (rc, SolveInfo)."""
    n = tuple(int(v) for v in n)
    L = tuple(float(v) for v in (L if L is not None else (1.0, 1.0)))
    if len(n) != 2 or len(L) != 2:
        raise ValueError("2D grids only")
    ss, vs = (n[1], n[0]), (2, n[1], n[0])
    nn = (ctypes.c_int64 * 2)(*n)
    LL = (ctypes.c_double * 2)(*L)
    info = nf_solve_info()
    rc = _lib.nf_pressure_solve_noalloc(nn, LL, _current_stream(), _ptr(m, vs, "m"), _ptr(r, ss, "r"),
                                        _ptr(S, ss, "S"), _ptr(p, ss, "p"), float(rtol), int(max_iter),
                                        ctypes.byref(info))
    if rc != NF_OK and not (allow_notconv and rc == NF_ENOTCONV):
        raise NfError(rc, _lib.nf_last_error(None).decode())
    return rc, _si(info)


def nf_step(g, c2, D2, gamma, dt, m, p, r, S, rtol=1e-10, max_iter=1000):
    return g.step(c2, D2, gamma, dt, m, p, r, S, rtol, max_iter)


def nf_run(g, c2, D2, gamma, dt, max_steps, m, p, r, S, eps_dm=0.0, stop_on_energy_increase=False, rtol=1e-10,
           max_iter=1000):
    return g.run(c2, D2, gamma, dt, max_steps, m, p, r, S, eps_dm, stop_on_energy_increase, rtol, max_iter)


def nf_energy(g, c2, D2, gamma, m, r, S, p=None):
    return g.energy(c2, D2, gamma, m, r, S, p)


def nf_step_adjoint(g, c2, D2, gamma, dt, m, p, r, S, lam_next, lam_k, grad_r, grad_S, mu, rtol=1e-12,
                    max_iter=2000):
    return g.step_adjoint(c2, D2, gamma, dt, m, p, r, S, lam_next, lam_k, grad_r, grad_S, mu, rtol, max_iter)


def nf_set_autotune(mode):
    """Process-wide tuning of the tile variants at the first nf_create_grid of a
    shape: 2 (default) under three concurrent launches, 1 alone, 0 off."""
    rc = _lib.nf_set_autotune(int(mode))
    if rc != NF_OK:
        raise NfError(rc, "nf_set_autotune: mode must be 0, 1 or 2")


def nf_tuning(g):
    return g.tuning()


def nf_set_tiles(g, flux_var=-1, div_var=-1, update_var=-1):
    return g.set_tiles(flux_var, div_var, update_var)


def nf_set_inner_tolerance(g, floor_rtol):
    g.set_inner_tolerance(floor_rtol)


def nf_batch_create(shapes, L=None, dtype=NF_F64):
    return Batch(shapes, L, dtype)


def nf_batch_destroy(b):
    b.close()


def nf_batch_run(b, params, dt, steps, m, p, r, S, rtol=1e-10, max_iter=1000):
    return b.run(params, dt, steps, m, p, r, S, rtol, max_iter)


def nf_batch_set_partitions(b, parts):
    return b.set_partitions(parts)


def nf_batch_partitions(b):
    return b.partitions()


def nf_batch_set_graphs(b, on):
    return b.set_graphs(on)
