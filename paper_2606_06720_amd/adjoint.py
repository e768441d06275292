"""Reverse-mode differentiation of a run of the time loop through the C ABI.

``run_gradient`` advances m from m0 for a fixed number of steps (nf_step),
then sweeps nf_step_adjoint backwards.  States are checkpointed every
``stride`` steps (default ceil(sqrt(steps))); each segment is recomputed from its
checkpoint, on a second handle and stream while the adjoint steps of the segment
after it run, so the memory holds about 3 sqrt(steps) states.  The kernels are
deterministic, so a recomputed segment reproduces the forward states bit for
bit.

``NetworkRun`` wraps the same sweep as a ``torch.autograd.Function`` mapping
(r, S) to the final conductivity m_T; any torch loss on m_T can then be
differentiated with respect to the fields r(x, y) and S(x, y).

All arithmetic runs in the library's kernels; this module only orders calls
and keeps device buffers.
"""

from __future__ import annotations

import math
import threading

import torch

from . import nf as NF


def _zeros_like(t):
    return torch.zeros_like(t)


_recompute_streams = {}


def _recompute_stream():
    """The stream of the overlapped recomputation, one per device for the
    process: a fresh stream per sweep can land on the hardware queue of another
    busy stream, which serialises the two."""
    dev = torch.cuda.current_device()
    if dev not in _recompute_streams:
        _recompute_streams[dev] = torch.cuda.Stream(device=dev)
    return _recompute_streams[dev]


def forward_states(grid, prm, dt, steps, m0, r, S, rtol, max_iter, stride):
    """Run `steps` nf_step calls from (m0, p = 0); return m_T and the checkpoints
    {k: (m_k, p_{k-1})} for k = 0, stride, 2 stride, ..."""
    c2, D2, gamma = prm
    m = m0.clone()
    p = torch.zeros_like(r)
    ckpt = {}
    for k in range(steps):
        if k % stride == 0:
            ckpt[k] = (m.clone(), p.clone())
        grid.step(c2, D2, gamma, dt, m, p, r, S, rtol=rtol, max_iter=max_iter)
    return m, ckpt


def _recompute(grid, prm, dt, c, end, ckpt, r, S, rtol, max_iter):
    """Forward steps c .. end - 1 from checkpoint c; returns [(m_k, p[m_k])] and
    the PCG iterations spent."""
    c2, D2, gamma = prm
    m, p = ckpt[c][0].clone(), ckpt[c][1].clone()
    seg, iters = [], 0
    for _ in range(c, end):
        m_k = m.clone()
        _, si = grid.step(c2, D2, gamma, dt, m, p, r, S, rtol=rtol, max_iter=max_iter)
        seg.append((m_k, p.clone()))  # p now holds p[m_k]
        iters += si.solve.iters
    return seg, iters


def _adjoint_segment(grid, prm, dt, c, seg, r, S, lam, lam_k, grad_r, grad_S, mu, rtol, max_iter):
    """Adjoint steps of a recomputed segment, last step first; returns the
    buffers (lam, lam_k) with lam = dL/dm_c, and the PCG iterations spent."""
    c2, D2, gamma = prm
    iters = 0
    for k in range(c + len(seg) - 1, c - 1, -1):
        m_k, p_k = seg[k - c]
        _, ai = grid.step_adjoint(c2, D2, gamma, dt, m_k, p_k, r, S, lam, lam_k, grad_r, grad_S, mu, rtol=rtol,
                                  max_iter=max_iter)
        lam, lam_k = lam_k, lam
        iters += ai.iters
    return lam, lam_k, iters


def adjoint_sweep(grid, prm, dt, steps, r, S, ckpt, lam_T, rtol, max_iter, stride, stats=None, overlap=True,
                  streams=None):
    """Backward sweep from lam_T = dL/dm_T; returns (dL/dm0, dL/dr, dL/dS).
    If `stats` is a dict, PCG iteration counts of the recomputed forward steps
    and of the adjoint steps are accumulated in it.

    overlap: the recomputation of segment j - 1 runs on a second handle (same
    grid, box and precision) and a stream of its own, from its own host thread,
    while `grid` runs the adjoint steps of segment j on the caller's current
    stream (or the pair `streams` = (adjoint, recomputation)); the two meet
    after each segment.  Each call's result depends only on its inputs, so the
    gradients are bitwise those of the sequential sweep."""
    grad_r = torch.zeros_like(r)
    grad_S = torch.zeros_like(S)
    mu = torch.zeros_like(r)
    lam = lam_T.clone()
    lam_k = torch.empty_like(lam)
    starts = sorted(ckpt.keys())
    ends = {c: min(c + stride, steps) for c in starts}
    rec_iters = adj_iters = 0
    if not overlap or len(starts) < 2:
        for c in reversed(starts):
            seg, it = _recompute(grid, prm, dt, c, ends[c], ckpt, r, S, rtol, max_iter)
            rec_iters += it
            lam, lam_k, it = _adjoint_segment(grid, prm, dt, c, seg, r, S, lam, lam_k, grad_r, grad_S, mu, rtol,
                                              max_iter)
            adj_iters += it
    else:
        helper = NF.Grid(grid.n, grid.L, dtype=grid.dtype)
        s_adj, s_rec = streams if streams is not None else (torch.cuda.current_stream(), _recompute_stream())
        torch.cuda.synchronize()
        try:
            with torch.cuda.stream(s_rec):
                seg, it = _recompute(helper, prm, dt, starts[-1], ends[starts[-1]], ckpt, r, S, rtol, max_iter)
            rec_iters += it
            torch.cuda.synchronize()
            for j in range(len(starts) - 1, -1, -1):
                out = {}

                def rec(c=starts[j - 1] if j > 0 else None):
                    try:
                        with torch.cuda.stream(s_rec):
                            out["seg"] = _recompute(helper, prm, dt, c, ends[c], ckpt, r, S, rtol, max_iter)
                    except BaseException as e:  # re-raised on the calling thread
                        out["err"] = e

                th = threading.Thread(target=rec) if j > 0 else None
                if th is not None:
                    th.start()
                try:
                    with torch.cuda.stream(s_adj):
                        lam, lam_k, it = _adjoint_segment(grid, prm, dt, starts[j], seg, r, S, lam, lam_k, grad_r,
                                                          grad_S, mu, rtol, max_iter)
                    adj_iters += it
                finally:
                    if th is not None:
                        th.join()
                torch.cuda.synchronize()
                if "err" in out:
                    raise out["err"]
                if th is not None:
                    seg, it = out["seg"]
                    rec_iters += it
        finally:
            torch.cuda.synchronize()
            helper.close()
    if stats is not None:
        stats["recompute_iters"] = stats.get("recompute_iters", 0) + rec_iters
        stats["adjoint_iters"] = stats.get("adjoint_iters", 0) + adj_iters
    return lam, grad_r, grad_S


def misfit_loss(m, m_target):
    """L = 1/2 sum (|m| - |m_target|)^2 and dL/dm (zero where |m| = 0)."""
    a = torch.sqrt((m * m).sum(0))
    at = torch.sqrt((m_target * m_target).sum(0))
    diff = a - at
    lam = torch.where(a > 0, diff / torch.where(a > 0, a, torch.ones_like(a)), torch.zeros_like(a))[None] * m
    return 0.5 * float((diff * diff).sum()), lam


def run_gradient(grid, prm, dt, steps, m0, r, S, m_target, rtol=1e-12, max_iter=2000, stride=None):
    """Misfit of the final |m| against |m_target| after `steps` steps, and its
    gradients with respect to r and S.  Returns (loss, dL/dr, dL/dS)."""
    stride = stride or max(1, int(math.ceil(math.sqrt(steps))))
    m_T, ckpt = forward_states(grid, prm, dt, steps, m0, r, S, rtol, max_iter, stride)
    loss, lam_T = misfit_loss(m_T, m_target)
    _, gr, gS = adjoint_sweep(grid, prm, dt, steps, r, S, ckpt, lam_T, rtol, max_iter, stride)
    return loss, gr, gS


class NetworkRun(torch.autograd.Function):
    """(r, S) -> m_T after `steps` time steps from m0 (p^0 = 0)."""

    @staticmethod
    def forward(ctx, r, S, grid, prm, dt, steps, m0, rtol, max_iter, stride):
        stride = stride or max(1, int(math.ceil(math.sqrt(steps))))
        r = r.detach().contiguous()
        S = S.detach().contiguous()
        m_T, ckpt = forward_states(grid, prm, dt, steps, m0.detach().contiguous(), r, S, rtol, max_iter, stride)
        ctx.saved = (grid, prm, dt, steps, r, S, ckpt, rtol, max_iter, stride)
        return m_T

    @staticmethod
    def backward(ctx, grad_mT):
        grid, prm, dt, steps, r, S, ckpt, rtol, max_iter, stride = ctx.saved
        _, gr, gS = adjoint_sweep(grid, prm, dt, steps, r, S, ckpt, grad_mT.contiguous(), rtol, max_iter, stride)
        return gr, gS, None, None, None, None, None, None, None, None


def network_run(r, S, grid, prm, dt, steps, m0, rtol=1e-12, max_iter=2000, stride=None):
    """Differentiable final state m_T(r, S) (see NetworkRun)."""
    return NetworkRun.apply(r, S, grid, prm, dt, steps, m0, rtol, max_iter, stride)
