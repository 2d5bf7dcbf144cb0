"""Differentiation through many sweep steps: a torch.autograd.Function whose
backward pass is the library's hand-written adjoint with segment
checkpointing (the forward keeps the state every `ckpt` steps; the backward
recomputes each segment from its checkpoint and reverses it).  The last
segment is never recomputed: the forward runs it with
vdwlb_adjoint_forward, which keeps its densities and momenta in a
workspace that the backward reverses first.  With Spec.keep_moments the
forward keeps every segment's that way and the backward recomputes
nothing: 3 C nx ny doubles per step plus the per-segment fields (about 7 GB
for 2000 steps of a 256^2 two-component lattice), for callers with the
memory to spare.

Parameters theta = [kT, a^{cd} (c <= d), b^c, kappa] with the gradient
matrix kappa^{cd} = kappa * K_hat^{cd} (K_hat fixed), i.e. for two
components theta = [kT, a11, a12, a22, b1, b2, kappa].  The output is the
density field rho^c [C, ny, nx] of the final state.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import vdwlb as V
from .lattice import Plan, _stream_ptr


def theta_layout(C: int):
    pairs = [(c, d) for c in range(C) for d in range(c, C)]
    return pairs


def theta_from_params(kT, a, b, kappa_scalar):
    C = len(b)
    pairs = theta_layout(C)
    return np.array([kT] + [a[c][d] for c, d in pairs] + list(b) + [kappa_scalar], dtype=np.float64)


def params_from_theta(theta, C, k_hat):
    pairs = theta_layout(C)
    kT = float(theta[0])
    a = np.zeros((C, C))
    for q, (c, d) in enumerate(pairs):
        a[c, d] = a[d, c] = float(theta[1 + q])
    b = np.array([float(v) for v in theta[1 + len(pairs):1 + len(pairs) + C]])
    kappa = float(theta[-1]) * np.asarray(k_hat, dtype=np.float64)
    return kT, a, b, kappa


@dataclass
class Spec:
    """Everything but the differentiated parameters."""

    nx: int
    ny: int
    C: int
    k_hat: np.ndarray
    nsteps: int
    ckpt: int = 100
    tau: float = 1.0
    gamma_mu: float = 1.0
    lam: np.ndarray | None = None
    force: int = V.FORCE_LOG
    # sweep schedule of the forward and the recompute: "auto" (the autotuner's
    # choice, found once per lattice shape and kept), None (the plan's
    # default) or a schedule index; every schedule gives the same results
    schedule: int | str | None = "auto"
    graphs: bool = False  # replay the backward's recompute / reverse parts from captured hipGraphs
    keep_moments: bool = False  # keep every segment's moments from the forward: no recompute in the backward


class VdwLBFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, rho0, spec: Spec):
        th = theta.detach().cpu().numpy().astype(np.float64)
        kT, a, b, kappa = params_from_theta(th, spec.C, spec.k_hat)
        plan = Plan(spec.nx, spec.ny, kT, a, b, kappa, spec.tau, spec.gamma_mu, spec.lam, "f64", spec.force)
        if spec.graphs:
            V.check(V.lib().vdwlb_set_adjoint_graphs(plan.handle, 1), "vdwlb_set_adjoint_graphs")
        dev = rho0.device
        n = plan.state_elems
        bufs = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(2)]
        r0 = rho0.detach().to(torch.float64).contiguous()
        s = _stream_ptr()
        V.check(V.lib().vdwlb_init(plan.handle, bufs[0].data_ptr(), r0.data_ptr(), None, s), "vdwlb_init")
        _apply_schedule(plan, spec, bufs, s)
        segs = [min(spec.ckpt, spec.nsteps - d) for d in range(0, spec.nsteps, spec.ckpt)]
        n_rec = 0 if spec.keep_moments else len(segs) - 1  # segments the backward recomputes (the first n_rec)
        ckpts = []  # the states they start from
        kept = []  # workspaces of the other segments, whose moments the forward keeps
        cur = 0
        which = ctypes.c_int32()
        for k, m in enumerate(segs):
            if k < n_rec:
                ckpts.append(bufs[cur].clone())
                V.check(V.lib().vdwlb_step(plan.handle, bufs[cur].data_ptr(), bufs[1 - cur].data_ptr(), m, s,
                                           ctypes.byref(which)), "vdwlb_step")
                if which.value == 1:
                    cur = 1 - cur
            else:
                ws = torch.empty(int(V.lib().vdwlb_adjoint_workspace_bytes(plan.handle, m)) // 8 + 1,
                                 dtype=torch.float64, device=dev)
                V.check(V.lib().vdwlb_adjoint_forward(plan.handle, bufs[cur].data_ptr(), m, bufs[1 - cur].data_ptr(),
                                                      ws.data_ptr(), s), "vdwlb_adjoint_forward")
                kept.append(ws)
                cur = 1 - cur
        C, ny, nx = spec.C, spec.ny, spec.nx
        rho = torch.empty((C, ny, nx), dtype=torch.float64, device=dev)
        mom = torch.empty((C, 2, ny, nx), dtype=torch.float64, device=dev)
        V.check(V.lib().vdwlb_moments(plan.handle, bufs[cur].data_ptr(), rho.data_ptr(), mom.data_ptr(), None, None,
                                      s), "vdwlb_moments")
        ctx.plan, ctx.spec, ctx.ckpts, ctx.segs, ctx.kept = plan, spec, ckpts, segs, kept
        ctx.forward_done = torch.cuda.Event()
        ctx.forward_done.record(torch.cuda.current_stream(dev))
        ctx.theta_dtype, ctx.theta_device = theta.dtype, theta.device
        return rho

    @staticmethod
    def backward(ctx, grad_rho):
        plan, spec = ctx.plan, ctx.spec
        dev = grad_rho.device
        s = _stream_ptr()
        gb = grad_rho.detach().to(torch.float64).contiguous()
        fbar = torch.empty(plan.state_elems, dtype=torch.float64, device=dev)
        V.check(V.lib().vdwlb_moments_adjoint(plan.handle, gb.data_ptr(), None, fbar.data_ptr(), s),
                "vdwlb_moments_adjoint")
        npar = int(V.lib().vdwlb_adjoint_param_count(plan.handle))
        pbar = torch.zeros(npar, dtype=torch.float64, device=dev)
        segs = ctx.segs
        n_rec = len(ctx.ckpts)
        torch.cuda.current_stream(dev).wait_event(ctx.forward_done)  # the kept segments' workspaces

        def reverse_kept():  # the segments the forward kept, last first
            for m, ws in zip(reversed(segs[n_rec:]), reversed(ctx.kept)):
                V.check(V.lib().vdwlb_adjoint_reverse(plan.handle, int(m), fbar.data_ptr(), ws.data_ptr(),
                                                      pbar.data_ptr(), s), "vdwlb_adjoint_reverse")

        if n_rec == 0:
            reverse_kept()
        else:
            ws_bytes = int(V.lib().vdwlb_adjoint_workspace_bytes(plan.handle, max(segs[:n_rec])))
            if os.environ.get("VDWLB_ADJ_SERIAL") != "1":
                _reverse_overlapped(plan, ctx.ckpts, segs[:n_rec], fbar, pbar, ws_bytes, dev, first=reverse_kept)
            else:
                reverse_kept()
                ws = torch.empty(ws_bytes // 8 + 1, dtype=torch.float64, device=dev)
                for ck, m in zip(reversed(ctx.ckpts), reversed(segs[:n_rec])):
                    V.check(V.lib().vdwlb_adjoint_segment(plan.handle, ck.data_ptr(), int(m), fbar.data_ptr(),
                                                          ws.data_ptr(), pbar.data_ptr(), s), "vdwlb_adjoint_segment")
        g = pbar.cpu().numpy()
        C = spec.C
        pairs = theta_layout(C)
        na = len(pairs)
        k_hat = np.asarray(spec.k_hat)
        dkappa = sum(g[1 + na + C + q] * k_hat[c, d] for q, (c, d) in enumerate(pairs))
        grad = np.concatenate([g[:1 + na + C], [dkappa]])
        return torch.as_tensor(grad, dtype=ctx.theta_dtype, device=ctx.theta_device), None, None


_TUNED = {}


def _apply_schedule(plan, spec: Spec, bufs, stream) -> None:
    """Set the sweep schedule of the forward and the recompute: an explicit
    index, the plan's default (None), or the autotuner's choice for this
    lattice shape, component count and kernel variant, timed on the first
    call (on the initial state in bufs[0], overwriting only bufs[1]) and
    kept for later calls."""
    if spec.schedule is None:
        return
    if spec.schedule != "auto":
        V.check(V.lib().vdwlb_set_schedule(plan.handle, int(spec.schedule)), "vdwlb_set_schedule")
        return
    key = (bufs[0].device.index, spec.nx, spec.ny, spec.C, spec.tau == 1.0, int(spec.force))
    if key not in _TUNED:
        k = ctypes.c_int32()
        V.check(V.lib().vdwlb_autotune(plan.handle, bufs[0].data_ptr(), bufs[1].data_ptr(), stream, ctypes.byref(k)),
                "vdwlb_autotune")
        _TUNED[key] = k.value
    else:
        V.check(V.lib().vdwlb_set_schedule(plan.handle, _TUNED[key]), "vdwlb_set_schedule")


_AUX_STREAMS = {}


def _aux_stream(dev):
    """The second stream of the backward pass on device dev (default priority),
    created once per device."""
    d = torch.device(dev)
    key = d.index if d.index is not None else torch.cuda.current_device()
    if key not in _AUX_STREAMS:
        _AUX_STREAMS[key] = torch.cuda.Stream(device=key)
    return _AUX_STREAMS[key]


def _reverse_overlapped(plan, ckpts, segs, fbar, pbar, ws_bytes, dev, first=None):
    """Reverse the segments from the last to the first with the forward
    recompute of segment k - 1 on a second stream, into a second workspace,
    while the reverse sweep of segment k runs on the current stream.  first,
    if given, enqueues a reverse sweep that precedes them on the current
    stream (one that needs no recompute); the recompute of the last segment
    here runs beside it.  The reverse sweeps run in the same order on one
    stream as the one-stream loop, so the results are the same bit for bit."""
    lib = V.lib()
    main = torch.cuda.current_stream(dev)
    aux = _aux_stream(dev)
    ws = [torch.empty(ws_bytes // 8 + 1, dtype=torch.float64, device=dev) for _ in range(2)]
    aux.wait_stream(main)  # checkpoints and workspaces are ready
    freed = [None, None]  # per workspace: the end of the last reverse sweep that reads it

    def recompute(k):
        j = k % 2
        if freed[j] is not None:
            aux.wait_event(freed[j])
        V.check(lib.vdwlb_adjoint_recompute(plan.handle, ckpts[k].data_ptr(), int(segs[k]), ws[j].data_ptr(),
                                            aux.cuda_stream), "vdwlb_adjoint_recompute")
        ev = torch.cuda.Event()
        ev.record(aux)
        return ev

    ready = recompute(len(segs) - 1)
    if first is not None:
        first()
    for k in range(len(segs) - 1, -1, -1):
        nxt = recompute(k - 1) if k > 0 else None
        main.wait_event(ready)
        V.check(lib.vdwlb_adjoint_reverse(plan.handle, int(segs[k]), fbar.data_ptr(), ws[k % 2].data_ptr(),
                                          pbar.data_ptr(), main.cuda_stream), "vdwlb_adjoint_reverse")
        ev = torch.cuda.Event()
        ev.record(main)
        freed[k % 2] = ev
        ready = nxt
    # every use of the workspaces on the second stream ends before the last
    # reverse sweep starts, so the current stream may reuse their memory


def run_and_grad(theta, rho0, spec: Spec, loss_fn):
    """Loss of the final densities and its gradient with respect to theta."""
    t = torch.as_tensor(theta, dtype=torch.float64).clone().requires_grad_(True)
    rho = VdwLBFunction.apply(t, rho0, spec)
    loss = loss_fn(rho)
    loss.backward()
    return float(loss.detach().cpu()), t.grad.detach().cpu().numpy()
