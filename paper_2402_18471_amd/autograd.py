"""torch.autograd.Function around repeated coagulation calls, with the
hand-written adjoint of libcoag (coag_step_backward) as its backward.

Forward: n_steps calls of coag_rates + coag_step (ADAPTIVE, or FIXED with
`fixed_nsub` equal sub-steps per call), recording each call's accepted step
sizes and keeping the state every `ckpt_every` calls.  The split-BF16 form
takes FP32 rates in the 16-cell-blocked layout, as its step streams them.
Backward: for each checkpoint segment, from the last to the first, the
segment is recomputed from its checkpoint with the recorded step sizes
(REPLAY, so the step sequence is exactly the one the forward pass took) and
the adjoint runs through its calls in reverse, in the forward's precision:
FP64, or split BF16 (the transposed gain contraction as split-BF16 matrix
products, everything else FP64).  Gradients are returned for the initial
density, alpha and v_frag (per cell); the other inputs are not
differentiated.  Each call's step log is kept only as wide as its longest
step sequence.
"""
from __future__ import annotations

import torch

from . import _lib as L


def _rates(coag, cells, v_dust, vf, prec, out=None):
    """The rates one call's step reads, as the (Kc, Kf) coag_step takes: FP32,
    16-cell-blocked for the split form (both kinds in Kc, Kf None); FP64
    [C][P] for the FP64 form; into `out` (from an earlier call) when given,
    so that a run holds one set of rate arrays."""
    Kc, Kf = out if out is not None else (None, None)
    if prec == L.PREC_SPLIT_BF16:
        return coag.coag_rates_blocked(cells, v_dust, vf, dtype=torch.float32, K=Kc), None
    return coag.coag_rates(cells, v_dust, vf, Kc=Kc, Kf=Kf)


class CoagStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, alpha, v_frag, coag, cells, v_dust, dt, n_steps, ckpt_every=20,
                prec=L.PREC_FP64, max_sub=64, fixed_nsub=None, rtol=1e-2, atol_rel=1e-10,
                progress=None):
        C = rho0.shape[0]
        dev = rho0.device
        cells = dict(cells)
        cells["alpha"] = alpha.detach().contiguous()
        vf = v_frag.detach().contiguous()
        rho = rho0.detach().clone()
        h = torch.zeros(C, dtype=torch.float64, device=dev)
        log = torch.zeros((C, max_sub), dtype=torch.float64, device=dev)
        logs, nsubs, ckpts = [], torch.zeros((n_steps, C), dtype=torch.int32, device=dev), []
        mode = L.ADAPTIVE if fixed_nsub is None else L.FIXED
        if fixed_nsub is not None:
            if not 1 <= int(fixed_nsub) <= max_sub:
                raise ValueError("fixed_nsub must lie in [1, max_sub]")
            nsubs.fill_(int(fixed_nsub))
        K = None
        for s in range(n_steps):
            if s % ckpt_every == 0:
                ckpts.append(rho.clone())
            K = _rates(coag, cells, v_dust, vf, prec, K)
            Kc, Kf = K
            r = coag.coag_step(rho, Kc, Kf, dt, h=h, mode=mode, prec=prec, rtol=rtol,
                               atol_rel=atol_rel, max_sub=max_sub, nsub=nsubs[s], h_log=log,
                               check_status=False)
            st = r["status"]
            if bool((st != 0).any()):
                bad = int((st != 0).sum())
                raise RuntimeError(f"coag_step: {bad} cells failed at call {s} "
                                   f"(status codes {sorted(set(st.tolist()))})")
            width = max(1, int(nsubs[s].max()))
            logs.append(log[:, :width].clone())
            if progress is not None and (s + 1) % ckpt_every == 0:
                progress("forward", s + 1, n_steps)
        del K, Kc, Kf, r
        ctx.progress = progress
        ctx.coag, ctx.cells, ctx.v_dust, ctx.vf = coag, cells, v_dust, vf
        ctx.dt, ctx.n_steps, ctx.ckpt_every, ctx.prec = dt, n_steps, ckpt_every, prec
        ctx.logs, ctx.nsubs, ctx.ckpts = logs, nsubs, ckpts
        return rho

    @staticmethod
    def backward(ctx, g_out):
        coag, cells, v_dust, vf = ctx.coag, ctx.cells, ctx.v_dust, ctx.vf
        g = g_out.detach().contiguous().clone()
        C = g.shape[0]
        g_alpha = torch.zeros(C, dtype=torch.float64, device=g.device)
        g_vfrag = torch.zeros_like(g_alpha)
        n, E = ctx.n_steps, ctx.ckpt_every
        K = None
        for seg in range((n + E - 1) // E - 1, -1, -1):
            s0, s1 = seg * E, min((seg + 1) * E, n)
            # recompute the segment from its checkpoint, keeping each call's start state
            rho = ctx.ckpts[seg].clone()
            starts = []
            for s in range(s0, s1):
                starts.append(rho.clone())
                if s + 1 < s1:
                    K = _rates(coag, cells, v_dust, vf, ctx.prec, K)
                    coag.coag_step(rho, K[0], K[1], ctx.dt, mode=L.REPLAY, prec=ctx.prec,
                                   nsub=ctx.nsubs[s], h_log=ctx.logs[s])
            for s in range(s1 - 1, s0 - 1, -1):
                gi, ga, gv = coag.coag_step_backward(starts[s - s0], cells, v_dust, vf,
                                                     ctx.logs[s], ctx.nsubs[s], g,
                                                     prec=ctx.prec)
                g = gi
                g_alpha += ga
                g_vfrag += gv
            if ctx.progress is not None:
                ctx.progress("backward", n - s0, n)
        return (g, g_alpha, g_vfrag) + (None,) * 12


def coag_evolve(coag, rho0, alpha, v_frag, cells, v_dust, dt, n_steps, ckpt_every=20,
                prec=L.PREC_FP64, max_sub=64, fixed_nsub=None, rtol=1e-2, atol_rel=1e-10,
                progress=None):
    """Differentiable n_steps coagulation calls (see CoagStep).  progress, if
    given, is called as progress(phase, calls_done, n_steps) after every
    checkpoint segment of either pass (phase "forward" or "backward"; the
    backward counts the calls it has gone back through)."""
    return CoagStep.apply(rho0, alpha, v_frag, coag, cells, v_dust, dt, n_steps, ckpt_every,
                          prec, max_sub, fixed_nsub, rtol, atol_rel, progress)
