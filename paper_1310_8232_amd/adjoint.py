"""Misfit and gradient with respect to squared slowness, with checkpointed
forward wavefields: the backward (reverse-time) pass that RTM runs around the
"3D model" step of Algorithm 1.

Orchestration only: every arithmetic step (forward steps, receiver samples,
residuals and the FP64 misfit, adjoint steps, the FP64 gradient
accumulation) is a library kernel reached through the C ABI.

Conventions. Forward: u^{n+1} = 2u^n - u^{n-1} + kappa L u^n + sources,
u^0 = u^{-1} = 0, n = 0..nt-1; traces row k-1 holds u^k at the receivers.
Misfit J = 1/2 sum (traces - observed)^2. The adjoint variable is
mu = kappa * lambda (see stencil_adjoint_step); the gradient is
dJ/dm = -(h^2/dt^2) sum_n mu^{n+1} (u^{n+1} - 2u^n + u^{n-1}), m = 1/v^2.

Checkpoints: (u^n, u^{n-1}) every C steps during the forward pass; the
backward pass recomputes each segment of C steps from its checkpoint into a
buffer of C+2 wavefields (no copies: the out-of-place step writes each level
into its slot), then runs the segment's adjoint steps in reverse. With C = 0
every level is kept (nt + 2 wavefields; 31 GiB at 256^3 and 500 steps) and
nothing is recomputed.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import (Propagator, StencilSrc, make_src, stencil_gradient_terms, stencil_misfit, stencil_sample,
               stencil_step, stencil_step_to, stencil_stream_probe)


@dataclass
class Survey:
    """Sources (device idx [n] int64, amp [nt, n] float32) and receivers
    (device idx [nrec] int64) of one shot."""
    src_idx: torch.Tensor
    src_amp: torch.Tensor
    rec_idx: torch.Tensor

    @property
    def nt(self) -> int:
        return int(self.src_amp.shape[0])

    def src(self) -> StencilSrc:
        return make_src(self.src_idx, self.src_amp)


def _copy(dst: torch.Tensor, src: torch.Tensor):
    stencil_stream_probe(src, None, None, dst, src.numel() * 4)


def forward(prop: Propagator, survey: Survey, checkpoint_every: int = 0, keep_levels: bool = False):
    """Forward pass from rest. Returns (traces [nt, nrec] float32,
    checkpoints {n: (u^n, u^{n-1})} every `checkpoint_every` steps (none if 0),
    final (u^nt, u^{nt-1})).

    keep_levels=True instead keeps every time level: one [nt+2, nz, ny, nx]
    buffer with u^n in row n+1, each step written out of place into its own
    row (no copies); the checkpoint dict is then {"levels": buffer}."""
    nt = survey.nt
    src = survey.src()
    if keep_levels:
        levels = torch.empty((nt + 2,) + tuple(prop.store_shape), device=prop.device)
        levels[0].zero_()
        levels[1].zero_()
        traces = torch.empty((nt, survey.rec_idx.numel()), device=prop.device)
        for n in range(nt):
            stencil_step_to(prop.ctx, prop.kappa, levels[n + 1], levels[n], levels[n + 2], n, src)
            stencil_sample(prop.ctx, levels[n + 2], survey.rec_idx, traces[n])
        return traces, {"levels": levels}, (levels[nt + 1], levels[nt])
    a = torch.zeros(prop.store_shape, device=prop.device)
    b = torch.zeros(prop.store_shape, device=prop.device)
    traces = torch.empty((nt, survey.rec_idx.numel()), device=prop.device)
    ckpts = {}
    for n in range(nt):
        if checkpoint_every and n % checkpoint_every == 0:
            ca, cb = torch.empty_like(a), torch.empty_like(b)
            _copy(ca, a)
            _copy(cb, b)
            ckpts[n] = (ca, cb)
        stencil_step(prop.ctx, prop.kappa, a, b, n, src)
        a, b = b, a
        stencil_sample(prop.ctx, a, survey.rec_idx, traces[n])
    return traces, ckpts, (a, b)


def misfit(traces: torch.Tensor, observed: torch.Tensor):
    """(J as a float64 device scalar, residual traces float32)."""
    resid = torch.empty_like(traces)
    J = torch.zeros((), dtype=torch.float64, device=traces.device)
    stencil_misfit(traces, observed.contiguous(), resid, J)
    return J, resid


def backward(prop: Propagator, survey: Survey, resid: torch.Tensor, ckpts: dict, checkpoint_every: int):
    """Adjoint pass: returns dJ/dm (float64, in the stored layout: prop.grid() gives the grid points)."""
    nt = survey.nt
    C = checkpoint_every
    src = survey.src()
    rsrc = make_src(survey.rec_idx, resid)
    grad = torch.zeros(prop.store_shape, dtype=torch.float64, device=prop.device)
    # Four buffers of mu: the pair (mu^{k+1}, mu^{k+2}) that the next adjoint
    # step reads, and room for up to four new levels whose gradient terms are
    # then added in one pass.
    bufs = [torch.zeros(prop.store_shape, device=prop.device) for _ in range(4)]
    state = [bufs[0], bufs[1]]  # [mu^{k+1}, mu^{k+2}]

    def adjoint_range(k_hi, k_lo, level):
        # Adjoint steps k = k_hi .. k_lo + 1 with level(j) = u^j, in groups of
        # up to four: each step writes mu^{k-j} out of place (the step with the
        # residuals of row k-j-1 injected), then stencil_gradient_terms adds the
        # group's terms in step order (the bits of one accumulation per step).
        k = k_hi
        while k > k_lo:
            m = min(4, k - k_lo)
            cur, prev = state
            free = [x for x in bufs if x is not cur and x is not prev]
            outs = (free + [prev, cur])[:m]  # prev is read last by step 0, cur by step 1
            c, pv = cur, prev
            for j in range(m):
                stencil_step_to(prop.ctx, prop.kappa, c, pv, outs[j], k - j - 1, rsrc)  # mu^{k-j}
                c, pv = outs[j], c
            stencil_gradient_terms(prop.ctx, outs, [level(k - i) for i in range(m + 2)], grad)
            state[0], state[1] = c, pv
            k -= m

    if "levels" in ckpts:  # every level kept: no recompute
        L = ckpts["levels"]  # L[n + 1] = u^n
        adjoint_range(nt, 0, lambda j: L[j + 1])
        return grad
    buf = torch.empty((C,) + tuple(prop.store_shape), device=prop.device)
    for n0 in sorted(ckpts, reverse=True):
        n1 = min(n0 + C, nt)
        u0, um1 = ckpts[n0]
        levels = [um1, u0] + [buf[i] for i in range(n1 - n0)]  # levels[j] = u^{n0-1+j}
        for n in range(n0, n1):
            j = n - n0 + 1
            stencil_step_to(prop.ctx, prop.kappa, levels[j], levels[j - 1], levels[j + 1], n, src)
        adjoint_range(n1, n0, lambda j, n0=n0, levels=levels: levels[j - n0 + 1])  # levels[j - n0 + 1] = u^j
    return grad


def misfit_gradient(prop: Propagator, survey: Survey, observed: torch.Tensor, checkpoint_every: int = 50):
    """(J float64 device scalar, dJ/dm float64 field, traces).

    checkpoint_every = C > 0 keeps (u^n, u^{n-1}) every C steps and recomputes
    each segment in the backward pass (memory: 2 nt/C + C wavefields);
    checkpoint_every = 0 keeps every level instead (nt + 2 wavefields, no
    recompute), which HBM holds for moderate grids and step counts."""
    if checkpoint_every < 0:
        raise ValueError("checkpoint_every must be >= 0")
    traces, ckpts, _ = forward(prop, survey, checkpoint_every, keep_levels=checkpoint_every == 0)
    J, resid = misfit(traces, observed)
    grad = backward(prop, survey, resid, ckpts, checkpoint_every)
    return J, grad, traces


class SlownessMisfit(torch.autograd.Function):
    """J(m) for squared slowness m (float32 CUDA tensor [nz, ny, nx]).

    Forward: kappa from m, forward pass with checkpoints, residuals, misfit.
    Backward: the adjoint pass; returns grad_output * dJ/dm (cast to m's dtype).
    """

    @staticmethod
    def forward(ctx, m, survey: Survey, observed, h: float, dt: float, radius: int = 4,
                checkpoint_every: int = 50, tile=None):
        prop = Propagator(m.detach().contiguous(), h, dt, radius, slowness2=True, tile=tile)
        if checkpoint_every < 0:
            raise ValueError("checkpoint_every must be >= 0")
        traces, ckpts, _ = forward(prop, survey, checkpoint_every, keep_levels=checkpoint_every == 0)
        J, resid = misfit(traces, observed)
        ctx.state = (prop, survey, resid, ckpts, checkpoint_every)
        return J

    @staticmethod
    def backward(ctx, gJ):
        prop, survey, resid, ckpts, C = ctx.state
        grad = backward(prop, survey, resid, ckpts, C)
        ctx.state = None
        return (gJ * grad).to(torch.float32), None, None, None, None, None, None, None
