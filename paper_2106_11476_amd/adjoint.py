"""Gradient of a receiver-trace misfit with respect to the sound-speed map.

Sec. 5 names full waveform inversion as the extension of the method; the
memory-variable recursion dissipates, so the gradient needs the transpose of
the discrete step rather than a backwards run of it.  libfw2 implements that
transpose as hand-written reverse-step kernels (fw2_adjoint_step): the exact
transpose of one step of the time-centred scheme, linearised about the
forward state at the step's input.  This module drives them from a
torch.autograd.Function:

  forward   runs the simulation, keeping one state block (p, v, psi1, psi2)
            every `checkpoint_every` steps in HBM, and returns
            J = 1/2 sum_n sum_r (trace[n, r] - obs[n, r])^2;
  backward  walks the checkpoint segments from the last to the first,
            recomputes the segment's states from its checkpoint (forward
            kernels), then runs the reverse steps of the segment with the
            residual rows as the adjoint sources, and returns dJ/dc.

Memory: ceil(n / K) checkpoint blocks plus K recompute blocks; the default
K = ceil(sqrt(n)) balances the two (one extra forward pass in total).  The
recompute steps out of place into the segment's blocks (fw2_step_into), so no
state is copied per step, and replays one HIP graph per segment.
"""
import math

import numpy as np

from . import fw2


def _problem_with_c(prob, c):
    """prob with its sound speed replaced by c.  The stencil's Courant number
    and the boundary layer's reference speed are fixed inputs of the scheme
    (taken from prob, or from prob.c's maximum where prob leaves them unset),
    so c enters the step only through kappa0 = 1/(rho c^2)."""
    fields = {k: getattr(prob, k) for k in prob.__dataclass_fields__}
    cmax = float(np.max(prob.c))
    if not fields["fd_r"]:
        fields["fd_r"] = cmax * prob.dt / prob.h
    if not fields["pml_cp"]:
        fields["pml_cp"] = cmax
    fields["c"] = np.asarray(c, np.float64).reshape(np.asarray(prob.c).shape)
    return type(prob)(**fields)


def _misfit_function():
    import torch

    class SoundSpeedMisfit(torch.autograd.Function):
        @staticmethod
        def forward(ctx, c, obs, prob, n_steps, checkpoint_every):
            n = int(n_steps)
            if n < 1:
                raise ValueError("n_steps must be at least 1")
            K = int(checkpoint_every) if checkpoint_every else int(math.ceil(math.sqrt(n)))
            K = max(1, min(K, n))
            if prob.relax_scheme != fw2.RELAX_CENTRED:
                raise fw2.Fw2Error(6, "the adjoint is derived for the time-centred memory scheme")
            if getattr(prob, "stencil_mode", fw2.STENCIL_GLOBAL) != fw2.STENCIL_GLOBAL:
                raise fw2.Fw2Error(6, "the adjoint is derived for global stencil weights")
            p = _problem_with_c(prob, c.detach().cpu().numpy())
            dev = obs.device
            dom = fw2.Domain(p, device=dev, stream=torch.cuda.current_stream(dev))
            if len(p.src_idx):
                dom.add_source(p.src_idx, p.src_sig, p.src_w, p.signals)
            has_rcv = len(p.rcv_idx) > 0
            if has_rcv:
                dom.add_receivers(p.rcv_idx, n)
            n_seg = (n + K - 1) // K
            ckpts = dom.new_state_buffer(n_seg)
            for s in range(n_seg):
                dom.save_state(ckpts[s])
                dom.step(min(K, n - s * K))
            if has_rcv:
                residual = (dom.trace[:n] - obs[:n].to(torch.float32)).contiguous()
                J = 0.5 * (residual.double() ** 2).sum()
            else:
                residual = None
                J = torch.zeros((), dtype=torch.float64, device=dev)
            ctx.dom, ctx.ckpts, ctx.residual, ctx.K, ctx.n = dom, ckpts, residual, K, n
            ctx.c_meta = (c.shape, c.dtype, c.device)
            return J

        @staticmethod
        def backward(ctx, gJ):
            dom, ckpts, K, n = ctx.dom, ctx.ckpts, ctx.K, ctx.n
            res = None if ctx.residual is None else (ctx.residual * gJ.to(torch.float32)).contiguous()
            dom.adjoint_begin()
            # seg[k] holds the state at step n0 + k: the segment's checkpoint
            # copied into seg[0], the others recomputed from it out of place
            # (fixed buffers, so every full segment replays one HIP graph)
            seg = dom.new_state_buffer(K)
            for s in reversed(range(ckpts.shape[0])):
                n0 = s * K
                m = min(K, n - n0)
                with torch.cuda.stream(dom.stream):
                    seg[0].copy_(ckpts[s])
                if m > 1:
                    dom.set_current_step(n0)
                    dom.step_into(m - 1, seg[0], seg[1:])
                for k in reversed(range(m)):
                    dom.adjoint_step(seg[k], n0 + k, None if res is None else res[n0 + k],
                                     prev=seg[k - 1] if k > 0 else None)
            g = dom.adjoint_gradient()
            shape, dtype, device = ctx.c_meta
            grad = g.reshape(shape).to(device=device, dtype=dtype)
            dom.destroy_domain()
            ctx.dom = ctx.ckpts = ctx.residual = None
            return grad, None, None, None, None

    return SoundSpeedMisfit


_FN = None


def misfit(c, obs, prob, n_steps, checkpoint_every=None):
    """J(c) = 1/2 ||trace(c) - obs||^2 over n_steps steps, differentiable in c.

    c    -- torch tensor of the grid's shape (prob.c's layout, x fastest)
    obs  -- torch device tensor [n_steps, n_rcv]; its device runs the solver
    prob -- workloads.Problem-like inputs (its c is replaced by `c`); the
            time-centred memory scheme is required
    """
    global _FN
    if _FN is None:
        _FN = _misfit_function()
    return _FN.apply(c, obs, prob, n_steps, checkpoint_every)
