"""The wave solver as a differentiable torch operator.

The paper composes PDE operators and losses into a graph whose gradient is
taken by the adjoint method, each operator providing a forward and an adjoint
(Sec. 2.2: every function is an Operator with forward and adjoint; a Variable
with needs_grad collects its gradient).  Here the same role is played by a
torch.autograd.Function: forward runs the HIP forward solve and keeps binomial
checkpoints of the forward wavefield in a device workspace; backward runs the
HIP adjoint solve fused with the imaging condition and returns dJ/dvp (and,
when asked, dJ/dwavelet) for any loss torch builds on the traces.
"""
from __future__ import annotations

import torch

from . import _abi
from ._abi import STRIDE_MODE_GRADIENT, Plan


class StrideWave(torch.autograd.Function):
    """traces = StrideWave.apply(vp, wavelet, plan, budget_bytes)

    vp: physical-shape float32 CUDA tensor; wavelet: [nsrc][nt] float32.
    budget_bytes caps the checkpoint workspace (0 = keep every state).
    The workspace holds the forward checkpoints until backward has consumed
    them, so backward runs once per forward (no retain_graph).
    """

    @staticmethod
    def forward(ctx, vp, wavelet, plan: Plan, budget_bytes: int = 0):
        vp = vp.contiguous()
        wavelet = wavelet.contiguous()
        ws = plan.workspace(STRIDE_MODE_GRADIENT, budget_bytes, device=vp.device)
        traces = plan.forward_save(vp, wavelet, ws)
        ctx.save_for_backward(vp, wavelet)
        ctx.plan = plan
        ctx.ws = ws
        return traces

    @staticmethod
    def backward(ctx, grad_traces):
        if ctx.ws is None:
            raise RuntimeError("StrideWave.backward can run once per forward: the checkpoint "
                               "workspace has been consumed (retain_graph is not supported)")
        vp, wavelet = ctx.saved_tensors
        want_wav = bool(ctx.needs_input_grad[1])
        dvp, dwav = ctx.plan.backward(vp, wavelet, grad_traces.contiguous(), ctx.ws,
                                      want_dwavelet=want_wav)
        ctx.ws = None
        return (dvp if ctx.needs_input_grad[0] else None), dwav, None, None


def wave_traces(vp, wavelet, plan: Plan, budget_bytes: int = 0):
    """Differentiable receiver traces of one shot."""
    return StrideWave.apply(vp, wavelet, plan, budget_bytes)


class WavePropagator(torch.nn.Module):
    """Module form: holds a plan (grid + shot geometry); forward(vp, wavelet)."""

    def __init__(self, plan: Plan, budget_bytes: int = 0):
        super().__init__()
        self.plan = plan
        self.budget_bytes = budget_bytes

    def forward(self, vp, wavelet):
        return StrideWave.apply(vp, wavelet, self.plan, self.budget_bytes)


__all__ = ["StrideWave", "wave_traces", "WavePropagator", "_abi"]
