"""PyTorch autograd over the library's adjoint gradient.

``qaoa_expectation_fn(gamma, beta, handle)`` returns E(gamma, beta) as a
0-dimensional float64 tensor.  When either angle tensor requires a gradient,
the forward call runs ``qaoa_gradient`` -- the expectation and all 2p partial
derivatives from one forward sweep plus the adjoint reverse sweep, with layer
states recomputed by inverse layers (Sec. II-B, IV-C) -- and backward only
scales the stored derivatives by the incoming gradient.  Without gradients it
runs the cheaper fused forward sweep (``qaoa_evaluate``).  All arithmetic runs
in the HIP library; torch only carries the angles and the result.
"""
from __future__ import annotations

import numpy as np
import torch

from ._binding import QaoaHandle, qaoa_evaluate, qaoa_gradient


def _as_np(t: torch.Tensor) -> np.ndarray:
    return t.detach().to("cpu", torch.float64).contiguous().numpy()


class QaoaExpectation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma: torch.Tensor, beta: torch.Tensor, handle):
        raw = handle.raw if isinstance(handle, QaoaHandle) else handle
        g, b = _as_np(gamma), _as_np(beta)
        if gamma.shape != beta.shape or gamma.dim() != 1:
            raise ValueError("gamma and beta must be 1-D tensors of equal length")
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            E, dg, db = qaoa_gradient(raw, g, b)
            ctx.save_for_backward(torch.from_numpy(dg).to(gamma.device),
                                  torch.from_numpy(db).to(beta.device))
        else:
            E = qaoa_evaluate(raw, g, b)
        return torch.tensor(E, dtype=torch.float64, device=gamma.device)

    @staticmethod
    def backward(ctx, grad_E: torch.Tensor):
        dg, db = ctx.saved_tensors
        return grad_E * dg.to(grad_E.dtype), grad_E * db.to(grad_E.dtype), None


def qaoa_expectation_fn(gamma: torch.Tensor, beta: torch.Tensor, handle) -> torch.Tensor:
    """E(gamma, beta) with autograd support (see the module docstring)."""
    return QaoaExpectation.apply(gamma, beta, handle)


class QaoaExpectationModule(torch.nn.Module):
    """Angles as parameters; ``forward()`` returns E.  Owns its handle."""

    def __init__(self, instance, gamma, beta, precision: str = "c128"):
        super().__init__()
        self.handle = QaoaHandle.from_instance(instance, precision)
        self.gamma = torch.nn.Parameter(torch.as_tensor(np.asarray(gamma, np.float64)))
        self.beta = torch.nn.Parameter(torch.as_tensor(np.asarray(beta, np.float64)))

    def forward(self) -> torch.Tensor:
        return qaoa_expectation_fn(self.gamma, self.beta, self.handle)
