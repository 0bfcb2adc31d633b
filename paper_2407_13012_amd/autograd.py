"""PyTorch autograd over the library's adjoint gradient.

``qaoa_expectation_fn(gamma, beta, handle)`` returns E(gamma, beta) as a
0-dimensional float64 tensor.  The forward call always runs the fused forward
sweep (``qaoa_evaluate``), which leaves the final state in the handle.  The
backward call runs only the adjoint reverse sweep from that state
(``qaoa_gradient_from_state``: lam = C phi, then the inverse layers with the
<lam|H_k|phi> terms, Sec. II-B, IV-C) and scales the 2p partials by the
incoming gradient; a forward whose result is never differentiated costs one
forward sweep.  If the handle's state has been replaced in between (another
evaluation on the same handle), backward recomputes it with the full
``qaoa_gradient``.  All arithmetic runs in the HIP library; torch only carries
the angles and the result.
"""
from __future__ import annotations

import numpy as np
import torch

from ._binding import (QaoaError, QaoaHandle, qaoa_evaluate, qaoa_gradient,
                       qaoa_gradient_from_state)

_NO_STATE = 4  # QAOA_ERR_NO_STATE


def _as_np(t: torch.Tensor) -> np.ndarray:
    return t.detach().to("cpu", torch.float64).contiguous().numpy()


class QaoaExpectation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma: torch.Tensor, beta: torch.Tensor, handle):
        raw = handle.raw if isinstance(handle, QaoaHandle) else handle
        if gamma.shape != beta.shape or gamma.dim() != 1:
            raise ValueError("gamma and beta must be 1-D tensors of equal length")
        g, b = _as_np(gamma), _as_np(beta)
        E = qaoa_evaluate(raw, g, b)
        ctx.raw, ctx.angles = raw, (g.copy(), b.copy())
        return torch.tensor(E, dtype=torch.float64, device=gamma.device)

    @staticmethod
    def backward(ctx, grad_E: torch.Tensor):
        g, b = ctx.angles
        try:
            dg, db = qaoa_gradient_from_state(ctx.raw, g, b)
        except QaoaError as e:
            if e.status != _NO_STATE:
                raise
            _, dg, db = qaoa_gradient(ctx.raw, g, b)
        dev = grad_E.device
        dg = torch.from_numpy(dg).to(dev, grad_E.dtype)
        db = torch.from_numpy(db).to(dev, grad_E.dtype)
        return grad_E * dg, grad_E * db, None


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
