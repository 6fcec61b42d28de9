"""The smoothed MWU potential as a ``torch.autograd.Function``.

Phi(x) = smax_eta(P x) - smin_eta(C x) (Section 4.1; Section 2.2 for smax,
smin and their gradients) is evaluated by the library's kernels on the GPU,
and its backward is the library's hand-written transpose-product kernel: the
gradient P^T grad smax(Px) - C^T grad smin(Cx) is exactly the g - h that an
MWU step moves along.  PyTorch provides only the device memory and the
stream; nothing is computed by torch operators.

Usage::

    s = paper_2307_03307_amd.dominating_set(ptr, col, n, precision=FP64, flags=FLAG_GENERIC)
    pot = MwuPotential.bind(s, param=M)          # starts a probe at param M
    x = torch.rand(n, dtype=torch.float64, device="cuda", requires_grad=True)
    y = pot(x)                                   # 0-dim tensor
    y.backward()                                 # x.grad = g - h
"""
from __future__ import annotations

import torch


class _PotentialFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, solver) -> torch.Tensor:
        if x.device.type != "cuda" or x.dtype != torch.float64 or not x.is_contiguous():
            raise ValueError("x must be a contiguous float64 CUDA tensor")
        if x.numel() != solver.num_variables:
            raise ValueError(f"x has {x.numel()} entries, the LP has {solver.num_variables} variables")
        stream = torch.cuda.current_stream(x.device).cuda_stream
        val = solver.potential_forward(x.data_ptr(), stream)
        ctx.solver = solver
        ctx.save_for_backward(x)
        return torch.tensor(val, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (x,) = ctx.saved_tensors
        grad = torch.empty_like(x)
        stream = torch.cuda.current_stream(x.device).cuda_stream
        ctx.solver.potential_backward(x.data_ptr(), float(grad_out.item()), grad.data_ptr(), stream)
        return grad, None


class MwuPotential:
    """Callable wrapper binding a solver handle at a fixed param (M or D)."""

    def __init__(self, solver, param: float):
        self.solver = solver
        self.param = float(param)
        solver.probe_begin(self.param)

    @classmethod
    def bind(cls, solver, param: float) -> "MwuPotential":
        return cls(solver, param)

    def __call__(self, x: torch.Tensor) -> torch.Tensor:
        return _PotentialFn.apply(x, self.solver)
