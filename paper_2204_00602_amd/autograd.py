"""torch.autograd wrappers: amplitudes of a SLOS plan and the MZI mesh.

Forward and backward both run in the HIP library (slos_amplitudes /
slos_backward, slos_mesh_unitary / slos_mesh_backward); torch only records the
graph.  A plan keeps the layers of its last forward call, so each amplitude
node checks that no other forward ran on its plan before its backward.
"""
from __future__ import annotations

import torch

from . import slos


class SlosAmplitudes(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, plan):
        a = plan.amplitudes(U)
        ctx.plan = plan
        ctx.token = plan.forward_count
        ctx.save_for_backward(U)
        return a

    @staticmethod
    def backward(ctx, grad_a):
        (U,) = ctx.saved_tensors
        if ctx.plan.forward_count != ctx.token:
            raise RuntimeError("the plan ran another forward pass before this backward; "
                               "use one plan per differentiated amplitude call")
        gU = ctx.plan.backward(U, grad_a.to(U.dtype).contiguous())
        return gU, None


class SlosAmplitudesMany(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, plan):
        a = plan.amplitudes_many(U)
        ctx.plan = plan
        ctx.token = plan.forward_count
        ctx.save_for_backward(U)
        return a

    @staticmethod
    def backward(ctx, grad_a):
        (U,) = ctx.saved_tensors
        if ctx.plan.forward_count != ctx.token:
            raise RuntimeError("the plan ran another forward pass before this backward; "
                               "use one plan per differentiated amplitude call")
        gU = ctx.plan.backward_many(U, grad_a.to(U.dtype).contiguous())
        return gU, None


class MeshUnitary(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phases, m, dtype):
        ctx.save_for_backward(phases)
        return slos.mesh_unitary(phases, m, dtype)

    @staticmethod
    def backward(ctx, grad_U):
        (phases,) = ctx.saved_tensors
        return slos.mesh_backward(phases, grad_U), None, None


def amplitudes(plan, U):
    """Differentiable a(S) for all S (plan built with keep_layers=True)."""
    return SlosAmplitudes.apply(U, plan)


def amplitudes_many(plan, U):
    """Differentiable a(S) for a batch of unitaries (batch x m x m) through one
    plan built with keep_layers=True and max_batch >= batch: batch x M."""
    return SlosAmplitudesMany.apply(U, plan)


def mesh(phases, m: int, dtype: str = "c64"):
    """Differentiable U (batch x m x m) of the rectangular MZI mesh."""
    return MeshUnitary.apply(phases, m, dtype)
