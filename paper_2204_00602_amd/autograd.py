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


class MeshLossGradient:
    """dL/dphases of L = sum_b sum_{S in targets} (P_b(S) - P_t,b(S))^2 for a batch
    of Clements meshes, recorded once into a HIP graph and replayed.

    One replay runs the mesh (phases -> U), the amplitudes of every unitary
    through one plan (slos_amplitudes_many), the loss with the adjoint of the
    recurrence (slos_sq_loss_backward_many: dL/da = 4 (P - P_t) a in the
    PyTorch convention on the targets, zero elsewhere, seeded straight into the
    reverse layers with the targets' normalisation factors, which
    slos_output_scales computes once here) and the mesh adjoint, all library
    kernels on bound buffers: write new phases into `phases` and replay().

    plan: built with keep_layers=True and max_batch >= batch.
    targets: ranks of the target outputs (int64, device); p_target: batch x
    len(targets) FP64 (device).
    """

    def __init__(self, plan, m: int, batch: int, targets, p_target, dtype: str = "c64"):
        dev = torch.device("cuda")
        k = slos.mesh_mzi_count(m)
        self.plan, self.m, self.batch, self.dtype = plan, m, batch, dtype
        cdt = torch.complex64 if dtype == "c64" else torch.complex128
        self.targets = torch.as_tensor(targets, dtype=torch.int64, device=dev).contiguous()
        self.p_target = torch.as_tensor(p_target, dtype=torch.float64, device=dev).reshape(batch, -1).contiguous()
        if self.p_target.shape[1] != self.targets.numel():
            raise ValueError("p_target needs one value per target and batch entry")
        self.phases = torch.zeros((batch, 2 * k), dtype=torch.float64, device=dev)
        self.U = torch.empty((batch, m, m), dtype=cdt, device=dev)
        self.a = torch.empty((batch, plan.num_outputs), dtype=cdt, device=dev)
        self.scales = torch.from_numpy(plan.output_scales(self.targets.cpu().numpy())).to(dev)
        self.grad_U = torch.empty_like(self.U)
        self.grad_phases = torch.empty((batch, 2 * k), dtype=torch.float64, device=dev)
        self.losses = torch.zeros(batch, dtype=torch.float64, device=dev)
        self.graph = None

    def _step(self):
        slos.mesh_unitary(self.phases, self.m, self.dtype, out=self.U)
        self.plan.amplitudes_many(self.U, out=self.a)
        self.plan.sq_loss_backward_many(self.U, self.a, self.targets, self.scales, self.p_target, grad_U=self.grad_U,
                                        loss=self.losses)
        slos.mesh_backward(self.phases, self.grad_U, out=self.grad_phases)

    def eager(self, phases=None):
        """Run the step without the graph; returns the bound grad_phases."""
        if phases is not None:
            self.phases.copy_(phases)
        self._step()
        return self.grad_phases

    def capture(self):
        """Record the step (after two eager warm-up steps on a side stream)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(2):
                self._step()
        torch.cuda.current_stream().wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step()
        return self

    def replay(self, phases=None):
        """Replay the recorded step; returns the bound grad_phases."""
        if self.graph is None:
            raise RuntimeError("capture() first")
        if phases is not None:
            self.phases.copy_(phases)
        self.graph.replay()
        return self.grad_phases

    def loss(self) -> float:
        """L of the last step: the per-instance losses it wrote, summed in order."""
        return float(sum(self.losses.cpu().tolist()))
