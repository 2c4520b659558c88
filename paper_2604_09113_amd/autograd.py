"""Compliance of the lattice as a differentiable torch function.

`Compliance.apply(ctrl, t, solver, prec, rtol, max_iter)` returns the
compliance J_r = f_r^T u_r of every load case r for the control net `ctrl`
[(m ny + 1), (m nx + 1), 2] and the thickness parameters `t` [ny nx] (float64
tensors on the solver's device).  Forward: the library re-assembles, sets up
and solves with this geometry (`lbddc_set_geometry_device`, assemble, setup,
solve).  The gradient is the library's hand-written adjoint
(`lbddc_compliance_gradient_device`): compliance is self-adjoint, so the
adjoint state is u itself and no second solve is needed,
dJ = 2 u^T df - u^T dK u.  It is evaluated in the forward pass, while the
solver still holds this u, and only when an input requires a gradient.

All arithmetic runs in the library's kernels; torch provides the device
buffers and the stream.  The solver must have been created on the current
torch stream, a non-default one (torch.cuda.Stream()): the library then
enqueues on the stream that torch's own reads and writes of the inputs and
outputs use, so no other ordering is needed.  (On torch's default stream the
library would run on a stream of its own, ordered with torch's work only by
the legacy default-stream rules; that case is refused.)
"""
import torch

from . import lbddc


class Compliance(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ctrl, t, solver, prec=lbddc.FP64, rtol=1e-10, max_iter=1000):
        if ctrl.dtype != torch.float64 or t.dtype != torch.float64 or not ctrl.is_cuda or not t.is_cuda:
            raise TypeError("Compliance: ctrl and t must be float64 device tensors")
        cur = torch.cuda.current_stream(ctrl.device)
        if solver.stream is None or solver.stream != cur.cuda_stream:
            raise ValueError("Compliance: the solver must be created on the current (non-default) torch stream")
        nx, ny, p, q, m = solver.shape
        if tuple(ctrl.shape) != (m * ny + 1, m * nx + 1, 2) or tuple(t.shape) != (nx * ny,):
            raise ValueError("Compliance: ctrl or t does not match the solver's problem")
        ctrl_c, t_c = ctrl.detach().contiguous(), t.detach().contiguous()
        solver.set_geometry_device(ctrl_c.data_ptr(), t_c.data_ptr())
        solver.assemble(lbddc.FP64)
        solver.setup(prec)
        solver.solve(rtol=rtol, max_iter=max_iter)
        nrhs = solver.nrhs
        J = torch.empty(nrhs, dtype=torch.float64, device=ctrl.device)
        need = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
        gX = torch.empty((nrhs,) + tuple(ctrl.shape), dtype=torch.float64, device=ctrl.device) if need else None
        gt = torch.empty((nrhs, nx * ny), dtype=torch.float64, device=ctrl.device) if need else None
        solver.compliance_gradient_device(J.data_ptr(), gX.data_ptr() if need else 0, gt.data_ptr() if need else 0)
        if need:
            ctx.save_for_backward(gX, gt)
        return J

    @staticmethod
    def backward(ctx, gJ):
        gX, gt = ctx.saved_tensors
        dctrl = torch.tensordot(gJ, gX, dims=1) if ctx.needs_input_grad[0] else None
        dt = torch.tensordot(gJ, gt, dims=1) if ctx.needs_input_grad[1] else None
        return dctrl, dt, None, None, None, None


def compliance(ctrl, t, solver, prec=lbddc.FP64, rtol=1e-10, max_iter=1000):
    """J[nrhs] = Compliance.apply(ctrl, t, solver, prec, rtol, max_iter)."""
    return Compliance.apply(ctrl, t, solver, prec, rtol, max_iter)
