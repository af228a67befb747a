"""torch.autograd.Function wrappers over the C entry points.

ConsEnergy: E = U(x) per replica; its backward returns dE/dx = -F from the
library's hand-written reverse pass (no torch differentiation is involved).
NCForces: F_NC(theta, x); its backward returns dL/dtheta from the library's
weight-gradient kernels (nnp_nc_weight_grad).  Position derivatives of the
non-conservative forces are not provided: the model is only ever used through
its forces (the paper's reason for it), so a position tensor that requires
grad is rejected.
"""

import torch

from . import nnp


class ConsEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, model, system, nlist, ws):
        """pos: device float64 [3][n]; returns energies float64 [n_rep]."""
        pos = pos.contiguous()
        energy = torch.empty(system.n_rep, dtype=torch.float64, device=pos.device)
        forces = torch.empty(3, system.n, dtype=torch.float32, device=pos.device)
        import ctypes as C
        nnp.check(nnp.lib().nnp_cons_energy_forces(model.handle, C.byref(system.c(pos)), C.byref(nlist.c()),
                                                   nnp._ptr(ws), ws.numel(), nnp._ptr(energy), nnp._ptr(forces),
                                                   nnp._stream()))
        ctx.save_for_backward(forces)
        ctx.rep_of_atom = system.rep_of_atom
        return energy

    @staticmethod
    def backward(ctx, grad_energy):
        (forces,) = ctx.saved_tensors
        scale = grad_energy[ctx.rep_of_atom.long()]  # dL/dE of each atom's replica
        return -(forces.double() * scale[None, :]), None, None, None, None


class NCForces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, pos, model, system, nlist, ws):
        """theta: device float32 [n_weights] (manifest order); pos: device
        float64 [3][n] (not differentiable); returns F_NC float32 [3][n]."""
        if pos.requires_grad:
            raise RuntimeError("NCForces provides weight gradients only")
        import ctypes as C
        pos = pos.contiguous()
        model.set_weights_f32(theta.detach().contiguous())
        forces = torch.empty(3, system.n, dtype=torch.float32, device=pos.device)
        nnp.check(nnp.lib().nnp_nc_forces(model.handle, C.byref(system.c(pos)), C.byref(nlist.c()), nnp._ptr(ws),
                                          ws.numel(), nnp._ptr(forces), nnp._stream()))
        ctx.args = (pos, model, system, nlist, ws)
        return forces

    @staticmethod
    def backward(ctx, grad_forces):
        import ctypes as C
        pos, model, system, nlist, ws = ctx.args
        g = grad_forces.contiguous().float()
        out = torch.empty(model.n_weights, dtype=torch.float32, device=g.device)
        nnp.check(nnp.lib().nnp_nc_weight_grad(model.handle, C.byref(system.c(pos)), C.byref(nlist.c()), nnp._ptr(g),
                                               nnp._ptr(out), nnp._ptr(ws), ws.numel(), nnp._stream()))
        return out, None, None, None, None, None
