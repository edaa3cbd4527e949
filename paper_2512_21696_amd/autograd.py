"""torch.autograd binding of the library's discrete adjoint: the outlet-flux
history of a one-component run as a differentiable function of the gray
porosity field.  Argument marshalling only; the forward steps and the reverse
sweep run in the HIP library."""
import numpy as np
import torch

from . import lbm_create


class FluxHistory(torch.autograd.Function):
    """Q = FluxHistory.apply(phi, run) with phi a float64 tensor [z, y, x]
    (read on gray voxels) and run a dict holding "params", "cls", "ptype",
    "tables", the initial density "rho" [z, y, x] (the water density, with
    "rho_o" the oil density for two components), "steps" and optionally
    "checkpoint_every" and "start_state" (a state blob loaded after the
    initialisation, e.g. residual amounts and side flags of a running job).  Returns the (water) outlet flux of every step, a
    float64 CPU tensor [steps].  The backward pass restarts from the same
    initial state and calls the library's adjoint with the incoming dL/dQ."""

    @staticmethod
    def forward(ctx, phi, run):
        ph = phi.detach().to("cpu", torch.float64).numpy()
        lb = lbm_create(run["params"])
        try:
            lb.set_geometry(run["cls"], ph, run["ptype"], run["tables"])
            lb.init_fluid(run["rho"], run.get("rho_o"))
            if run.get("start_state") is not None:
                lb.set_state(run["start_state"])
            start = lb.get_state()
            q = lb.step_flux(int(run["steps"]))[:, 0].copy()
        except Exception:
            lb.destroy()
            raise
        ctx.lb, ctx.start, ctx.run = lb, start, run
        ctx.phi_device, ctx.phi_dtype = phi.device, phi.dtype
        return torch.from_numpy(q)

    @staticmethod
    def backward(ctx, grad_q):
        lb = ctx.lb
        try:
            lb.set_state(ctx.start)
            out = lb.adjoint_flux(int(ctx.run["steps"]), grad_q.detach().cpu().numpy(),
                                  ctx.run.get("checkpoint_every", 0))
        finally:
            lb.destroy()
        g = torch.from_numpy(np.ascontiguousarray(out["dL_dphi"]))
        return g.to(ctx.phi_device, ctx.phi_dtype), None
