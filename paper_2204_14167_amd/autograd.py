"""torch.autograd.Function over the library's energy / electro-osmotic-flux pair.

Forward: U = (1/2) dV <rho, phi> and Q = sum_i w(z_i) q_i (E^P_x,i + E_ext,x) of the
electrostatic pass (charge spreading with wall images, Poisson solve with the wall
conditions, interpolation of the staggered field).  Backward: the library's
hand-written reverse sweep (one transposed interpolation, one Poisson solve, one
gradient gather) from the checkpointed potential.  Argument marshalling only: every
step runs in the HIP library.
"""
import torch

from . import discos


class EnergyFlux(torch.autograd.Function):
    """(U, Q) = EnergyFlux.apply(pos, q, bc_lo, bc_hi, e_ext, ctx, params)

    pos [3, n], q [n], bc_lo / bc_hi [ny, nx] (wall potential or surface charge of each
    column, per the wall types in `params`): float64 tensors on the GPU; e_ext: float64
    CPU tensor [3] (it enters the parameter block by value).  `ctx` is a
    discos.Context, `params` a parameter dict as accepted by discos.Params (its
    bc_values and e_ext are replaced by the tensors given here).
    """

    @staticmethod
    def forward(fctx, pos, q, bc_lo, bc_hi, e_ext, ctx, params):
        p = dict(params)
        p["bc_values"] = (bc_lo.detach().contiguous(), bc_hi.detach().contiguous())
        p["e_ext"] = [float(v) for v in e_ext.detach().cpu()]
        prm = ctx.params(p)
        pos_d, q_d = pos.detach().contiguous(), q.detach().contiguous()
        out, phi = ctx.energy_flux(pos_d, q_d, prm)
        fctx.dctx = ctx
        fctx.prm = prm
        fctx.e_device = e_ext.device
        fctx.save_for_backward(pos_d, q_d, phi)
        return out[0].clone(), out[1].clone()

    @staticmethod
    def backward(fctx, gU, gQ):
        pos, q, phi = fctx.saved_tensors
        need = fctx.needs_input_grad
        names = ("pos", "q", "bc_lo", "bc_hi", "e_ext")
        want = tuple(nm for nm, nd in zip(names, need[:5]) if nd)
        gU = torch.zeros((), dtype=torch.float64, device="cuda") if gU is None else gU
        gQ = torch.zeros((), dtype=torch.float64, device="cuda") if gQ is None else gQ
        g = torch.stack([gU.reshape(()), gQ.reshape(())]).to(torch.float64).contiguous()
        # the saved tensors are the forward's (autograd rejects in-place changes to them),
        # so the forward's cell list may serve, unless another call rebuilt it
        res = fctx.dctx.energy_flux_backward(pos, q, fctx.prm, phi, g, want=want, reuse_cells=True)
        de = res["e_ext"]
        if de is not None:
            de = de.to(fctx.e_device)
        return res["pos"], res["q"], res["bc_lo"], res["bc_hi"], de, None, None


def energy_flux(pos, q, bc_lo, bc_hi, e_ext, ctx, params):
    """Differentiable (U, Q); see EnergyFlux."""
    return EnergyFlux.apply(pos, q, bc_lo, bc_hi, e_ext, ctx, params)
