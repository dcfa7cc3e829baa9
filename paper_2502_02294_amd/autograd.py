"""torch.autograd.Function over the library's forward run and hand-written reverse pass."""

import torch


class DiffHydroFn(torch.autograd.Function):
    """rho_final = DiffHydroFn.apply(white, theta, sim, a_final).

    white: (n, n, n) float32 CUDA white noise; theta: float64 tensor (eps_sf, delta_c) of the
    star-formation parameters.  The backward calls the library's reverse pass and returns
    dL/dwhite and dL/dtheta; the time schedule of the forward run is held fixed."""

    @staticmethod
    def forward(ctx, white, theta, sim, a_final):
        if sim.S != 1:
            raise ValueError("DiffHydroFn takes a single-sample handle (config.batch = 1)")
        eps_sf, delta_c = [float(v) for v in theta.detach().cpu()]
        sim.set_params(eps_sf=eps_sf, delta_c=delta_c)
        sim.forward(white.detach().contiguous(), float(a_final))
        ctx.sim = sim
        ctx.theta_dtype, ctx.theta_device = theta.dtype, theta.device
        return sim.get("rho")

    @staticmethod
    def backward(ctx, grad_rho):
        gw, gp = ctx.sim.backward(grad_rho.contiguous().float())
        gtheta = torch.tensor(gp[2:4], dtype=ctx.theta_dtype, device=ctx.theta_device)
        return gw, gtheta, None, None
