"""PyTorch autograd over the flood run: gauge depths as a differentiable
function of the per-cell Manning field and the inflow hydrograph samples.

The forward and the gradients run in libflood's kernels (fl_adj_forward,
fl_adj_backward); this module only moves tensors across the C interface.
"""
import torch

from . import Flood


class GaugeSeries(torch.autograd.Function):
    """series = GaugeSeries.apply(n_field, q_samples, flood, nsteps, inflow)

    n_field: [ny, nx] Manning coefficients; q_samples: [nsamples] hydrograph
    discharges (m^3/s) at the times of `inflow` = (side, first, count, slope,
    t_samples).  `flood` is a Flood context with DEM, outflow and parameters
    (fixed dt) set and adj_setup done.  Returns the gauge depths
    [nsteps/obs_every, ngauges] on n_field's device; any differentiable loss
    of them back-propagates to n_field and q_samples through the hand-written
    adjoint with checkpointing.
    """

    @staticmethod
    def forward(ctx, n_field, q_samples, flood: Flood, nsteps: int, inflow):
        side, first, count, slope, t_samples = inflow
        flood.set_manning(n_field.detach())
        flood.set_inflow(side, first, count, slope, t_samples,
                         q_samples.detach().double().cpu().numpy())
        flood.commit()
        flood.adj_setup(flood._adj_gauges, flood._adj_obs_every, None, flood._adj_ckpt)
        nobs = nsteps // flood._adj_obs_every
        dtype = torch.float64 if flood.dtype.__name__ == "float64" else torch.float32
        series = torch.empty((nobs, len(flood._adj_gauges)), dtype=dtype, device=n_field.device)
        if n_field.is_cuda:
            torch.cuda.synchronize(n_field.device)
            flood.adj_forward(nsteps, out=series)
        else:
            s, _ = flood.adj_forward(nsteps)
            series = torch.from_numpy(s)
        ctx.flood = flood
        ctx.nsamples = q_samples.numel()
        ctx.n_dtype = n_field.dtype
        ctx.q_dtype = q_samples.dtype
        ctx.q_device = q_samples.device
        return series

    @staticmethod
    def backward(ctx, grad_series):
        flood = ctx.flood
        g = grad_series.detach().contiguous()
        if g.is_cuda:
            gn = torch.empty((flood.ny, flood.nx), dtype=torch.float64, device=g.device)
            torch.cuda.synchronize(g.device)
            gn, gq = flood.adj_backward(g, ctx.nsamples, grad_n_out=gn)
        else:
            gn, gq = flood.adj_backward(g.numpy(), ctx.nsamples)
            gn = torch.from_numpy(gn)
        gq = torch.as_tensor(gq, dtype=ctx.q_dtype, device=ctx.q_device)
        return gn.to(ctx.n_dtype), gq, None, None, None


def gauge_series(flood: Flood, n_field, q_samples, nsteps: int, inflow, gauges, obs_every: int,
                 ckpt_stride: int = 0):
    """Differentiable gauge depths (see GaugeSeries)."""
    flood._adj_gauges = list(gauges)
    flood._adj_obs_every = obs_every
    flood._adj_ckpt = ckpt_stride
    return GaugeSeries.apply(n_field, q_samples, flood, nsteps, inflow)
