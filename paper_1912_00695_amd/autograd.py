"""torch.autograd.Function over the HIP solver: receiver data as a differentiable
function of the velocity model and the source wavelet.

forward:  (vel, wavelet) -> d = F(vel) wavelet        (wave_forward, keeping
          checkpoints of (u^{kC}, u^{kC-1}) every C steps on the device)
backward: dL/dd -> (dL/dvel, dL/dwavelet)             (wave_gradient: segment
          recompute from the checkpoints, adjoint steps with the gradient
          accumulated in the adjoint kernel)

The sponge strength is a fixed property of the grid (its vmax), so it is held
constant when the velocity is differentiated. The FWI misfit
J = 0.5 ||d - d_obs||^2 gives dL/dd = d - d_obs.
"""
import torch

from . import wave


class WaveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vel, wavelet, grid, src_xyz, rec_xyz, ckpt_every=50):
        out = wave.forward(grid, vel.detach(), wavelet.detach(), src_xyz, rec_xyz,
                           ckpt_every=ckpt_every)
        ctx.grid, ctx.src, ctx.rec, ctx.C = grid, src_xyz, rec_xyz, ckpt_every
        ctx.save_for_backward(vel.detach(), wavelet.detach(), out["ckpt"])
        return out["rec"]

    @staticmethod
    def backward(ctx, grad_rec):
        vel, wavelet, ckpt = ctx.saved_tensors
        res = wave.gradient(ctx.grid, vel, wavelet, ctx.src, ctx.rec,
                            grad_rec.contiguous().float(), ckpt=ckpt, ckpt_every=ctx.C,
                            want_wavelet_grad=ctx.needs_input_grad[1])
        gv = res["grad_vel"] if ctx.needs_input_grad[0] else None
        gw = res["grad_wavelet"] if ctx.needs_input_grad[1] else None
        return gv, gw, None, None, None, None


def shot(vel, wavelet, grid, src_xyz, rec_xyz, ckpt_every=50):
    """Receiver data of one shot, differentiable in vel and wavelet."""
    return WaveFn.apply(vel, wavelet, grid, src_xyz, rec_xyz, ckpt_every)


def fwi_misfit(vel, wavelet, grid, src_xyz, rec_xyz, d_obs, ckpt_every=50):
    """J = 0.5 ||d(vel) - d_obs||^2 (differentiable)."""
    d = shot(vel, wavelet, grid, src_xyz, rec_xyz, ckpt_every)
    return 0.5 * torch.sum((d - d_obs) ** 2)
