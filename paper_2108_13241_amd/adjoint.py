"""Autograd wrapper of the hand-written adjoint: gradients of a channel objective.

J(alpha, g) = mean u_x over the fluid nodes of the outlet column after T steps from rest,
for a lattice with a per-node Brinkman drag field alpha and body force g.  The forward
pass runs the T steps on the GPU and keeps a checkpoint every K steps (K = ceil(sqrt T)
by default); the backward pass replays each segment from its checkpoint and runs the
adjoint kernel backwards through it (lbm_run_checkpointed / lbm_adjoint_checkpointed in
the C ABI).  Everything numeric runs in the HIP kernels; this class marshals buffers.
"""
from __future__ import annotations

import math

import numpy as np
import torch


class ChannelObjective(torch.autograd.Function):
    """J = ChannelObjective.apply(alpha, g, spec).

    alpha : tensor [ny, nx] with values in [0, 1] (any float dtype, any device)
    g     : tensor [2], the body-force acceleration (g_x, g_y)
    spec  : dict with keys mask (uint8 [ny, nx]), tau, steps (T), x_out, and optionally
            dtype ("f32" or "f64", default "f32"), K (checkpoint interval).
    Returns J as a 0-d float64 tensor on the GPU.  backward gives dJ/dalpha (alpha's
    dtype) and dJ/dg (g's dtype); the FP64 accumulators are kept on
    ``ChannelObjective.last_grads`` for inspection."""

    last_grads = None

    @staticmethod
    def forward(ctx, alpha, g, spec):
        from . import Lattice

        mask = np.ascontiguousarray(spec["mask"], dtype=np.uint8)
        T = int(spec["steps"])
        K = int(spec.get("K") or max(1, math.ceil(math.sqrt(T))))
        gh = [float(v) for v in g.detach().cpu().double().tolist()]
        lat = Lattice(mask, float(spec["tau"]), force=gh, dtype=spec.get("dtype", "f32"),
                      layout="dense_ab")
        lat.set_porosity(alpha.detach().cpu().float().numpy())
        sb = lat.state_bytes()
        nseg = max(1, math.ceil(T / K))
        ckpt = torch.empty(nseg * sb, dtype=torch.uint8, device="cuda")
        lat.run_checkpointed(T, K, ckpt)
        J = lat.objective_outlet_ux(int(spec["x_out"]))
        ctx.lat, ctx.ckpt, ctx.T, ctx.K, ctx.x_out = lat, ckpt, T, K, int(spec["x_out"])
        ctx.alpha_dtype, ctx.g_dtype = alpha.dtype, g.dtype
        ctx.alpha_device, ctx.g_device = alpha.device, g.device
        return torch.tensor(J, dtype=torch.float64, device="cuda")

    @staticmethod
    def backward(ctx, gJ):
        lat = ctx.lat
        sb = lat.state_bytes()
        seg = torch.empty(ctx.K * sb, dtype=torch.uint8, device="cuda")
        ga = torch.zeros((lat.ny, lat.nx), dtype=torch.float64, device="cuda")
        gg = torch.zeros(2, dtype=torch.float64, device="cuda")
        lat.adjoint_checkpointed(ctx.T, ctx.K, ctx.ckpt, seg, ctx.x_out, float(gJ.item()), ga, gg)
        torch.cuda.current_stream().synchronize()
        ChannelObjective.last_grads = (ga, gg)
        return (ga.to(dtype=ctx.alpha_dtype, device=ctx.alpha_device),
                gg.to(dtype=ctx.g_dtype, device=ctx.g_device), None)
