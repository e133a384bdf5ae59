"""torch.autograd.Function over the library's recorded forward and adjoint.

WindowDensity.apply(seed, e0_scale, A, beta, cfg, weights, steps, ckpt_every,
device, fine_rows) returns F = sum_nodes w n(t_final) (float64 scalar tensor) of
a refined run
started from the base-level seed density; its backward calls the
library's hand-written adjoint kernels (dmr_backward) and returns dF/dseed,
dF/de0_scale (the incident amplitude is e0_scale times the one cfg gives),
dF/dA and dF/dbeta.  Every step of both sweeps runs in libdmr.so.
fine_rows: the most fine node rows the run's patch spans (sizes the tape's
fine slots; 0: the whole fine grid).
"""
from __future__ import annotations

import torch

from . import binding as B


class WindowDensity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, seed, e0_scale, A, beta, cfg, weights, steps, ckpt_every=45,
                device="cuda:0", fine_rows=0):
        run = dict(cfg)
        run["erms_over_ebd"] = float(cfg["erms_over_ebd"]) * float(e0_scale)
        run["A_ion"] = float(A)
        run["beta_ion"] = float(beta)
        sim = B.Sim(run, seed.detach().to("cpu", torch.float64).numpy(), None, device=device)
        sim.record(int(steps), int(ckpt_every), int(fine_rows))
        F = sim.weighted_sum(weights, 0)
        ctx.sim, ctx.weights = sim, weights
        ctx.seed_dtype, ctx.seed_device = seed.dtype, seed.device
        # peak incident amplitude of cfg (V/m) per unit e0_scale, as the
        # library derives it
        ctx.e0_unit = B.derived(cfg)["E0"]
        return torch.tensor(F, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gF):
        g = ctx.sim.backward(ctx.weights)
        s = float(gF)
        gseed = (g["seed"].to(torch.float64) * s).to(ctx.seed_device, ctx.seed_dtype)
        f64 = lambda v: torch.tensor(v * s, dtype=torch.float64)
        return (gseed, f64(g["E0"] * ctx.e0_unit), f64(g["A"]), f64(g["beta"]),
                None, None, None, None, None, None)

