"""Cases shared by the reference-adjoint tests (CPU) and the GPU adjoint
tests: a fixed patch, the uniform mesh, a growing patch and the fixed patch
with the Townsend source and recombination, each with a wavelength-square
objective window centred on the seed."""
import numpy as np

from oracle import oracle as O
from paper_2105_13276_amd import workloads as W

LAM = 299792458.0 / 110e9
CENTRE = {"static": (57 * LAM / 32, 24 * LAM / 32), "uniform": (57 * LAM / 32, 24 * LAM / 32),
          "dynamic": (96 * 0.62 * LAM / 32, 24 * LAM / 32),
          "townsend": (57 * LAM / 32, 24 * LAM / 32)}
PEAK = {"static": 3e17, "uniform": 3e17, "dynamic": 3e17, "townsend": 1e20}


def case(mode="static", periods=10):
    if mode == "static":
        cfg = W.make(96, 48, 32, "static", periods, static_ext=(48, 16, 64, 32),
                     erms_over_ebd=2.5)
    elif mode == "dynamic":
        # grows once, after 8 of the 10 periods (regrid every 2 periods)
        cfg = W.make(96, 48, 32, "dynamic", periods, erms_over_ebd=3.0)
        cfg["regrid_every"] = 2 * cfg["steps_per_period"]
    elif mode == "townsend":
        # the fixed patch with the Townsend source and recombination of
        # Eq. (4); a dense seed so that the n^2 loss matters
        cfg = W.make(96, 48, 32, "static", periods, static_ext=(48, 16, 64, 32),
                     erms_over_ebd=2.0, source_model="townsend", beta_rec=1.0)
    else:
        cfg = W.make(64, 32, 32, "uniform", periods, erms_over_ebd=2.5)
    sb, _ = W.seeds(cfg, [CENTRE[mode]], [PEAK[mode]])
    return cfg, sb


def window(cfg, centre):
    """dx^2 on the base nodes within half a wavelength of centre (per axis)."""
    return W.window_weights(cfg, centre)


def history(cfg, sb):
    """C oracle run to t_final: (sim, patch at t = 0, {steps done: new patch})."""
    o = O.Sim(cfg, sb)
    if cfg["mode"] == "uniform":
        o.step(cfg["steps"])
        return o, None, {}
    ext0 = o.patch()
    growth, cur, k = {}, ext0, 0
    every = cfg["regrid_every"] if cfg["mode"] == "dynamic" else cfg["steps"]
    while k < cfg["steps"]:
        q = min(every, cfg["steps"] - k)
        o.step(q)
        k += q
        if o.patch() != cur:
            growth[k] = cur = o.patch()
    return o, ext0, growth


def reference_gradients(cfg, sb, w, ext0, growth, seg=45):
    """F and its FP64 gradients (dF/dseed, dF/dE0, dF/dA, dF/dbeta) from the
    torch float64 model of the update with autograd."""
    import torch
    from oracle import torch_model as TM
    m = TM.Model(cfg, ext0, growth)
    seed = torch.tensor(sb, requires_grad=True)
    e0 = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    A = torch.tensor(cfg["A_ion"], dtype=torch.float64, requires_grad=True)
    beta = torch.tensor(cfg["beta_ion"], dtype=torch.float64, requires_grad=True)
    cs, _ = m.run(seed, e0, A, beta, cfg["steps"], seg=seg)
    F = (torch.tensor(w) * cs["n"]).sum()
    F.backward()
    g = lambda t: 0.0 if t.grad is None else t.grad.item()   # unused: zero
    return dict(F=F.item(), seed=seed.grad.numpy(), E0=e0.grad.item() / m.d["E0"],
                A=g(A), beta=g(beta))
