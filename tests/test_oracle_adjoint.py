"""The FP64 reference adjoint (oracle/torch_model.py + torch.autograd) of
F = dx^2 * sum over a wavelength-sized window of n(t_final): its forward is
the C oracle's, and its gradients match central finite differences of the C
oracle (relative step 1e-4).  Cases: a fixed patch, the uniform mesh, and a
growing patch (one growth, with the schedule the C oracle decided)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import torch_model as TM
from paper_2105_13276_amd import workloads as W

LAM = 299792458.0 / 110e9


CENTRE = {"static": (57 * LAM / 32, 24 * LAM / 32), "uniform": (57 * LAM / 32, 24 * LAM / 32),
          "dynamic": (96 * 0.62 * LAM / 32, 24 * LAM / 32)}


def _case(mode="static", periods=10):
    if mode == "static":
        cfg = W.make(96, 48, 32, "static", periods, static_ext=(48, 16, 64, 32),
                     erms_over_ebd=2.5)
        sb, _ = W.seeds(cfg, [CENTRE[mode]], [3e17])
    elif mode == "dynamic":
        # grows once, after 8 of the 10 periods (regrid every 2 periods)
        cfg = W.make(96, 48, 32, "dynamic", periods, erms_over_ebd=3.0)
        cfg["regrid_every"] = 2 * cfg["steps_per_period"]
        sb, _ = W.seeds(cfg, [CENTRE[mode]], [3e17])
    else:
        cfg = W.make(64, 32, 32, "uniform", periods, erms_over_ebd=2.5)
        sb, _ = W.seeds(cfg, [CENTRE[mode]], [3e17])
    return cfg, sb


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


def _window(cfg, centre):
    dx = LAM / cfg["cells_per_lambda"]
    x = np.arange(cfg["nx"] + 1) * dx
    y = np.arange(cfg["ny"] + 1) * dx
    X, Y = np.meshgrid(x, y)
    w = ((np.abs(X - centre[0]) <= LAM / 2) & (np.abs(Y - centre[1]) <= LAM / 2)).astype(float)
    return w * dx * dx


def _c_objective(cfg, sb, w, layout):
    """Objective of a perturbed C oracle run; the perturbation must leave the
    patch history as it was (else the difference quotient is meaningless)."""
    o, ext0, growth = history(cfg, sb)
    assert (ext0, growth) == layout
    return float((w * o.get("n")).sum())


@pytest.mark.parametrize("mode", ["static", "uniform", "dynamic"])
def test_forward_matches_c_oracle(mode):
    cfg, sb = _case(mode)
    o, ext0, growth = history(cfg, sb)
    if mode == "dynamic":
        assert growth, "the case is meant to grow the patch"
    m = TM.Model(cfg, ext0, growth)
    cs, fs = m.run(sb, 1.0, cfg["A_ion"], cfg["beta_ion"], cfg["steps"], grad=False)
    for f in ("hz", "ey", "jy", "n", "acc"):
        a, b = o.get(f, 0), cs[f].numpy()
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max(), f
        if fs is not None:
            a, b = o.get(f, 1), fs[f].numpy()
            assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max(), f


@pytest.mark.parametrize("mode", ["static", "uniform", "dynamic"])
def test_gradients_match_central_differences(mode):
    cfg, sb = _case(mode)
    steps = cfg["steps"]
    w = _window(cfg, CENTRE[mode])
    _, ext0, growth = history(cfg, sb)
    layout = (ext0, growth)
    m = TM.Model(cfg, ext0, growth)
    seed = torch.tensor(sb, requires_grad=True)
    e0 = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    A = torch.tensor(cfg["A_ion"], dtype=torch.float64, requires_grad=True)
    beta = torch.tensor(cfg["beta_ion"], dtype=torch.float64, requires_grad=True)
    cs, _ = m.run(seed, e0, A, beta, steps, seg=17)
    F = (torch.tensor(w) * cs["n"]).sum()
    F.backward()
    h = 1e-4
    # incident amplitude: E0 is proportional to erms_over_ebd.  Fourth-order
    # central differences with relative step h (the exponent's third
    # derivative is large enough to show in second-order ones at 1e-6)
    fd = {}
    for name, key in (("e0", "erms_over_ebd"), ("A", "A_ion"), ("beta", "beta_ion")):
        f = {q: _c_objective(dict(cfg, **{key: cfg[key] * (1 + q * h)}), sb, w, layout)
             for q in (-2, -1, 1, 2)}
        fd[name] = (8 * (f[1] - f[-1]) - (f[2] - f[-2])) / (12 * h * cfg[key])
    ad = {"e0": e0.grad.item() / 1.0 / cfg["erms_over_ebd"], "A": A.grad.item(),
          "beta": beta.grad.item()}
    for k in fd:
        assert ad[k] == pytest.approx(fd[k], rel=1e-6), (k, ad[k], fd[k])
    # seed: directional derivative along a positive random field
    rng = np.random.default_rng(4)
    v = rng.random(sb.shape) * sb  # relative: keeps the density positive
    fdv = (_c_objective(cfg, sb + h * v, w, layout) - _c_objective(cfg, sb - h * v, w, layout)) / (2 * h)
    adv = float((seed.grad.numpy() * v).sum())
    assert adv == pytest.approx(fdv, rel=1e-6)
