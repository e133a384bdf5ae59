"""The FP64 reference adjoint (oracle/torch_model.py + torch.autograd) of
F = dx^2 * sum over a wavelength-sized window of n(t_final): its forward is
the C oracle's, and its gradients match central finite differences of the C
oracle (relative step 1e-4).  Cases: a fixed patch, the uniform mesh, a
growing patch (one growth, with the schedule the C oracle decided), and the
fixed patch with the Townsend source and recombination of Eq. (4) (where A
and beta do not enter: both gradients and both difference quotients are
zero)."""
import numpy as np
import pytest
import torch

from oracle import torch_model as TM

from adjoint_cases import CENTRE, case as _case, history, window


def _window(cfg, centre):
    return window(cfg, centre)


def _c_objective(cfg, sb, w, layout):
    """Objective of a perturbed C oracle run; the perturbation must leave the
    patch history as it was (else the difference quotient is meaningless)."""
    o, ext0, growth = history(cfg, sb)
    assert (ext0, growth) == layout
    return float((w * o.get("n")).sum())


@pytest.mark.parametrize("mode", ["static", "uniform", "dynamic", "townsend"])
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


@pytest.mark.parametrize("mode", ["static", "uniform", "dynamic", "townsend"])
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
    g = lambda t: 0.0 if t.grad is None else t.grad.item()   # unused (Townsend): zero
    ad = {"e0": e0.grad.item() / 1.0 / cfg["erms_over_ebd"], "A": g(A), "beta": g(beta)}
    for k in fd:
        assert ad[k] == pytest.approx(fd[k], rel=1e-6), (k, ad[k], fd[k])
    # seed: directional derivative along a positive random field
    rng = np.random.default_rng(4)
    v = rng.random(sb.shape) * sb  # relative: keeps the density positive
    fdv = (_c_objective(cfg, sb + h * v, w, layout) - _c_objective(cfg, sb - h * v, w, layout)) / (2 * h)
    adv = float((seed.grad.numpy() * v).sum())
    assert adv == pytest.approx(fdv, rel=1e-6)
