"""The full Eq. (4) source on the GPU (Townsend ionisation with separate
attachment, recombination) against the FP64 oracle, on the uniform mesh and
with a patch; the adjoint refuses this source."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_13276_amd import binding as B
from paper_2105_13276_amd import workloads as W

from gpu_helpers import assert_parity, both

pytestmark = pytest.mark.gpu

LAM = 299792458.0 / 110e9
DX = LAM / 32


def _nc(cfg):
    return O.derived(cfg)["n_c"]


def test_townsend_and_recombination_uniform():
    # a dense seed (r_ei n ~ 1e8/s, comparable with the ionisation rate) in a
    # strong field; 16 periods = 15 continuity updates
    cfg = W.make(128, 64, 32, "uniform", 16, erms_over_ebd=2.0, source_model="townsend",
                 beta_rec=2.0)
    sb = W.gaussian_seed(128, 64, DX, [(80 * DX, 32 * DX)], [1e22], LAM / 10)
    g, o = both(cfg, sb)
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    n0 = sb.max()
    assert o.get("n", 0).max() != pytest.approx(n0, rel=1e-3)  # the source acts
    assert_parity(g, o, _nc(cfg), levels=(0,), tag="townsend-uniform")
    g.close()


def test_townsend_with_patch():
    cfg = W.make(128, 64, 32, "static", 16, static_ext=(48, 16, 96, 48),
                 erms_over_ebd=2.0, source_model="townsend", beta_rec=1.0)
    sb, sf = W.seeds(cfg, [(72 * DX, 32 * DX)], [1e20])
    g, o = both(cfg, sb, sf)
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    assert_parity(g, o, _nc(cfg), tag="townsend-patch")
    g.close()


@pytest.mark.parametrize("over", [dict(source_model="townsend"), dict(beta_rec=1.0)])
def test_adjoint_refuses_other_sources(over):
    cfg = W.make(64, 32, 32, "uniform", 2, **over)
    sb, _ = W.seeds(cfg)
    g = B.Sim(cfg, sb, None)
    with pytest.raises(B.DmrError, match="EINVAL"):
        g.record(cfg["steps"], 45)
    g.close()
