"""Refinement factor r = 4 (the paper validates r = 2 and 4): coarse lambda/16
with a lambda/64 patch, four fine substeps per coarse step, against the FP64
oracle: a fixed patch off the tile grid, and a growing patch."""
import pytest

from oracle import oracle as O
from paper_2105_13276_amd import workloads as W

from gpu_helpers import assert_parity, both

pytestmark = pytest.mark.gpu

LAM = 299792458.0 / 110e9
DXC = LAM / 16


def _nc(cfg):
    return O.derived(cfg)["n_c"]


def test_r4_static_patch():
    # patch of 26 x 14 coarse cells = 104 x 56 fine: ragged against 64-wide tiles
    cfg = W.make(64, 32, 16, "static", 20, r=4, block=8, static_ext=(22, 9, 48, 23),
                 erms_over_ebd=2.0)
    sb, sf = W.seeds(cfg, [(36 * DXC, 16 * DXC)], [3e17])
    g, o = both(cfg, sb, sf)
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    assert g.patch() == o.patch() == (22, 9, 48, 23)
    assert_parity(g, o, _nc(cfg), tag="r4-static")
    g.close()


def test_r4_dynamic_growth():
    cfg = W.make(48, 24, 16, "dynamic", 60, r=4, block=8, erms_over_ebd=2.5)
    sb, sf = W.seeds(cfg, [(29.75 * DXC, 12 * DXC)], [1e17])
    g, o = both(cfg, sb, sf)
    p0 = g.patch()
    assert p0 == o.patch()
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    assert g.patch() == o.patch() != p0
    assert_parity(g, o, _nc(cfg), tag="r4-growth")
    g.close()
