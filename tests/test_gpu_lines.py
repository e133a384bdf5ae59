"""The threshold-line growth rule (Sec. III.D) on the GPU against the FP64
oracle: identical extents from identical float32 densities, and a run that
grows twice (right side, then top and bottom) with the same patch history and
fields within the parity tolerance."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_13276_amd import binding as B
from paper_2105_13276_amd import workloads as W

from gpu_helpers import assert_parity, both

pytestmark = pytest.mark.gpu

LAM = 299792458.0 / 110e9
DX = LAM / 32
THR = 1e15


def _cfg(periods=2, **over):
    kw = dict(erms_over_ebd=3.0, regrid_rule="lines", m_lx=8, m_ly=8, m_ex=8, m_ey=4,
              n_line=THR)
    kw.update(over)
    cfg = W.make(96, 48, 32, "dynamic", periods, **kw)
    cfg["regrid_every"] = 2 * cfg["steps_per_period"]
    return cfg


def test_same_extents_from_the_same_density():
    cfg = _cfg()
    sb, sf = W.seeds(cfg, [(60 * DX, 24 * DX)], [3e17])
    g, o = both(cfg, sb, sf)
    assert g.patch() == o.patch() == (56, 20, 64, 28)
    rng = np.random.default_rng(7)
    for case in range(24):
        e = g.patch()
        assert e == o.patch()
        # a float32 density near the threshold, a few hot nodes around the lines
        n = (rng.uniform(0.0, 0.999, (49, 97)) * THR).astype(np.float32)
        for _ in range(rng.integers(0, 4)):
            i = int(rng.integers(e[0] - 1, e[2] + 2))
            j = int(rng.integers(e[1] - 1, e[3] + 2))
            n[j, i] = np.float32(THR) * np.float32(rng.choice([1.0, 1.0000001, 2.0]))
        g.set("n", 0, n)
        o.set("n", 0, n.astype(np.float64))
        g.regrid()
        o.regrid()
        assert g.patch() == o.patch(), "case %d" % case
    g.close()


def test_growth_history_and_fields():
    cfg = _cfg(periods=14)
    sb, sf = W.seeds(cfg, [(59.5 * DX, 24 * DX)], [3e17])
    g, o = both(cfg, sb, sf)
    hist_g, hist_o = [g.patch()], [o.patch()]
    for _ in range(cfg["steps"] // cfg["regrid_every"]):
        g.step(cfg["regrid_every"])
        o.step(cfg["regrid_every"])
        hist_g.append(g.patch())
        hist_o.append(o.patch())
    print("patch history", hist_g, flush=True)
    assert hist_g == hist_o
    assert hist_g[0] == (55, 20, 63, 28) and hist_g[-1] == (55, 16, 71, 32)
    assert_parity(g, o, O.derived(cfg)["n_c"], tag="lines")
    g.close()
