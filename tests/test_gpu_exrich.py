"""GPU parity on the x-edge-rich cavity of `cavity_case`: Ex and Ey of equal
amplitude, Jx as large as Jy, across a rectangle (r = 2 and 4) and a union of
blocks with a concave corner.  Every component (Ex, Ey, Hz, Jx, Jy, E_rms^2)
of both levels is held to relative L2 <= 1e-4 against its own norm, so the
x-edge update, PEC on the horizontal walls, Eq. (5b) on the horizontal
patch sides and the Ex/Jx fine -> coarse transfer are each checked."""
import numpy as np
import pytest

from oracle import oracle as O

import cavity_case as K
from gpu_helpers import assert_parity, both

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["rect", "r4", "union"])
def test_x_edge_rich_parity(kind):
    cfg, extra = K.config(kind, periods=10)
    sb, sf = K.seeds(cfg)
    g, o = both(cfg, sb, sf)
    K.start(g, cfg, extra)
    K.start(o, cfg, extra)
    assert g.patch() == o.patch()
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    g.sync()
    rep = assert_parity(g, o, O.derived(cfg)["n_c"], tag="x-edge-rich %s" % kind,
                        every_component=True)
    for lv in (0, 1):
        sh = rep[lv]["share"]
        assert sh["ex"] > 0.3 and sh["jx"] > 0.3, (lv, sh)
    g.close()
