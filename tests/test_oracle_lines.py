"""The threshold-line growth rule of Sec. III.D in the FP64 oracle, pinned to
hand-derived extents.

The rule as read from the paper: the threshold lines coincide with the sides
of the fine patch; a side whose line carries a base node with density above
the threshold density moves outward, by m_ex for the sides that bound x and
by m_ey for those that bound y (m_ex > m_ey); the first patch is m_lx x m_ly
base cells around the initial density.  The expected extents below are
worked out by hand from that reading (96 x 48 base cells, 16-cell blocks,
source line at column 8, so the patch stays within x in [32, 80] and y in
[16, 32])."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_13276_amd import workloads as W

LAM = 299792458.0 / 110e9
DX = LAM / 32
THR = 1e15


def _cfg(**over):
    kw = dict(erms_over_ebd=3.0, regrid_rule="lines", m_lx=8, m_ly=8, m_ex=8, m_ey=4,
              n_line=THR)
    kw.update(over)
    return W.make(96, 48, 32, "dynamic", 2, **kw)


def _sim(cfg, centre=(60.0, 24.0), peak=3e17):
    sb, sf = W.seeds(cfg, [(centre[0] * DX, centre[1] * DX)], [peak])
    return O.Sim(cfg, sb, sf)


def test_first_patch_centred_on_the_seed_peak():
    # peak node (60, 24): [60 - 4, 60 + 4) x [24 - 4, 24 + 4)
    assert _sim(_cfg()).patch() == (56, 20, 64, 28)
    # 32 x 16 around (40, 24): x from 24 is clipped to the source margin 32
    assert _sim(_cfg(m_lx=32, m_ly=16), centre=(40.0, 24.0)).patch() == (32, 16, 56, 32)
    # a peak between two nodes (59.5): equal values, the first one (59) wins
    assert _sim(_cfg(), centre=(59.5, 24.0)).patch() == (55, 20, 63, 28)


@pytest.mark.parametrize("hot,value,expect", [
    ((64, 24), 2 * THR, (56, 20, 72, 28)),   # right line: + m_ex
    ((56, 22), 2 * THR, (48, 20, 64, 28)),   # left line:  - m_ex
    ((60, 28), 2 * THR, (56, 20, 64, 32)),   # top line:   + m_ey
    ((60, 20), 2 * THR, (56, 16, 64, 28)),   # bottom line: - m_ey
    ((64, 28), 2 * THR, (56, 20, 72, 32)),   # a corner is on two lines
    ((64, 24), THR, (56, 20, 64, 28)),       # at the threshold: no move
    ((63, 24), 1e20, (56, 20, 64, 28)),      # inside, not on a line
    ((65, 24), 1e20, (56, 20, 64, 28)),      # outside
])
def test_lines_move_their_sides(hot, value, expect):
    o = _sim(_cfg())
    assert o.patch() == (56, 20, 64, 28)
    n = np.zeros((49, 97))
    n[hot[1], hot[0]] = value
    o.set("n", 0, n)
    o.regrid()
    assert o.patch() == expect


def test_growth_is_clipped_and_monotone():
    o = _sim(_cfg(m_ex=30, m_ey=30))
    n = np.zeros((49, 97))
    for (i, j) in [(56, 24), (64, 24), (60, 20), (60, 28)]:
        n[j, i] = 1e20
    o.set("n", 0, n)
    o.regrid()
    assert o.patch() == (32, 16, 80, 32)     # every side at its margin
    o.set("n", 0, np.zeros((49, 97)))
    o.regrid()
    assert o.patch() == (32, 16, 80, 32)     # never shrinks


def test_invalid_steps_rejected():
    with pytest.raises(Exception):
        _sim(_cfg(m_ex=0))
