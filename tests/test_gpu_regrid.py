"""Growth test and prolongation on the GPU against the oracle on identical
float32 density fields: flags, prefix sum, compacted list and extents must be
bit-exact; prolonged fields agree to float32 rounding."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_13276_amd import binding as B
from paper_2105_13276_amd import workloads as W

pytestmark = pytest.mark.gpu

LAM = 299792458.0 / 110e9


def _blobs(cfg, rng, k):
    dx = LAM / cfg["cells_per_lambda"]
    cen = [(rng.uniform(0.05, 0.95) * cfg["nx"] * dx, rng.uniform(0.05, 0.95) * cfg["ny"] * dx)
           for _ in range(k)]
    pk = list(10.0 ** rng.uniform(15.0, 18.5, size=k))
    n = W.gaussian_seed(cfg["nx"], cfg["ny"], dx, cen, pk, LAM / 20)
    return n.astype(np.float32)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("shape", [(96, 48, 8), (512, 256, 16), (256, 192, 16)])
def test_regrid_bitexact(seed, shape):
    nx, ny, blk = shape
    cfg = W.make(nx, ny, 32, "dynamic", 1, block=blk)
    rng = np.random.default_rng(1000 * seed + nx)
    zero = np.zeros((ny + 1, nx + 1))
    g = B.Sim(cfg, zero)
    o = O.Sim(cfg, zero)
    for rnd in range(3):  # successive tests: monotone growth from each state
        n32 = _blobs(cfg, rng, 1 + rnd)
        g.set("n", 0, n32)
        o.set("n", 0, n32.astype(np.float64))
        g.regrid()
        o.regrid()
        fg, sg, lg, cg = g.regrid_info()
        fo, so, lo, co = o.regrid_info()
        assert (fg == fo).all(), "flags"
        assert (sg == so).all() and cg == co and (lg == lo).all()
        assert g.patch() == o.patch()


def test_regrid_empty_and_clip():
    cfg = W.make(96, 48, 32, "dynamic", 1, block=8)
    zero = np.zeros((49, 97))
    g = B.Sim(cfg, zero)
    assert g.patch() == (0, 0, 0, 0)
    assert g.regrid_info()[3] == 0
    n = np.zeros((49, 97), np.float32)
    n[2:12, 2:40] = 1e19
    g.set("n", 0, n)
    g.regrid()
    o = O.Sim(cfg, n.astype(np.float64))
    assert g.patch() == o.patch() == (16, 8, 40, 16)


def test_prolongation_parity():
    """Force growth with arbitrary coarse fields and compare every prolonged
    fine entity (and the copied old part) with the oracle."""
    cfg = W.make(96, 48, 32, "dynamic", 1, block=8)
    rng = np.random.default_rng(5)
    n0 = np.zeros((49, 97), np.float32)
    n0[20:22, 30:33] = 1e19
    g = B.Sim(cfg, n0)
    o = O.Sim(cfg, n0.astype(np.float64))
    assert g.patch() == o.patch()
    # one step so that every buffer holds data, then arbitrary fields
    g.step(1)
    o.step(1)
    for lv in (0, 1):
        for f in ("hz", "ex", "ey", "jx", "jy", "acc"):
            r, c = o.dims(f, lv)
            scale = {"hz": 1e3, "jx": 1e6, "jy": 1e6}.get(f, 1e5)
            v = (scale * rng.standard_normal((r, c))).astype(np.float32)
            g.set(f, lv, v)
            o.set(f, lv, v.astype(np.float64))
        r, c = o.dims("ring", lv)
        v = (1e12 * rng.random((r, c))).astype(np.float32)
        g.set("ring", lv, v)
        o.set("ring", lv, v.astype(np.float64))
    n2 = n0.copy()
    n2[34:36, 70:72] = 1e19
    g.set("n", 0, n2)
    o.set("n", 0, n2.astype(np.float64))
    g.regrid()
    o.regrid()
    assert g.patch() == o.patch() == (24, 16, 72, 40)
    for f in ("hz", "ex", "ey", "jx", "jy", "n", "acc", "ring", "erms2"):
        a = np.asarray(g.get(f, 1), np.float64)
        b = o.get(f, 1)
        assert a.shape == b.shape, f
        err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)
        assert err < 3e-6, (f, err)
