"""The union-of-blocks fine level on the GPU (the growth test's flagged blocks
refined as they are, Sec. III.A/B, instead of their bounding box): bitwise
the rectangular patch's run on a rectangle of blocks, the FP64 oracle's
fields within the parity tolerance on a non-convex static level and through a
growth, and identical block maps from identical float32 densities."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_13276_amd import binding as B
from paper_2105_13276_amd import workloads as W

from gpu_helpers import assert_parity, both, load_plane_packet

pytestmark = pytest.mark.gpu

LAM = 299792458.0 / 110e9
DX = LAM / 32
FIELDS = ("hz", "ex", "ey", "jx", "jy", "n", "acc", "ring")


def test_rectangle_of_blocks_is_the_patch_bitwise():
    over = dict(static_ext=(48, 16, 96, 48), erms_over_ebd=2.5)
    cr = W.make(128, 64, 32, "static", 1, **over)
    cu = W.make(128, 64, 32, "static", 1, regrid_rule="union", **over)
    sb, sf = W.seeds(cr, [(72.5 * DX, 32 * DX)], [1e17])
    a, b = B.Sim(cr, sb, sf), B.Sim(cu, sb, sf)
    assert a.patch() == b.patch() == (48, 16, 96, 48)
    assert b.blocks().sum() == 6
    steps = 12 * cr["steps_per_period"] + 5
    a.step(steps)
    b.step(steps)
    for lv in (0, 1):
        for f in FIELDS:
            x, y = a.get(f, lv), b.get(f, lv)
            d = np.abs(x.astype(np.float64) - y).max()
            print("%s level %d max |diff| %.3e" % (f, lv, d), flush=True)
            assert np.array_equal(x, y), (f, lv)
    a.close()
    b.close()


def _static_l(periods=1):
    cfg = W.make(128, 64, 32, "static", periods, regrid_rule="union", block=8,
                 static_ext=(48, 16, 96, 32), erms_over_ebd=2.5)
    m = np.zeros((8, 16), np.uint8)
    m[4:6, 6:8] = 1          # an arm up from the left end: a concave corner
    m[5, 10] = 1             # a separate block touching nothing
    m[4, 12] = 1             # and one touching the rectangle at a corner only
    return cfg, m


def test_static_l_shape_matches_oracle():
    cfg, m = _static_l(periods=10)
    sb, sf = W.seeds(cfg, [(56.5 * DX, 32 * DX), (84 * DX, 44 * DX)], [1e17, 1e17])
    g, o = both(cfg, sb, sf)
    g.add_blocks(m)
    o.add_blocks(m)
    assert np.array_equal(g.blocks(), o.blocks()) and g.blocks().sum() == 18
    assert g.patch() == o.patch() == (48, 16, 104, 48)
    steps = cfg["steps"] + 3
    g.step(steps)
    o.step(steps)
    assert o.get("n", 1).max() > 1.05e17
    assert_parity(g, o, O.derived(cfg)["n_c"], tag="union static")
    # nothing outside the level: nodes with no active cell around them
    e = g.patch()
    cb = np.kron(g.blocks(), np.ones((16, 16), np.uint8))[2 * e[1]:2 * e[3], 2 * e[0]:2 * e[2]]
    cb = cb.astype(bool)
    node = np.zeros((cb.shape[0] + 1, cb.shape[1] + 1), bool)
    node[:-1, :-1] |= cb
    node[1:, :-1] |= cb
    node[:-1, 1:] |= cb
    node[1:, 1:] |= cb
    assert (~node).sum() > 0
    for f in ("n", "acc"):
        assert not g.get(f, 1)[~node].any(), f
    assert not g.get("hz", 1)[~cb].any()
    g.close()


def test_growth_history_and_fields():
    cfg = W.make(128, 64, 32, "dynamic", 12, block=8, erms_over_ebd=3.0,
                 regrid_rule="union")
    cfg["regrid_every"] = 2 * cfg["steps_per_period"]
    sb, sf = W.seeds(cfg, [(46.5 * DX, 21 * DX), (92.5 * DX, 45.5 * DX)], [3e17, 2e17])
    g, o = both(cfg, sb, sf)
    hist = [int(g.blocks().sum())]
    assert np.array_equal(g.blocks(), o.blocks())
    for _ in range(cfg["steps"] // cfg["regrid_every"]):
        g.step(cfg["regrid_every"])
        o.step(cfg["regrid_every"])
        assert np.array_equal(g.blocks(), o.blocks())
        hist.append(int(g.blocks().sum()))
    print("active blocks", hist, flush=True)
    assert hist[0] == 7 and hist[-1] == 8
    assert g.patch() == o.patch()
    assert_parity(g, o, O.derived(cfg)["n_c"], tag="union growth")
    g.close()


def test_same_blocks_from_the_same_density():
    cfg = W.make(128, 64, 32, "dynamic", 1, block=8, regrid_rule="union")
    sb, sf = W.seeds(cfg, [(60 * DX, 32 * DX)], [1e17])
    g, o = both(cfg, sb, sf)
    n_c = O.derived(cfg)["n_c"]
    rng = np.random.default_rng(11)
    for case in range(16):
        n = np.zeros((65, 129), np.float32)
        for _ in range(3):   # a few Gaussians around the flag thresholds
            x0, y0 = rng.uniform(0, 128), rng.uniform(0, 64)
            pk = 10 ** rng.uniform(-4.5, -2.5) * n_c
            X, Y = np.meshgrid(np.arange(129.0), np.arange(65.0))
            n += (pk * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / 2.6)).astype(np.float32)
        g.set("n", 0, n)
        o.set("n", 0, n.astype(np.float64))
        g.regrid()
        o.regrid()
        assert np.array_equal(g.blocks(), o.blocks()), "case %d" % case
        fg, _, _, _ = g.regrid_info()
        fo, _, _, _ = o.regrid_info()
        assert np.array_equal(fg, fo), "case %d" % case
    assert g.blocks().sum() > 8
    g.close()


def test_union_errors():
    cfg, m = _static_l()
    g = B.Sim(cfg, np.zeros((65, 129)))
    bad = np.zeros((8, 16), np.uint8)
    bad[0, 5] = 1                     # inside the outer margin
    with pytest.raises(B.DmrError):
        g.add_blocks(bad)
    assert g.blocks().sum() == 12     # unchanged
    g.close()
    r = B.Sim(W.make(128, 64, 32, "static", 1, static_ext=(48, 16, 96, 32)),
              np.zeros((65, 129)))
    with pytest.raises(B.DmrError):
        r.blocks()
    r.close()


def test_union_with_townsend_and_recombination():
    """The full Eq. (4) source on the union level (same continuity update)."""
    cfg, m = _static_l(periods=16)
    cfg.update(erms_over_ebd=2.0, source_model="townsend", beta_rec=1.0)
    sb, sf = W.seeds(cfg, [(56.5 * DX, 32 * DX)], [1e20])
    g, o = both(cfg, sb, sf)
    g.add_blocks(m)
    o.add_blocks(m)
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    assert_parity(g, o, O.derived(cfg)["n_c"], tag="union townsend")
    g.close()


def test_full_size_rectangle_of_blocks_is_the_patch():
    """Config 2 at full size (coarse 4096x2048, 8-seed layout) with the fine
    level fixed to the seeds' bounding box and a plane-wave packet loaded
    just left of it (as in test_gpu_parity.py, whose rectangle run is
    compared with the oracle at this size): the union kernels (large level:
    16-row tiles) give the rectangular patch's run bit for bit over 4
    periods while the packet crosses into the level."""
    cfg = W.config2(periods=4)
    centres, peaks = W.config2_seed_layout(cfg)
    sb, sf = W.seeds(cfg, centres, peaks)
    ext = (2896, 352, 3664, 1888)
    cr = dict(cfg, mode="static", static_ext=ext)
    cu = dict(cr, regrid_rule="union")
    E0 = O.derived(cfg)["E0"]
    a = B.Sim(cr, sb, sf)
    load_plane_packet(a, cfg, E0, ext[0] - 72, 64)
    a.step(cfg["steps"])
    ref = {(f, lv): a.get(f, lv) for lv in (0, 1) for f in FIELDS}
    a.close()
    assert np.abs(ref[("ey", 1)]).max() > 0.5 * E0
    b = B.Sim(cu, sb, sf)
    assert b.patch() == ext and b.blocks().sum() == 48 * 96
    load_plane_packet(b, cfg, E0, ext[0] - 72, 64)
    b.step(cfg["steps"])
    for (f, lv), x in ref.items():
        assert np.array_equal(x, b.get(f, lv)), (f, lv)
    b.close()


def test_full_size_blocks_match_oracle():
    """Config 2 at full size: the union's active blocks at t = 0 equal the
    oracle's (integer decisions on the same float32 density)."""
    cfg = dict(W.config2(periods=1), regrid_rule="union")
    centres, peaks = W.config2_seed_layout(cfg)
    sb, sf = W.seeds(cfg, centres, peaks)
    g = B.Sim(cfg, sb, sf)
    gb = g.blocks()
    g.close()
    o = O.Sim(cfg, sb, sf)
    ob = o.blocks()
    print("config 2 union: %d active blocks" % gb.sum(), flush=True)
    assert gb.sum() > 8 and np.array_equal(gb, ob)
    o.close()
