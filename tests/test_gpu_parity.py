"""GPU (float32, HIP) against the FP64 oracle on the same seeded inputs.

Tolerance: relative L2 <= 1e-4 per field group (E = (Ex, Ey), Hz,
J = (Jx, Jy), E_rms^2) per level and per component (each against its own
norm, with the scattered-field allowance of `gpu_helpers.component_limit`),
<= 1e-3 on log(max(n, 1e-12 n_c)); integer regrid results (block flags,
prefix sum, compacted list, patch extents) equal.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_13276_amd import binding as B
from paper_2105_13276_amd import workloads as W

from gpu_helpers import assert_parity, both, load_plane_packet

pytestmark = pytest.mark.gpu

LAM = 299792458.0 / 110e9


def _nc(cfg):
    return O.derived(cfg)["n_c"]


def test_uniform_config0():
    """Plain method: 256x128 at lambda/64, 40 periods (5120 steps)."""
    cfg = W.config0()
    sb, _ = W.seeds(cfg)
    g, o = both(cfg, sb)
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    g.sync()
    assert g.time()[1] == o.time()[1] == cfg["steps"]
    assert_parity(g, o, _nc(cfg), levels=(0,), tag="config0")


@pytest.mark.parametrize("nx,ny,bc", [(200, 72, "mur"), (130, 66, "pec")])
def test_uniform_ragged(nx, ny, bc):
    """Grids that are not multiples of the 64 x TY tile: ragged tails on both
    axes; PEC walls; a stronger field so density and current evolve."""
    cfg = W.make(nx, ny, 32, "uniform", 12, bc_x=bc, bc_y=bc, erms_over_ebd=2.0)
    dx = LAM / 32
    sb = W.gaussian_seed(nx, ny, dx, [(0.6 * nx * dx, 0.45 * ny * dx)], [3e18], LAM / 20)
    g, o = both(cfg, sb)
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    assert_parity(g, o, _nc(cfg), levels=(0,), tag="ragged %dx%d %s" % (nx, ny, bc))


def test_static_patch():
    cfg = W.make(128, 64, 32, "static", 20, static_ext=(48, 16, 96, 48),
                 erms_over_ebd=2.0)
    sb, sf = W.seeds(cfg)
    g, o = both(cfg, sb, sf)
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    assert g.patch() == o.patch() == (48, 16, 96, 48)
    assert_parity(g, o, _nc(cfg), tag="static")


def test_dynamic_growth():
    """The patch grows from 1x1 to 2x1 blocks during the run (seed half a cell
    off a block edge, strong field)."""
    dxc = LAM / 32
    cfg = W.make(96, 48, 32, "dynamic", 60, erms_over_ebd=2.5)
    sb, sf = W.seeds(cfg, [(59.5 * dxc, 24 * dxc)], [1e17])
    g, o = both(cfg, sb, sf)
    p0 = g.patch()
    assert p0 == o.patch()
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    assert g.patch() == o.patch() != p0
    fg, sg, lg, cg = g.regrid_info()
    fo, so, lo, co = o.regrid_info()
    assert (fg == fo).all() and (sg == so).all() and cg == co and (lg == lo).all()
    assert_parity(g, o, _nc(cfg), tag="growth")


def test_config1_dmr_full():
    """Config 1 as benchmarked: coarse 512x256 at lambda/32, r = 2 patch,
    regrid every 4 periods, 200 periods (12800 coarse steps)."""
    cfg = W.config1_dmr()
    sb, sf = W.seeds(cfg)
    g, o = both(cfg, sb, sf)
    assert g.patch() == o.patch() == (240, 112, 272, 144)
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    g.sync()
    assert g.patch() == o.patch()
    fg, sg, lg, cg = g.regrid_info()
    fo, so, lo, co = o.regrid_info()
    assert (fg == fo).all() and (sg == so).all() and cg == co and (lg == lo).all()
    assert_parity(g, o, _nc(cfg), tag="config1")


def test_config1_uniform_fine_prefix():
    """The uniform-fine 1024x512 run of config 1 at full size (the launch
    shape the benchmark times) over its first 16 periods."""
    cfg = W.config1_uniform(periods=16)
    sb, _ = W.seeds(cfg)
    g, o = both(cfg, sb)
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    assert_parity(g, o, _nc(cfg), levels=(0,), tag="config1-uniform")


# config 2's 8-seed bounding box (coarse cells); the incident wave would need
# ~90 periods to reach it, so the full-size tests load a plane-wave packet
# just left of it (2 wavelengths long, ending 8 cells before the patch)
CONFIG2_BOX = (2896, 352, 3664, 1888)
CONFIG2_PACKET = (CONFIG2_BOX[0] - 72, 64)


def test_config2_full_size_wave_on_the_patch():
    """Config 2 at full size (coarse 4096x2048, r = 2 patch over the 8-seed
    layout, E_rms/E_bd = 1.5) in the launch shape the large benchmark rows
    use (4.7 M fine cells: one-substep patch launches), over 4 periods (one
    period of window filling, three of continuity steps, the growth test at
    step 256), with a right-going plane-wave packet of the incident amplitude
    loaded just left of the patch at t = 0 (`load_plane_packet`): it crosses
    the coarse/fine boundary and travels ~90 fine columns into the patch.
    The level-1 field must carry it and agree with the oracle like every
    other case."""
    cfg = W.config2(periods=4)
    centres, peaks = W.config2_seed_layout(cfg)
    sb, sf = W.seeds(cfg, centres, peaks)
    g, o = both(cfg, sb, sf)
    print("config 2: patch %s" % (g.patch(),), flush=True)
    assert g.patch() == o.patch() == CONFIG2_BOX
    fg, sg, lg, cg = g.regrid_info()
    fo, so, lo, co = o.regrid_info()
    assert (fg == fo).all() and (sg == so).all() and cg == co and (lg == lo).all()
    E0 = O.derived(cfg)["E0"]
    for s in (g, o):
        load_plane_packet(s, cfg, E0, *CONFIG2_PACKET)
    g.step(cfg["steps"])
    o.step(cfg["steps"])
    g.sync()
    assert g.patch() == o.patch()
    colmax = np.abs(o.get("ey", 1)).max(axis=0)
    print("config 2: max |Ey| on the patch %.2f E0, %d fine columns above 0.1 E0"
          % (colmax.max() / E0, (colmax > 0.1 * E0).sum()), flush=True)
    assert colmax.max() > 0.5 * E0 and (colmax > 0.1 * E0).sum() >= 64
    assert_parity(g, o, _nc(cfg), tag="config2-wave")


@pytest.mark.parametrize("r", [2, 4])
def test_fused_forms_bitwise(r):
    """The one-launch step (base step + both patch substeps), the two-substep
    patch launch, two one-substep tile launches and two one-substep streaming
    launches give the same bits (each entity is computed with the same
    operations in all of them); for r = 4 the substeps run as two
    two-substep launches or four one-substep launches."""
    import os
    if r == 2:
        cfg = W.make(128, 64, 32, "dynamic", 10, erms_over_ebd=3.0)
        sb, sf = W.seeds(cfg, [(80 * LAM / 32, 32 * LAM / 32)], [3e17])
        forms = (("combined", {}), ("fused", {"DMR_COMBINE": "0"}),
                 ("separate", {"DMR_COMBINE": "0", "DMR_FUSE": "0", "DMR_FINE_STREAM": "0"}),
                 ("streamed", {"DMR_COMBINE": "0", "DMR_FUSE": "0", "DMR_FINE_STREAM": "1"}))
    else:
        cfg = W.make(64, 32, 16, "dynamic", 10, r=4, block=8, erms_over_ebd=3.0)
        sb, sf = W.seeds(cfg, [(40 * LAM / 16, 16 * LAM / 16)], [3e17])
        forms = (("combined", {}), ("separate", {"DMR_FUSE": "0"}))
    cfg["regrid_every"] = 2 * cfg["steps_per_period"]
    runs = {}
    for name, env in forms:
        old = {k: os.environ.get(k) for k in ("DMR_COMBINE", "DMR_FUSE", "DMR_FINE_STREAM")}
        os.environ.update(env)
        try:
            g = B.Sim(cfg, sb, sf)
        finally:
            for k, v in old.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        p0 = g.patch()
        g.step(cfg["steps"])
        runs[name] = {(f, lv): g.get(f, lv) for lv in (0, 1)
                      for f in ("hz", "ex", "ey", "jx", "jy", "n", "acc", "ring")}
        runs[name]["patch"] = (p0, g.patch())
        g.close()
    print("r = %d patch %s" % (r, runs["combined"]["patch"]), flush=True)
    for name, _ in forms[1:]:
        assert runs[name]["patch"] == runs["combined"]["patch"]
        for k, v in runs["combined"].items():
            if k != "patch":
                assert np.array_equal(v, runs[name][k]), (name, k)


def test_patch_tile_widths_bitwise():
    """The combined step's patch tiles at widths 64, 32 and 16 (the width is
    picked by patch size; DMR_TW forces one) give the same bits: the width
    changes which tile computes an entity, not how."""
    import os
    cfg = W.make(128, 64, 32, "dynamic", 10, erms_over_ebd=3.0)
    cfg["regrid_every"] = 2 * cfg["steps_per_period"]
    sb, sf = W.seeds(cfg, [(80 * LAM / 32, 32 * LAM / 32)], [3e17])
    runs = {}
    for tw in ("64", "32", "16"):
        old = os.environ.get("DMR_TW")
        os.environ["DMR_TW"] = tw
        try:
            g = B.Sim(cfg, sb, sf)
        finally:
            if old is None:
                os.environ.pop("DMR_TW", None)
            else:
                os.environ["DMR_TW"] = old
        g.step(cfg["steps"])
        runs[tw] = {(f, lv): g.get(f, lv) for lv in (0, 1)
                    for f in ("hz", "ex", "ey", "jx", "jy", "n", "acc", "ring")}
        runs[tw]["patch"] = g.patch()
        g.close()
    for tw in ("32", "16"):
        for k, v in runs["64"].items():
            assert np.array_equal(v, runs[tw][k]) if k != "patch" else v == runs[tw][k], (tw, k)


def test_merged_continuity_bitwise():
    """The continuity step of both levels in one launch (coarse blocks, patch
    blocks and one block for the patch boundary lines; the default for small
    rectangular patches) against a launch per level, over 10 periods with
    growth (window filling, then density updates): the same bits."""
    cfg = W.make(128, 64, 32, "dynamic", 10, erms_over_ebd=3.0)
    sb, sf = W.seeds(cfg, [(80 * LAM / 32, 32 * LAM / 32)], [3e17])
    cfg["regrid_every"] = 2 * cfg["steps_per_period"]
    a = _env_run(cfg, sb, sf, {"DMR_CONT_MERGE": "1"}, cfg["steps"])
    b = _env_run(cfg, sb, sf, {"DMR_CONT_MERGE": "0"}, cfg["steps"])
    assert a["patch"] == b["patch"]
    assert np.abs(a[("n", 1)]).max() > 0
    for k, v in a.items():
        if k != "patch":
            assert np.array_equal(v, b[k]), k


def test_merged_continuity_bitwise_r4():
    """The one-launch continuity step with an r = 4 patch (four patch nodes per
    coarse node on the boundary lines, linear along them) against a launch
    per level, over 10 periods with growth: the same bits."""
    cfg = W.make(64, 32, 16, "dynamic", 10, r=4, block=8, erms_over_ebd=3.0)
    sb, sf = W.seeds(cfg, [(40 * LAM / 16, 16 * LAM / 16)], [3e17])
    cfg["regrid_every"] = 2 * cfg["steps_per_period"]
    a = _env_run(cfg, sb, sf, {"DMR_CONT_MERGE": "1"}, cfg["steps"])
    b = _env_run(cfg, sb, sf, {"DMR_CONT_MERGE": "0"}, cfg["steps"])
    assert a["patch"] == b["patch"]
    assert np.abs(a[("n", 1)]).max() > 0
    for k, v in a.items():
        if k != "patch":
            assert np.array_equal(v, b[k]), k


def test_r4_patch_tile_widths_bitwise():
    """r = 4 with 4-row tiles runs both pairs of substeps in the frame tile of
    the combined step; its tiles at widths 16, 32 and 64 and the four
    one-substep launches give the same bits."""
    cfg = W.make(64, 32, 16, "dynamic", 10, r=4, block=8, erms_over_ebd=3.0)
    sb, sf = W.seeds(cfg, [(40 * LAM / 16, 16 * LAM / 16)], [3e17])
    cfg["regrid_every"] = 2 * cfg["steps_per_period"]
    runs = {tw: _env_run(cfg, sb, sf, {"DMR_TW": tw, "DMR_TY": "4"}, cfg["steps"])
            for tw in ("16", "32", "64")}
    runs["separate"] = _env_run(cfg, sb, sf, {"DMR_FUSE": "0"}, cfg["steps"])
    assert np.abs(runs["16"][("ey", 1)]).max() > 0
    for name in ("32", "64", "separate"):
        for k, v in runs["16"].items():
            assert np.array_equal(v, runs[name][k]) if k != "patch" else v == runs[name][k], (name, k)


def _env_run(cfg, sb, sf, env, steps):
    import os
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        g = B.Sim(cfg, sb, sf)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    g.step(steps)
    out = {(f, lv): g.get(f, lv) for lv in (0, 1)
           for f in ("hz", "ex", "ey", "jx", "jy", "n", "acc", "ring")}
    out["patch"] = g.patch()
    g.close()
    return out


@pytest.mark.parametrize("gamma", [1e-3, 0.0])
def test_streamed_patch_substep_bitwise_large(gamma):
    """The streaming form of the one-substep patch launch (selectable for
    large patches, off by default) against the tile form on a patch of 192 x 96 fine cells
    (several column waves, several row segments, odd offsets of the wave
    columns against the tiles), with and without the interface filter, with
    the incident wave and the density evolving: the same bits."""
    cfg = W.make(128, 64, 32, "static", 12, static_ext=(16, 8, 112, 56),
                 erms_over_ebd=3.0, fine_filter=gamma)
    sb, sf = W.seeds(cfg, [(70 * LAM / 32, 30 * LAM / 32)], [3e18])
    base = {"DMR_COMBINE": "0", "DMR_FUSE": "0"}
    a = _env_run(cfg, sb, sf, dict(base, DMR_FINE_STREAM="0"), cfg["steps"])
    b = _env_run(cfg, sb, sf, dict(base, DMR_FINE_STREAM="1"), cfg["steps"])
    assert np.abs(a[("ey", 1)]).max() > 0
    for k, v in a.items():
        if k == "patch":
            assert v == b[k]
        else:
            assert np.array_equal(v, b[k]), k
