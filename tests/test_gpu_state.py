"""Checkpoint / restart through dmr_save / dmr_load: a run continued from a
saved state equals the uninterrupted run bit for bit (the time stepping is
deterministic), across a patch growth, from host and device buffers."""
import numpy as np
import pytest

from paper_2105_13276_amd import binding as B
from paper_2105_13276_amd import workloads as W

pytestmark = pytest.mark.gpu

LAM = 299792458.0 / 110e9
FIELDS = ["hz", "ex", "ey", "jx", "jy", "n", "acc", "ring"]


def _case():
    # grows at step 512 (regrid every 2 periods, the seed spreads); the save
    # at step 300 lies inside the first patch, mid-window (300 % 8 != 0)
    cfg = W.make(96, 48, 32, "dynamic", 14, erms_over_ebd=3.0)
    cfg["regrid_every"] = 2 * cfg["steps_per_period"]
    sb, _ = W.seeds(cfg, [(96 * 0.62 * LAM / 32, 24 * LAM / 32)], [3e17])
    return cfg, sb


def _snapshot(g):
    out = {"patch": g.patch(), "time": g.time()}
    for lev in (0, 1):
        if lev == 1 and g.patch() == (0, 0, 0, 0):
            continue
        for f in FIELDS:
            out[(f, lev)] = g.get(f, lev)
    return out


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), k
        else:
            assert a[k] == b[k], k


@pytest.mark.parametrize("on_device", [False, True])
def test_restart_equals_uninterrupted_run(on_device):
    import torch
    cfg, sb = _case()
    g = B.Sim(cfg, sb, None)
    g.step(300)
    p0 = g.patch()
    if on_device:
        buf = torch.empty(g.state_bytes(), dtype=torch.uint8, device="cuda")
        g.save(buf)
    else:
        buf = g.save()
    g.step(400)
    ref = _snapshot(g)
    assert ref["patch"] != p0, "the continued run should grow the patch"
    # a fresh handle with the same parameters (seed irrelevant: overwritten)
    h = B.Sim(cfg, np.zeros_like(sb), None)
    h.load(buf)
    assert h.time()[1] == 300 and h.patch() == p0
    h.step(400)
    _same(_snapshot(h), ref)
    # the same handle, rewound
    g.load(buf)
    g.step(400)
    _same(_snapshot(g), ref)
    g.close()
    h.close()


def test_load_rejects_other_parameters_and_short_buffers():
    cfg, sb = _case()
    g = B.Sim(cfg, sb, None)
    g.step(16)
    buf = g.save()
    other = dict(cfg, erms_over_ebd=2.9)
    h = B.Sim(other, sb, None)
    with pytest.raises(B.DmrError, match="EINVAL"):
        h.load(buf)
    with pytest.raises(B.DmrError, match="ENOMEM"):
        g.load(buf[:-1])
    with pytest.raises(B.DmrError, match="ENOMEM"):
        g.save(np.empty(16, np.uint8))
    junk = np.zeros_like(buf)
    with pytest.raises(B.DmrError, match="EINVAL"):
        g.load(junk)
    # a rejected load leaves the handle as it was
    t = g.time()
    g.step(8)
    assert g.time()[1] == t[1] + 8
    g.close()
    h.close()


def test_union_restart_equals_uninterrupted_run():
    """The union-of-blocks level: the state carries the block map; a restart
    before a growth rebuilds the tile list and continues bit for bit."""
    cfg = W.make(128, 64, 32, "dynamic", 14, block=8, erms_over_ebd=3.0, regrid_rule="union")
    cfg["regrid_every"] = 2 * cfg["steps_per_period"]
    dx = LAM / 32
    sb, sf = W.seeds(cfg, [(46.5 * dx, 21 * dx), (92.5 * dx, 45.5 * dx)], [3e17, 2e17])
    g = B.Sim(cfg, sb, sf)
    g.step(300)
    b0 = g.blocks().copy()
    buf = g.save()
    g.step(500)
    ref = _snapshot(g)
    assert g.blocks().sum() > b0.sum(), "the continued run should grow the level"
    h = B.Sim(cfg, np.zeros_like(sb), None)   # its own (empty) level is replaced
    h.load(buf)
    assert np.array_equal(h.blocks(), b0)
    h.step(500)
    _same(ref, _snapshot(h))
    assert np.array_equal(h.blocks(), g.blocks())
    g.close()
    h.close()


def test_load_checks_the_header_before_changing_the_handle():
    """A saved state whose header names extents outside the domain, off the
    block grid, a bad tile height, or (union level) a block map that does not
    match its extents is refused with EINVAL, and the handle keeps its own
    state (the extents decide which fine rows a load writes)."""
    import struct
    cfg, sb = _case()
    g = B.Sim(cfg, sb, None)
    g.step(24)
    buf = g.save()
    before = _snapshot(g)
    # StateHeader: magic[8], version, header_bytes (u32), params_hash,
    # total_bytes (u64), step, blocks (i64), has_patch, ext[4], ty1 (i32)
    off_ext = 8 + 4 + 4 + 8 + 8 + 8 + 8 + 4
    off_ty1 = off_ext + 16
    bad = []
    # outside the domain, off the block grid, negative, inverted
    for ext in ((32, 16, 112, 32), (32, 16, 40, 32), (-16, 16, 32, 32), (48, 16, 32, 32)):
        b = buf.copy()
        b[off_ext:off_ext + 16] = np.frombuffer(struct.pack("<4i", *ext), np.uint8)
        bad.append(b)
    b = buf.copy()
    b[off_ty1:off_ty1 + 4] = np.frombuffer(struct.pack("<i", 5), np.uint8)
    bad.append(b)
    for b in bad:
        with pytest.raises(B.DmrError, match="EINVAL"):
            g.load(b)
        _same(_snapshot(g), before)
    g.close()


def test_union_load_checks_the_block_map():
    cfg = W.make(128, 64, 32, "dynamic", 2, block=8, erms_over_ebd=3.0, regrid_rule="union")
    dx = LAM / 32
    sb, sf = W.seeds(cfg, [(46.5 * dx, 21 * dx)], [3e17])
    g = B.Sim(cfg, sb, sf)
    g.step(16)
    buf = g.save()
    before = _snapshot(g)
    nbx, nby = 128 // 8, 64 // 8
    map0 = len(buf) - ((nbx * nby + 255) // 256) * 256
    assert np.array_equal(buf[map0:map0 + nbx * nby].reshape(nby, nbx), g.blocks())
    for b_id in (0, nbx * nby - 1, 5 * nbx + 9):
        # a block on the outer margin; a block inside the margins but away
        # from the saved extents
        b = buf.copy()
        if b[map0 + b_id]:
            continue
        b[map0 + b_id] = 1
        with pytest.raises(B.DmrError, match="EINVAL"):
            g.load(b)
        _same(_snapshot(g), before)
    g.close()
