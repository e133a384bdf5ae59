"""Batched form: every instance of one batched run equals its own plain run
bit for bit, whatever launch shape the batch uses (segment rows, load depth,
fine tile rows, graph replay or not, subcycle schedule: one-substep
launches, a two-substep launch, or the base step and both substeps in one
launch); and one instance checked against the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_13276_amd import binding as B
from paper_2105_13276_amd import workloads as W

from gpu_helpers import assert_parity

pytestmark = pytest.mark.gpu

FIELDS = ("hz", "ex", "ey", "jx", "jy", "n", "acc", "ring")


def _mixed(count=6, periods=12, grow=False):
    """Config-3-like instances on smaller grids (so the plain runs stay
    quick).  grow: a strong field and an off-centre seed half a cell from a
    block edge in every other instance, whose patch then grows during the
    run (regrid every 2 periods)."""
    cfgs, seeds = W.config3(count, periods)
    out_c, out_s = [], []
    for k, c in enumerate(cfgs):
        side = [128, 192, 256][k % 3]
        strong = grow and k % 2 == 0
        c2 = W.make(side, side // 2, 32, "dynamic", periods,
                    erms_over_ebd=4.0 if strong else c["erms_over_ebd"],
                    p_torr=c["p_torr"], freq_hz=c["freq_hz"], L_amb=c["L_amb"])
        if grow:
            c2["regrid_every"] = 2 * c2["steps_per_period"]
        out_c.append(c2)
        if strong:
            dx = 299792458.0 / c2["freq_hz"] / 32
            out_s.append(W.seeds(c2, [((side // 2 + 11.5) * dx, side // 4 * dx)], [3e17]))
        else:
            out_s.append(W.seeds(c2))
    return out_c, out_s


def _same(a, b):
    for lv in (0, 1):
        for f in FIELDS:
            x, y = a.get(f, lv), b.get(f, lv)
            assert x.shape == y.shape and np.array_equal(x, y), (lv, f)


def test_batch_equals_plain_runs():
    cfgs, seeds = _mixed()
    steps = cfgs[0]["steps"]
    bt = B.Batch(cfgs, seeds)
    bt.step(steps)            # tunes on real steps, then replays graphs
    bt.sync()
    print("batch config", bt.config(), flush=True)
    for k, (c, s) in enumerate(zip(cfgs, seeds)):
        g = B.Sim(c, *s)
        g.step(steps)
        inst = bt.instances[k]
        assert inst.time()[1] == steps
        assert inst.patch() == g.patch()
        _same(inst, g)


@pytest.mark.parametrize("shape", [(4, 4, 4, 0), (32, 2, 16, 1), (8, 4, 8, 1), (2, 2, 4, 1),
                                   (2, 2, 8, 0), (8, 4, 8, 1, "fused"), (4, 4, 16, 0, "fused"),
                                   (2, 2, 4, 1, "combined"), (16, 2, 16, 0, "combined"),
                                   (8, 4, 8, 1, "combined")])
def test_batch_launch_shape_invariance(shape):
    """12 periods with regrid every 2 periods: patches grow (tables rebuilt
    at both step parities of the two-substep schedules' buffer swap)."""
    cfgs, seeds = _mixed(count=4, periods=12, grow=True)
    steps = cfgs[0]["steps"]
    ref = B.Batch(cfgs, seeds)
    ref.set_config(16, 2, 4, 0)
    p0 = [ref.instances[k].patch() for k in range(len(cfgs))]
    ref.step(steps)
    bt = B.Batch(cfgs, seeds)
    bt.set_config(*shape)
    assert bt.config()[4] == (shape[4] if len(shape) > 4 else "separate")
    bt.step(steps)
    grew = sum(ref.instances[k].patch() != p0[k] for k in range(len(cfgs)))
    print("shape %s: %d patches grew" % (shape, grew), flush=True)
    assert grew >= 1
    for k in range(len(cfgs)):
        assert bt.instances[k].patch() == ref.instances[k].patch()
        _same(bt.instances[k], ref.instances[k])
    # and the plain runs of the same instances
    for k, (c, s) in enumerate(zip(cfgs[:2], seeds[:2])):
        g = B.Sim(c, *s)
        g.step(steps)
        _same(bt.instances[k], g)
        g.close()


def test_batch_instance_vs_oracle():
    cfgs, seeds = _mixed(count=3, periods=12)
    bt = B.Batch(cfgs, seeds)
    bt.step(cfgs[0]["steps"])
    k = 1
    o = O.Sim(cfgs[k], *seeds[k])
    o.step(cfgs[k]["steps"])
    assert bt.instances[k].patch() == o.patch()
    assert_parity(bt.instances[k], o, O.derived(cfgs[k])["n_c"], tag="batch[1]")


def _mixed_union(count=4, periods=12):
    """Union-of-blocks instances of three sizes, two seeds each, growing."""
    cfgs, seeds = W.config3(count, periods)
    out_c, out_s = [], []
    for k, c in enumerate(cfgs):
        side = [128, 192, 256][k % 3]
        c2 = W.make(side, side // 2, 32, "dynamic", periods, erms_over_ebd=3.0,
                    p_torr=c["p_torr"], freq_hz=c["freq_hz"], L_amb=c["L_amb"],
                    block=8, regrid_rule="union")
        c2["regrid_every"] = 2 * c2["steps_per_period"]
        dx = 299792458.0 / c2["freq_hz"] / 32
        cen = [(0.45 * side * dx, 0.15 * side * dx), (0.75 * side * dx, 0.35 * side * dx)]
        out_c.append(c2)
        out_s.append(W.seeds(c2, cen, [3e17, 2e17]))
    return out_c, out_s


def test_union_batch_equals_plain_runs():
    cfgs, seeds = _mixed_union()
    steps = cfgs[0]["steps"]
    bt = B.Batch(cfgs, seeds)
    b0 = [bt.instances[k].blocks().sum() for k in range(len(cfgs))]
    bt.step(steps)
    bt.sync()
    print("union batch config", bt.config(), "blocks", b0, "->",
          [bt.instances[k].blocks().sum() for k in range(len(cfgs))], flush=True)
    grew = 0
    for k, (c, s) in enumerate(zip(cfgs, seeds)):
        g = B.Sim(c, *s)
        g.step(steps)
        inst = bt.instances[k]
        assert np.array_equal(inst.blocks(), g.blocks())
        grew += int(inst.blocks().sum() > b0[k])
        _same(inst, g)
    assert grew >= 1


def test_union_batch_launch_shape_invariance():
    cfgs, seeds = _mixed_union(count=3, periods=8)
    steps = cfgs[0]["steps"]
    ref = B.Batch(cfgs, seeds)
    ref.set_config(16, 2, 4, 0)
    ref.step(steps)
    bt = B.Batch(cfgs, seeds)
    bt.set_config(32, 2, 16, 1)
    bt.step(steps)
    for k in range(len(cfgs)):
        _same(bt.instances[k], ref.instances[k])
    # union levels run the one-substep schedule only
    for sched in ("fused", "combined"):
        with pytest.raises(B.DmrError, match="EINVAL"):
            bt.set_config(8, 4, 8, 1, sched)


def test_batch_config3_full_size_prefix():
    """The benchmark's batch at full size (64 instances drawn as config 3:
    sides 256/512/1024, 35/110/170 GHz, 100-760 Torr, tuned launch shape,
    graph replay) over its first 4 periods (one growth test): every instance
    equals its own plain run bit for bit."""
    cfgs, seeds = W.config3(64, periods=4)
    steps = cfgs[0]["steps"]
    bt = B.Batch(cfgs, seeds)
    bt.step(steps)
    bt.sync()
    print("config 3 batch: launch shape", bt.config(), flush=True)
    for k, (c, s) in enumerate(zip(cfgs, seeds)):
        g = B.Sim(c, *s)
        g.step(steps)
        inst = bt.instances[k]
        assert inst.patch() == g.patch(), k
        _same(inst, g)
        g.close()


def test_r4_batch_equals_plain_runs():
    """Refinement factor 4 in the batched form: four one-substep fine launches
    per coarse step (substep 2 keeps its Hz for the fine -> coarse transfer
    after substep 4), bit for bit the plain runs (which take the substeps
    as two two-substep launches)."""
    lam = 299792458.0 / 110e9
    cfgs, seeds = [], []
    # the first grows its patch within the run (as in the plain r = 4 growth test)
    for side, e, x, pk in [(48, 2.5, 29.75, 1e17), (64, 2.5, 31.5, 1e17), (96, 2.0, 47.5, 3e17)]:
        c = W.make(side, side // 2, 16, "dynamic", 60, r=4, block=8, erms_over_ebd=e)
        cfgs.append(c)
        seeds.append(W.seeds(c, [(x * lam / 16, side // 4 * lam / 16)], [pk]))
    bt = B.Batch(cfgs, seeds)
    bf = B.Batch(cfgs, seeds)   # the two two-substep launches per coarse step
    bf.set_config(8, 4, 4, 1, "fused")
    with pytest.raises(B.DmrError, match="EINVAL"):   # combined: r = 2 only
        bf.set_config(8, 4, 4, 1, "combined")
    bf.set_config(8, 4, 4, 1, "fused")
    bt.step(cfgs[0]["steps"])
    bf.step(cfgs[0]["steps"])
    grown = 0
    for k, (c, s) in enumerate(zip(cfgs, seeds)):
        g = B.Sim(c, *s)
        p0 = g.patch()
        g.step(c["steps"])
        inst = bt.instances[k]
        assert inst.patch() == g.patch() == bf.instances[k].patch()
        grown += g.patch() != p0
        _same(inst, g)
        _same(bf.instances[k], g)
    print("r = 4 batch: %d of 3 patches grew" % grown, flush=True)
    assert grown >= 1
