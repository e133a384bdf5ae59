"""Batched form: every instance of one batched run equals its own plain run
bit for bit, whatever launch shape the batch uses (segment rows, load depth,
fine tile rows, graph replay or not); and one instance checked against the
FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_13276_amd import binding as B
from paper_2105_13276_amd import workloads as W

from gpu_helpers import assert_parity

pytestmark = pytest.mark.gpu

FIELDS = ("hz", "ex", "ey", "jx", "jy", "n", "acc", "ring")


def _mixed(count=6, periods=12):
    cfgs, seeds = W.config3(count, periods)
    # smaller grids than the benchmark's so the plain runs stay quick
    out_c, out_s = [], []
    for k, c in enumerate(cfgs):
        side = [128, 192, 256][k % 3]
        c2 = W.make(side, side // 2, 32, "dynamic", periods, erms_over_ebd=c["erms_over_ebd"],
                    p_torr=c["p_torr"], freq_hz=c["freq_hz"], L_amb=c["L_amb"])
        out_c.append(c2)
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
                                   (2, 2, 8, 0)])
def test_batch_launch_shape_invariance(shape):
    cfgs, seeds = _mixed(count=4, periods=8)
    steps = cfgs[0]["steps"]
    ref = B.Batch(cfgs, seeds)
    ref.set_config(16, 2, 4, 0)
    ref.step(steps)
    bt = B.Batch(cfgs, seeds)
    bt.set_config(*shape)
    bt.step(steps)
    for k in range(len(cfgs)):
        _same(bt.instances[k], ref.instances[k])


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
    bt.step(cfgs[0]["steps"])
    grown = 0
    for k, (c, s) in enumerate(zip(cfgs, seeds)):
        g = B.Sim(c, *s)
        p0 = g.patch()
        g.step(c["steps"])
        inst = bt.instances[k]
        assert inst.patch() == g.patch()
        grown += g.patch() != p0
        _same(inst, g)
    print("r = 4 batch: %d of 3 patches grew" % grown, flush=True)
    assert grown >= 1
