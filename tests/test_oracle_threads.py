"""The oracle's OpenMP loops update independent entities, so a run gives the
same bits for any thread count (refined dynamic run with growth, union of
blocks, Townsend source)."""
import numpy as np
import pytest

from paper_2105_13276_amd import workloads as W

LAM = 299792458.0 / 110e9
FIELDS = ("hz", "ex", "ey", "jx", "jy", "n", "acc", "ring")


def _run(oracle_mod, cfg, sb, sf, threads):
    oracle_mod.set_threads(threads)
    try:
        s = oracle_mod.Sim(cfg, sb, sf)
        s.step(cfg["steps"])
        out = {(f, lv): s.get(f, lv) for lv in (0, 1) for f in FIELDS}
        out["patch"] = s.patch()
        return out
    finally:
        oracle_mod.set_threads(0)


@pytest.mark.parametrize("rule", ["blocks", "union"])
def test_thread_count_does_not_change_bits(oracle_mod, rule):
    dx = LAM / 32
    cfg = W.make(96, 48, 32, "dynamic", 12, erms_over_ebd=3.0, regrid_rule=rule,
                 block=8 if rule == "union" else 16, source_model="townsend",
                 beta_rec=1.0)
    cfg["regrid_every"] = 2 * cfg["steps_per_period"]
    sb, sf = W.seeds(cfg, [(60.5 * dx, 24 * dx)], [3e17])
    a = _run(oracle_mod, cfg, sb, sf, 1)
    b = _run(oracle_mod, cfg, sb, sf, 4)
    assert a["patch"] == b["patch"] != (0, 0, 0, 0)
    for k in a:
        if k != "patch":
            assert np.array_equal(a[k], b[k]), k
