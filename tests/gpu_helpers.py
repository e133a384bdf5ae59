"""Shared helpers of the GPU parity tests: run the HIP path and the FP64
oracle on the same seeded inputs and compare them field by field."""
import numpy as np

from oracle import oracle as O
from paper_2105_13276_amd import binding as B

GROUPS = {"E": ("ex", "ey"), "H": ("hz",), "J": ("jx", "jy"), "Erms2": ("erms2",)}


def rel_l2(got, ref):
    got = [np.asarray(g, np.float64) for g in got]
    ref = [np.asarray(r, np.float64) for r in ref]
    num = np.sqrt(sum(((g - r) ** 2).sum() for g, r in zip(got, ref)))
    den = np.sqrt(sum((r ** 2).sum() for r in ref))
    return float(num / den) if den > 0 else float(num)


def errors(gpu, orc, level, n_c):
    """Relative L2 error of the float32 GPU state against the FP64 oracle per
    field group, and of log(max(n, 1e-12 n_c))."""
    out = {}
    for g, names in GROUPS.items():
        out[g] = rel_l2([gpu.get(f, level) for f in names],
                        [orc.get(f, level) for f in names])
    floor = 1e-12 * n_c
    ln_g = np.log(np.maximum(gpu.get("n", level).astype(np.float64), floor))
    ln_o = np.log(np.maximum(orc.get("n", level), floor))
    out["log_n"] = rel_l2([ln_g], [ln_o])
    return out


def both(cfg, seed_base, seed_fine=None):
    g = B.Sim(cfg, seed_base, seed_fine)
    o = O.Sim(cfg, seed_base, seed_fine)
    return g, o


def assert_parity(gpu, orc, n_c, levels=(0, 1), tol=1e-4, tol_logn=1e-3, tag=""):
    report = {}
    for lv in levels:
        e = errors(gpu, orc, lv, n_c)
        report[lv] = e
        print("%s level %d: %s" % (tag, lv, " ".join("%s=%.2e" % kv for kv in e.items())),
              flush=True)
    for lv, e in report.items():
        for k, v in e.items():
            lim = tol_logn if k == "log_n" else tol
            assert v <= lim, "%s level %d %s rel L2 %.3e > %.1e" % (tag, lv, k, v, lim)
    return report
