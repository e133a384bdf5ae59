"""An x-edge-rich refined case (test input only).

A lossless (PEC-walled) cavity of 2 x 1 wavelengths is started in its
TE_z (2, 1) mode, Hz = H0 cos(2 pi x / Lx) cos(pi y / Ly) with E = 0, so that
Ex and Ey carry equal amplitude (kx = ky); a Gaussian plasma of peak
5e19 m^-3 (a third of the critical density at 110 GHz) and width lambda/4
sits at the centre, so the Drude current has an x part as large as its y
part.  The fine level covers the middle of the cavity: a rectangle (r = 2,
or r = 4 on a lambda/16 base mesh) or a union of blocks with a concave
corner.  No incident wave; the continuity step runs (the field is near the
breakdown field at its antinodes).

Every case starts both the GPU library and the oracle from the same Hz
sampled on each level's own cell centres (zero outside a union level).
"""
import numpy as np

from paper_2105_13276_amd import workloads as W

LAM = 299792458.0 / 110e9
H0 = 1.5e4          # A/m: E peak ~ 4 MV/m
N0 = 5e19


def config(kind, periods=10):
    """(cfg, extra union blocks or None) of the case."""
    common = dict(bc_x="pec", bc_y="pec", tfsf_i=0)
    if kind == "rect":
        cfg = W.make(64, 32, 32, "static", periods, block=8, static_ext=(16, 8, 48, 24),
                     **common)
        return cfg, None
    if kind == "r4":
        cfg = W.make(32, 16, 16, "static", periods, r=4, block=4, static_ext=(8, 4, 24, 12),
                     **common)
        return cfg, None
    if kind == "union":
        cfg = W.make(64, 32, 32, "static", periods, block=8, regrid_rule="union",
                     static_ext=(16, 8, 48, 16), **common)
        return cfg, [(2, 2), (3, 2)]       # an L: a concave corner at (32, 16)
    raise ValueError(kind)


def seeds(cfg):
    dx = LAM / cfg["cells_per_lambda"]
    centre = [(0.5 * cfg["nx"] * dx, 0.5 * cfg["ny"] * dx)]
    r = cfg["r"]
    sb = W.gaussian_seed(cfg["nx"], cfg["ny"], dx, centre, [N0], LAM / 4)
    sf = W.gaussian_seed(r * cfg["nx"], r * cfg["ny"], dx / r, centre, [N0], LAM / 4)
    return sb, sf


def level_cells(sim, cfg):
    """[rows][cols] True on the level-1 view's cells that belong to the level."""
    rows, cols = sim.dims("hz", 1)
    if cfg["regrid_rule"] != "union":
        return np.ones((rows, cols), bool)
    e, B, r = sim.patch(), cfg["block"], cfg["r"]
    blk = sim.blocks()[e[1] // B:e[3] // B, e[0] // B:e[2] // B].astype(bool)
    return np.kron(blk, np.ones((r * B, r * B), bool))


def start(sim, cfg, extra):
    """Add the union's extra blocks and load the cavity mode into Hz."""
    if extra:
        m = np.zeros((cfg["ny"] // cfg["block"], cfg["nx"] // cfg["block"]), np.uint8)
        for bx, by in extra:
            m[by, bx] = 1
        sim.add_blocks(m)
    dx = LAM / cfg["cells_per_lambda"]
    Lx, Ly = cfg["nx"] * dx, cfg["ny"] * dx
    r = cfg["r"]

    def hz(h, cols, rows, i0, j0):
        X, Y = np.meshgrid((i0 + np.arange(cols) + 0.5) * h, (j0 + np.arange(rows) + 0.5) * h)
        return H0 * np.cos(2 * np.pi * X / Lx) * np.cos(np.pi * Y / Ly)

    sim.set("hz", 0, hz(dx, cfg["nx"], cfg["ny"], 0, 0))
    e = sim.patch()
    rows, cols = sim.dims("hz", 1)
    sim.set("hz", 1, hz(dx / r, cols, rows, r * e[0], r * e[1]) * level_cells(sim, cfg))


def level_masks(sim, cfg):
    """Per level-1 field: True on the view entries that belong to the level
    (edges and nodes touching a level cell)."""
    act = level_cells(sim, cfg)
    R, C = act.shape
    pa = np.pad(act, 1)
    ex = pa[0:R + 1, 1:C + 1] | pa[1:R + 2, 1:C + 1]
    ey = pa[1:R + 1, 0:C + 1] | pa[1:R + 1, 1:C + 2]
    nd = pa[0:R + 1, 0:C + 1] | pa[0:R + 1, 1:C + 2] | pa[1:R + 2, 0:C + 1] | pa[1:R + 2, 1:C + 2]
    return {"hz": act, "ex": ex, "jx": ex, "ey": ey, "jy": ey, "n": nd, "erms2": nd}
