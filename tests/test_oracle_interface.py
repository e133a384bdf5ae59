"""Pins of the oracle's coarse/fine transfers (Sec. III.C, Eq. (5b), Fig. 5):
each operator reproduces fields that are linear in space (and, for Eq. (5b),
in time) exactly, on exactly the entities the method assigns to it.

* Eq. (5b): the tangential fine E on the coarse/fine boundary is linear
  along the boundary line between the two nearest coarse edges (a fine edge
  sits 1/(2r) of a coarse cell off its coarse neighbours, Fig. 5(c)) and
  linear in time between the old and new coarse field at frac = m/r.  On a
  field linear in x, y and t this gives the field's own value at the fine
  edge's position and time.
* fine -> coarse: edge means of the r fine edges that make up a coarse edge
  (E, J) and the mean over the r x r fine cells and the two fine half levels
  that bracket coarse n+1/2 (Hz) give, on linear fields, the value at the
  coarse entity's position (and the mid time).
* density: the fine boundary nodes take the coarse density by Eq. (5a)
  weights (copy at coincident nodes, mean at mid nodes; exact for bilinear
  fields), the coarse nodes inside the level take the fine density
  (injection).

The boundary / interior sets are derived here from cell activity alone (an
edge is a boundary edge when exactly one of its two cells is refined; a
coarse entity is restricted when all of its cells are), independently of
how the oracle enumerates them.  Cases: a rectangle at r = 2 and r = 4, and
a union of blocks with a concave corner and two blocks touching at a corner.
"""
import numpy as np
import pytest

from paper_2105_13276_amd import workloads as W

RNG = np.random.default_rng(51)


def _cases():
    rect2 = W.make(64, 32, 32, "static", 1, static_ext=(24, 8, 48, 24), continuity_on=False)
    rect4 = W.make(64, 32, 16, "static", 1, r=4, block=8, static_ext=(24, 8, 48, 24),
                   continuity_on=False)
    uni = W.make(96, 48, 32, "static", 1, block=8, regrid_rule="union",
                 static_ext=(16, 8, 56, 16), continuity_on=False)
    return {"rect_r2": (rect2, None), "rect_r4": (rect4, None),
            "union_L": (uni, [(2, 2), (3, 2), (2, 3), (7, 2), (5, 3), (6, 3), (5, 4), (6, 4)])}


def _sim(oracle_mod, name):
    cfg, extra = _cases()[name]
    s = oracle_mod.Sim(cfg, np.zeros((cfg["ny"] + 1, cfg["nx"] + 1)))
    if extra:
        m = np.zeros((cfg["ny"] // cfg["block"], cfg["nx"] // cfg["block"]), np.uint8)
        for bx, by in extra:
            m[by, bx] = 1
        s.add_blocks(m)
    return cfg, s


def _coarse_active(cfg, s):
    """[ny][nx] refined coarse cells."""
    nx, ny, B = cfg["nx"], cfg["ny"], cfg["block"]
    act = np.zeros((ny, nx), bool)
    if cfg["regrid_rule"] == "union":
        blk = s.blocks().astype(bool)
        act = np.kron(blk, np.ones((B, B), bool))
    else:
        I0, J0, I1, J1 = s.patch()
        act[J0:J1, I0:I1] = True
    return act


def _lin(c, x, y, t=0.0):
    return 1e6 * (c[0] + c[1] * x / 40.0 + c[2] * y / 40.0 + c[3] * t)


def _coarse_pos(cfg, field):
    """Positions in coarse-cell units of a base-level field's entries."""
    nx, ny = cfg["nx"], cfg["ny"]
    field = {"jx": "ex", "jy": "ey"}.get(field, field)
    if field == "ex":
        return np.meshgrid(np.arange(nx) + 0.5, np.arange(ny + 1.0))
    if field == "ey":
        return np.meshgrid(np.arange(nx + 1.0), np.arange(ny) + 0.5)
    if field == "hz":
        return np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    return np.meshgrid(np.arange(nx + 1.0), np.arange(ny + 1.0))


def _fine_pos(cfg, s, field):
    """Positions in coarse-cell units of the level-1 view's entries, and the
    view's global fine indices (P, Q) of each entry."""
    r = cfg["r"]
    rows, cols = s.dims(field, 1)
    field = {"jx": "ex", "jy": "ey"}.get(field, field)
    P0, Q0 = r * s.patch()[0], r * s.patch()[1]
    P, Q = np.meshgrid(P0 + np.arange(cols), Q0 + np.arange(rows))
    ox = 0.5 if field in ("ex", "hz") else 0.0
    oy = 0.5 if field in ("ey", "hz") else 0.0
    return (P + ox) / r, (Q + oy) / r, P, Q


def _fine_cell_active(cfg, act, P, Q):
    r = cfg["r"]
    ok = (P >= 0) & (Q >= 0) & (P < r * cfg["nx"]) & (Q < r * cfg["ny"])
    out = np.zeros(P.shape, bool)
    out[ok] = act[Q[ok] // r, P[ok] // r]
    return out


@pytest.mark.parametrize("name", ["rect_r2", "rect_r4", "union_L"])
def test_eq5b_exact_on_fields_linear_in_space_and_time(oracle_mod, name):
    cfg, s = _sim(oracle_mod, name)
    r = cfg["r"]
    act = _coarse_active(cfg, s)
    cx, cy = RNG.standard_normal(4), RNG.standard_normal(4)
    X, Y = _coarse_pos(cfg, "ex")
    old_ex, new_ex = _lin(cx, X, Y, 0.0), _lin(cx, X, Y, 1.0)
    X, Y = _coarse_pos(cfg, "ey")
    old_ey, new_ey = _lin(cy, X, Y, 0.0), _lin(cy, X, Y, 1.0)
    s.set("ex", 0, new_ex)
    s.set("ey", 0, new_ey)
    s.set_old_e(old_ex, old_ey)
    # the boundary edges: exactly one of the edge's two fine cells refined
    x, y, P, Q = _fine_pos(cfg, s, "ey")
    bnd_ey = _fine_cell_active(cfg, act, P - 1, Q) != _fine_cell_active(cfg, act, P, Q)
    xe, ye, P, Q = _fine_pos(cfg, s, "ex")
    bnd_ex = _fine_cell_active(cfg, act, P, Q - 1) != _fine_cell_active(cfg, act, P, Q)
    assert bnd_ey.sum() > 0 and bnd_ex.sum() > 0
    for m in range(1, r + 1):
        t = m / r
        ex_b, ey_b = s.cfb_fill(t)
        assert np.array_equal(~np.isnan(ey_b), bnd_ey), (name, m)
        assert np.array_equal(~np.isnan(ex_b), bnd_ex), (name, m)
        ref_ey, ref_ex = _lin(cy, x, y, t), _lin(cx, xe, ye, t)
        err = max(np.abs(ey_b[bnd_ey] - ref_ey[bnd_ey]).max(),
                  np.abs(ex_b[bnd_ex] - ref_ex[bnd_ex]).max())
        assert err < 1e-14 * 1e6 * 8, (name, m, err)
    # the level's own fields are untouched by the hook
    assert not np.isnan(s.get("ey", 1)).any()


@pytest.mark.parametrize("name", ["rect_r2", "rect_r4", "union_L"])
def test_fine_to_coarse_exact_on_linear_fields(oracle_mod, name):
    cfg, s = _sim(oracle_mod, name)
    act = _coarse_active(cfg, s)
    sentinel = 7.25e5
    coef = {f: RNG.standard_normal(4) for f in ("hz", "ex", "ey", "jx", "jy")}
    for f in coef:
        s.set(f, 0, np.full(s.dims(f, 0), sentinel))
        if f != "hz":
            x, y, _, _ = _fine_pos(cfg, s, f)
            s.set(f, 1, _lin(coef[f], x, y))
    x, y, _, _ = _fine_pos(cfg, s, "hz")
    # the two half levels bracket coarse n+1/2 symmetrically (for r = 2 at
    # n+1/4 and n+3/4, for r = 4 at n+3/8 and n+5/8); here t = 0.25, 0.75
    s.set_hz_halves(_lin(coef["hz"], x, y, 0.25), _lin(coef["hz"], x, y, 0.75))
    s.restrict()
    pad = np.pad(act, 1)           # pad[J+1, I+1] = act[J, I]; False outside
    ny, nx = act.shape
    sets = {
        "hz": act,
        # coarse x-edge (I, J) between cells (I, J-1) and (I, J)
        "ex": pad[0:ny + 1, 1:nx + 1] & pad[1:ny + 2, 1:nx + 1],
        # coarse y-edge (I, J) between cells (I-1, J) and (I, J)
        "ey": pad[1:ny + 1, 0:nx + 1] & pad[1:ny + 1, 1:nx + 2],
    }
    sets["jx"], sets["jy"] = sets["ex"], sets["ey"]
    for f, c in coef.items():
        got = s.get(f, 0)
        X, Y = _coarse_pos(cfg, f)
        ref = _lin(c, X, Y, 0.5 if f == "hz" else 0.0)
        inside = sets[f]
        assert inside.sum() > 0
        assert np.abs(got[inside] - ref[inside]).max() < 1e-14 * 1e6 * 8, (name, f)
        assert (got[~inside] == sentinel).all(), (name, f)


@pytest.mark.parametrize("name", ["rect_r2", "rect_r4", "union_L"])
def test_density_transfers_exact_on_bilinear_fields(oracle_mod, name):
    cfg, s = _sim(oracle_mod, name)
    r = cfg["r"]
    act = _coarse_active(cfg, s)
    cf = RNG.uniform(1.0, 2.0, 4)
    cg = RNG.uniform(1.0, 2.0, 3)
    f = lambda x, y: 1e17 * (cf[0] + cf[1] * x / 40 + cf[2] * y / 40 + cf[3] * x * y / 1600)
    g = lambda x, y: 1e17 * (cg[0] + cg[1] * x / 40 + cg[2] * y / 40)
    X, Y = _coarse_pos(cfg, "n")
    s.set("n", 0, f(X, Y))
    x, y, P, Q = _fine_pos(cfg, s, "n")
    s.set("n", 1, g(x, y))
    s.transfer_density()
    # fine nodes: in the level when a cell around them is refined, interior
    # when all four are
    around = [_fine_cell_active(cfg, act, P + a, Q + b) for a in (-1, 0) for b in (-1, 0)]
    in_level = np.logical_or.reduce(around)
    interior = np.logical_and.reduce(around)
    bnd = in_level & ~interior
    fine = s.get("n", 1)
    assert bnd.sum() > 0 and interior.sum() > 0
    assert np.abs(fine[bnd] - f(x, y)[bnd]).max() < 1e-14 * 1e17 * 8
    assert np.array_equal(fine[interior], g(x, y)[interior])
    # coarse nodes with all four cells refined take the fine density
    pad = np.pad(act, 1)
    ny, nx = act.shape
    inj = (pad[0:ny + 1, 0:nx + 1] & pad[0:ny + 1, 1:nx + 2] &
           pad[1:ny + 2, 0:nx + 1] & pad[1:ny + 2, 1:nx + 2])
    coarse = s.get("n", 0)
    assert inj.sum() > 0
    assert np.abs(coarse[inj] - g(X, Y)[inj]).max() < 1e-14 * 1e17 * 8
    assert np.array_equal(coarse[~inj], f(X, Y)[~inj])
