"""Pins of the union-of-blocks fine level: the growth test's flagged blocks
(Sec. III.A/B) refined as they are instead of their bounding box (Sec. III.D
grows one rectangle).  It must reduce to the rectangular patch when the
blocks form a rectangle, prolong exactly on linear fields (Eq. (5a)), let a
plane wave cross a non-convex fine region without visible reflection, stay
bounded in a lossless cavity, and follow the uniform fine mesh (Sec. IV.B:
1-2%) with two separated seeds."""
import numpy as np
import pytest

from paper_2105_13276_amd import workloads as W

LAM = 299792458.0 / 110e9
FIELDS = ("hz", "ex", "ey", "jx", "jy", "n", "acc", "ring")


def test_rectangle_of_blocks_is_the_patch(oracle_mod):
    """A rectangle of blocks gives exactly the rectangular patch's run."""
    dxc = LAM / 32
    over = dict(static_ext=(48, 16, 96, 48), erms_over_ebd=2.5)
    cr = W.make(128, 64, 32, "static", 1, **over)
    cu = W.make(128, 64, 32, "static", 1, regrid_rule="union", **over)
    sb, sf = W.seeds(cr, [(72.5 * dxc, 32 * dxc)], [1e17])
    a, b = oracle_mod.Sim(cr, sb, sf), oracle_mod.Sim(cu, sb, sf)
    assert a.patch() == b.patch() == (48, 16, 96, 48)
    assert b.blocks().sum() == 6
    spp = cr["steps_per_period"]
    a.step(12 * spp + 5)
    b.step(12 * spp + 5)
    assert b.get("n", 1).max() > 1.05e17          # the density evolved
    for lv in (0, 1):
        for f in FIELDS:
            assert np.array_equal(a.get(f, lv), b.get(f, lv)), (f, lv)


def test_growth_prolongs_linear_fields_exactly(oracle_mod):
    """Entities new to the level take Eq. (5a) values: exact for linear
    coarse fields; entities the level had keep theirs."""
    cfg = W.make(64, 48, 32, "static", 1, block=8, regrid_rule="union",
                 static_ext=(24, 16, 40, 24), continuity_on=False)
    s = oracle_mod.Sim(cfg, np.zeros((49, 65)))
    f = lambda x, y: 3.0 + 0.25 * x - 0.5 * y            # x, y in coarse cells
    cpos = {"hz": (0.5, 0.5), "ex": (0.5, 0.0), "jx": (0.5, 0.0),
            "ey": (0.0, 0.5), "jy": (0.0, 0.5), "n": (0.0, 0.0),
            "acc": (0.0, 0.0)}
    for fld, (ox, oy) in cpos.items():
        r_, c_ = s.dims(fld, 0)
        X, Y = np.meshgrid(np.arange(c_) + ox, np.arange(r_) + oy)
        s.set(fld, 0, f(X, Y))
    X, Y = np.meshgrid(np.arange(65.0), np.arange(49.0))
    s.set("ring", 0, np.stack([(k + 1) * f(X, Y) for k in range(8)]))
    old = {fld: s.get(fld, 1).copy() for fld in FIELDS}
    m = np.zeros((6, 8), np.uint8)
    m[1:3, 5] = 1                          # right of the patch: an arm
    m[1, 3] = 1                            # below its left end
    s.add_blocks(m)
    assert s.patch() == (24, 8, 48, 24)
    blk = s.blocks()
    fpos = {"hz": (0.5, 0.5), "ex": (0.5, 0.0), "jx": (0.5, 0.0),
            "ey": (0.0, 0.5), "jy": (0.0, 0.5), "n": (0.0, 0.0),
            "acc": (0.0, 0.0)}
    P0, Q0 = 48, 16                        # bounding box origin, fine cells
    cell = lambda P, Q: (P >= 0) & (Q >= 0) & (P < 128) & (Q < 96) & \
        (blk[np.clip(Q, 0, 95) // 16, np.clip(P, 0, 127) // 16] == 1)
    was = lambda P, Q: (P >= 48) & (P < 80) & (Q >= 32) & (Q < 48)
    for fld, (ox, oy) in fpos.items():
        v = s.get(fld, 1)
        r_, c_ = v.shape
        P, Q = np.meshgrid(P0 + np.arange(c_), Q0 + np.arange(r_))
        if fld == "hz":
            has, had = cell(P, Q), was(P, Q)
        elif fld in ("ex", "jx"):
            has = cell(P, Q) | cell(P, Q - 1)
            had = was(P, Q) | was(P, Q - 1)
        elif fld in ("ey", "jy"):
            has = cell(P, Q) | cell(P - 1, Q)
            had = was(P, Q) | was(P - 1, Q)
        else:
            has = cell(P, Q) | cell(P - 1, Q) | cell(P, Q - 1) | cell(P - 1, Q - 1)
            had = was(P, Q) | was(P - 1, Q) | was(P, Q - 1) | was(P - 1, Q - 1)
        # the old patch sits at fine (48..80, 32..48): offset in the new box
        ov = np.zeros_like(v)
        o = old[fld]
        ov[16:16 + o.shape[0], 0:o.shape[1]] = o
        want = f((P + ox) / 2.0, (Q + oy) / 2.0)
        if fld == "hz":
            want = 1.25 * want             # Hz^{n-1/2} = 0: frac 5/4 in time
        new = has & ~had
        assert new.sum() > 0
        np.testing.assert_allclose(v[new], want[new], rtol=1e-13, atol=1e-13)
        assert np.array_equal(v[had], ov[had]), fld
        assert not v[~has].any(), fld
    ring = s.get("ring", 1)
    P, Q = np.meshgrid(P0 + np.arange(ring.shape[2]), Q0 + np.arange(ring.shape[1]))
    has = cell(P, Q) | cell(P - 1, Q) | cell(P, Q - 1) | cell(P - 1, Q - 1)
    had = was(P, Q) | was(P - 1, Q) | was(P, Q - 1) | was(P - 1, Q - 1)
    for k in range(8):
        want = (k + 1) * f(P / 2.0, Q / 2.0)
        np.testing.assert_allclose(ring[k][has & ~had], want[has & ~had], rtol=1e-13)
    with pytest.raises(RuntimeError):      # inside the outer margin
        bad = np.zeros((6, 8), np.uint8)
        bad[0, 4] = 1
        s.add_blocks(bad)


def test_vacuum_wave_crosses_an_l_shape(oracle_mod):
    """Plane wave through a non-convex fine region (an L with a concave
    corner): no visible reflection into the scattered-field strip, fine
    amplitude that of the incident wave."""
    cfg = W.make(128, 64, 32, "static", 1, regrid_rule="union", block=8,
                 static_ext=(48, 16, 96, 32), continuity_on=False)
    E0 = oracle_mod.derived(cfg)["E0"]
    s = oracle_mod.Sim(cfg, np.zeros((65, 129)))
    m = np.zeros((8, 16), np.uint8)
    m[4:6, 6:8] = 1                        # the L's vertical arm
    s.add_blocks(m)
    assert s.blocks().sum() == 16
    spp = cfg["steps_per_period"]
    peaks = []
    for per in range(1, 41):
        s.step(spp)
        if per >= 10 and per % 5 == 0:
            ey = s.get("ey")
            assert np.abs(ey[:, :cfg["tfsf_i"]]).max() < 0.01 * E0
            peaks.append(np.abs(s.get("ey", 1)).max() / E0)
    peaks = np.array(peaks)
    assert peaks.max() < 1.01 and np.ptp(peaks) < 2e-3


def test_pec_cavity_with_two_regions_bounded(oracle_mod):
    """Lossless cavity holding two separate fine regions: the interfaces add
    no energy over 4000 coarse steps; the two regions touch at one corner
    (a node with two active cells diagonally opposite)."""
    cfg = W.make(64, 64, 32, "static", 1, bc_x="pec", bc_y="pec", tfsf_i=0,
                 block=8, regrid_rule="union", static_ext=(16, 16, 32, 32),
                 continuity_on=False)
    s = oracle_mod.Sim(cfg, np.zeros((65, 65)))
    m = np.zeros((8, 8), np.uint8)
    m[4:6, 4:7] = 1
    s.add_blocks(m)
    mode = lambda x, y: 1e6 * np.sin(np.pi * x) * np.sin(np.pi * y)
    I, J = np.meshgrid(np.arange(65.0), np.arange(64) + 0.5)
    s.set("ey", 0, mode(I / 64, J / 64))

    def energy():
        return ((s.get("ex") ** 2).sum() + (s.get("ey") ** 2).sum()
                + ((376.73 * s.get("hz")) ** 2).sum())

    e0 = energy()
    for _ in range(20):
        s.step(200)
        assert energy() < 1.5 * e0
    assert np.isfinite(s.get("hz", 1)).all()


def _two_seed_case(rule):
    dxc = LAM / 32
    cfgd = W.make(128, 64, 32, "dynamic", 1, block=8, erms_over_ebd=2.5,
                  regrid_rule=rule)
    cfgu = W.make(256, 128, 64, "uniform", 1, erms_over_ebd=2.5)
    cen, pk = [(44.5 * dxc, 20 * dxc), (92.5 * dxc, 44 * dxc)], [1e17, 1e17]
    return cfgd, cfgu, W.seeds(cfgd, cen, pk), W.seeds(cfgu, cen, pk)[0]


@pytest.mark.slow
def test_union_matches_uniform_fine_with_two_seeds(oracle_mod):
    """Two seeds far apart, 80 periods with growth: density within 3% and
    E_rms^2 within 1% of the uniform fine mesh on the union's nodes.  (The
    bounding-box patch of the same run, 6x the fine area, gives 2.1% on the
    density: the union leaves more of the field around the plasma to the
    coarse mesh.)"""
    cfgd, cfgu, (sb, sf), su = _two_seed_case("union")
    d = oracle_mod.Sim(cfgd, sb, sf)
    u = oracle_mod.Sim(cfgu, su)
    b0 = d.blocks().copy()
    spp = cfgd["steps_per_period"]
    d.step(80 * spp)
    u.step(160 * spp)
    blk = d.blocks()
    assert (blk >= b0).all() and blk.sum() > b0.sum()     # it grew, only grew
    # two separate regions: the union is well below its bounding box
    e = d.patch()
    assert blk.sum() < 0.6 * ((e[2] - e[0]) // 8) * ((e[3] - e[1]) // 8)
    # compare on the fine nodes inside active blocks (bounding-box view)
    P0, Q0, P1, Q1 = (2 * v for v in e)
    nf, nu = d.get("n", 1), u.get("n")[Q0:Q1 + 1, P0:P1 + 1]
    ef, eu = d.get("erms2", 1), u.get("erms2")[Q0:Q1 + 1, P0:P1 + 1]
    cb = np.kron(blk, np.ones((16, 16), np.uint8))[Q0:Q1, P0:P1].astype(bool)
    node = np.zeros(nf.shape, bool)
    node[:-1, :-1] |= cb
    node[1:, :-1] |= cb
    node[:-1, 1:] |= cb
    node[1:, 1:] |= cb
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert nu.max() > 5e17
    assert rel(nf[node], nu[node]) < 0.03 and rel(ef[node], eu[node]) < 0.01
    assert abs(nf[node].sum() / nu[node].sum() - 1) < 0.03
    assert not nf[~node].any()            # nothing outside the union
    # injection: coarse nodes with all four cells active carry the fine n
    cact = np.kron(blk, np.ones((8, 8), np.uint8)).astype(bool)
    inner = np.zeros((65, 129), bool)
    inner[1:-1, 1:-1] = cact[:-1, :-1] & cact[1:, :-1] & cact[:-1, 1:] & cact[1:, 1:]
    nc = d.get("n", 0)
    fine_at = np.zeros_like(nc)
    fine_at[e[1]:e[3] + 1, e[0]:e[2] + 1] = nf[::2, ::2]
    assert inner.sum() > 0 and np.array_equal(nc[inner], fine_at[inner])


def test_union_blocks_are_the_flagged_blocks(oracle_mod):
    """At t = 0 the active blocks are the flagged blocks inside the margins
    (brute force over the seed's nodes, as the growth test's definition)."""
    cfgd, _, (sb, sf), _ = _two_seed_case("union")
    d = oracle_mod.Sim(cfgd, sb, sf)
    nc = oracle_mod.derived(cfgd)["n_c"]
    thr, flo = cfgd["n_thr_over_nc"] * nc, cfgd["n_floor_over_nc"] * nc
    n = sb.astype(np.float32).astype(np.float64)
    want = np.zeros((8, 16), np.uint8)
    for j in range(65):
        for i in range(129):
            v = n[j, i]
            flag = v > thr
            if not flag and v > flo and 0 < i < 128 and 0 < j < 64:
                gx, gy = (n[j, i + 1] - n[j, i - 1]) / 2, (n[j + 1, i] - n[j - 1, i]) / 2
                flag = gx * gx + gy * gy > cfgd["grad_thr"] ** 2 * v * v
            if flag:
                want[min(j // 8, 7), min(i // 8, 15)] = 1
    want[0, :] = want[-1, :] = 0
    want[:, :2] = 0
    want[:, -1] = 0
    got = d.blocks()
    assert got.sum() >= 2 and np.array_equal(got, want)
