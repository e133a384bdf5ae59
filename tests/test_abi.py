"""The C-ABI library loads, exports every entry point include/dmr.h declares,
and its host-side parameter checks behave (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2105_13276_amd import binding as B
from paper_2105_13276_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dmr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dmr_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 15
    lib = C.CDLL(B.LIB)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.SYMBOLS) == names


def test_params_struct_layout():
    # the binding's struct must match the C struct: a wrong size is refused
    cfg = W.config0()
    p = B.make_params(cfg)
    n = C.c_size_t()
    assert B.lib().dmr_workspace_bytes(C.byref(p), C.byref(n)) == 0
    assert n.value > 0
    p.struct_size += 8
    assert B.lib().dmr_workspace_bytes(C.byref(p), C.byref(n)) == -1


@pytest.mark.parametrize("over", [
    dict(courant=0.75),                 # beyond the 2-D Yee limit 1/sqrt(2)
    dict(courant=0.3),                  # N/S not a multiple of 8
    dict(nx=2),
    dict(tfsf_i=10_000),
    dict(bc_x="periodic"),
])
def test_invalid_params_rejected(over):
    cfg = dict(W.config0())
    cfg.update(over)
    if cfg["bc_x"] not in B.BC:
        cfg["bc_x"] = "mur"
        p = B.make_params(cfg)
        p.bc_x = 2
    else:
        p = B.make_params(cfg)
    n = C.c_size_t()
    assert B.lib().dmr_workspace_bytes(C.byref(p), C.byref(n)) == -1


@pytest.mark.parametrize("over", [
    dict(block=12),                     # does not divide 512
    dict(r=3),
    dict(regrid_every=100),             # not a multiple of 8 steps
])
def test_invalid_refinement_rejected(over):
    cfg = dict(W.config1_dmr())
    cfg.update(over)
    with pytest.raises(B.DmrError):
        B.workspace_bytes(cfg)


def test_workspace_covers_full_domain_patch():
    cfg = W.config1_dmr()
    nb = B.workspace_bytes(cfg)
    # 21 planes per level, fine level r^2 larger: > 21*4*(1+4)*nodes bytes
    nodes = (cfg["nx"] + 1) * (cfg["ny"] + 1)
    assert nb >= 21 * 4 * 5 * nodes


def test_adjoint_tape_sizing():
    cfg = W.config4(steps=2000)
    p = B.make_params(cfg)
    n = C.c_size_t()
    assert B.lib().dmr_adjoint_tape_bytes(C.byref(p), 2000, 45, C.byref(n)) == 0
    big = n.value
    assert B.lib().dmr_adjoint_tape_bytes(C.byref(p), 2000, 200, C.byref(n)) == 0
    assert n.value != big
    assert B.lib().dmr_adjoint_tape_bytes(C.byref(p), 0, 45, C.byref(n)) == -1
    assert B.lib().dmr_adjoint_tape_bytes(C.byref(p), 2000, 0, C.byref(n)) == -1


@pytest.mark.parametrize("over", [
    dict(r=4, block=8),                 # the union-of-blocks level is r = 2
    dict(block=12),                     # divides 384 x 192, not a power of two
    dict(block=4),                      # below 8
    dict(mode="static", static_ext=(40, 64, 96, 128)),  # not whole blocks
])
def test_invalid_union_rejected(over):
    cfg = dict(W.make(384, 192, 32, "dynamic", 1, regrid_rule="union"))
    B.workspace_bytes(cfg)              # valid as it stands
    cfg.update(over)
    with pytest.raises(B.DmrError):
        B.workspace_bytes(cfg)


def test_union_workspace_holds_maps_and_tiles():
    """The union-of-blocks level needs two block maps, two tile lists (64x4
    tiles over the fine domain) and the per-tile Eq. (5b) hand-off on top of
    the rectangle's workspace."""
    cfg = W.make(512, 256, 32, "dynamic", 1)
    rect = B.workspace_bytes(cfg)
    uni = B.workspace_bytes(dict(cfg, regrid_rule="union"))
    tiles = ((1024 + 1 + 63) // 64) * ((512 + 1 + 3) // 4)
    assert uni - rect >= 2 * (32 * 16) + 2 * 8 * tiles + 4 * 198 * tiles


@pytest.mark.parametrize("over", [
    dict(),
    dict(p_torr=200.0, freq_hz=60e9, erms_over_ebd=2.5, te_ev=1.5),
    dict(source_model="townsend", beta_rec=1.0),
    dict(cells_per_lambda=16, courant=0.5),
])
def test_library_derives_the_oracles_constants(oracle_mod, over):
    """The library's own host-side derivation of the run's scalars (collision
    rate, critical density, breakdown field, diffusivities, Drude decay and
    drive, incident wavenumber) against the oracle's, with no device call:
    FP64 values to rounding, those the kernels take in float32 to float32."""
    cfg = dict(W.config1_dmr())
    cfg.update(over)
    g, o = B.derived(cfg), oracle_mod.derived(cfg)
    assert list(g) == list(o)
    f32 = {"a", "b", "nu_att"}
    for k in g:
        tol = 2e-7 if k in f32 else 1e-13
        assert abs(g[k] - o[k]) <= tol * abs(o[k]), (k, g[k], o[k])
    p = B.make_params(cfg)
    p.courant = 0.75
    out = (C.c_double * 17)()
    assert B.lib().dmr_derived(C.byref(p), out, 17) == -1
