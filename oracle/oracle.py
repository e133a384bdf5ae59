"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this module.  The product path (``paper_2105_13276_amd``) never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dmr_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

BC = {"mur": 0, "pec": 1, "periodic": 2}
MODE = {"uniform": 0, "static": 1, "dynamic": 2}
DMODE = {"blend": 0, "const": 1}
FIELD = {"hz": 0, "ex": 1, "ey": 2, "jx": 3, "jy": 4, "n": 5, "acc": 6,
         "erms2": 7, "ring": 8}
DERIVED = ["omega", "lambda", "dx", "dt", "nu_m", "n_c", "eeff_fac", "E_bd",
           "E0", "D_e", "D_a", "n_amb", "a", "b", "ktilde", "nu_att",
           "steps_per_period"]


class OrcParams(C.Structure):
    _fields_ = [
        ("freq_hz", C.c_double), ("erms_over_ebd", C.c_double),
        ("p_torr", C.c_double), ("A_ion", C.c_double),
        ("beta_ion", C.c_double), ("ecr_over_p", C.c_double),
        ("te_ev", C.c_double), ("ti_ev", C.c_double),
        ("mu_i_760", C.c_double), ("L_amb", C.c_double),
        ("d_const", C.c_double), ("n_thr_over_nc", C.c_double),
        ("grad_thr", C.c_double), ("n_floor_over_nc", C.c_double),
        ("courant", C.c_double), ("fine_filter", C.c_double),
        ("nx", C.c_int32), ("ny", C.c_int32), ("cells_per_lambda", C.c_int32),
        ("r", C.c_int32), ("block", C.c_int32), ("regrid_every", C.c_int32),
        ("tfsf_i", C.c_int32), ("ramp_periods", C.c_int32),
        ("bc_x", C.c_int32), ("bc_y", C.c_int32), ("mode", C.c_int32),
        ("static_ext", C.c_int32 * 4), ("d_mode", C.c_int32),
        ("continuity_on", C.c_int32),
        ("regrid_rule", C.c_int32), ("m_lx", C.c_int32), ("m_ly", C.c_int32),
        ("m_ex", C.c_int32), ("m_ey", C.c_int32), ("n_line", C.c_double),
        ("source_model", C.c_int32), ("A_town", C.c_double), ("B_town", C.c_double),
        ("nu_att", C.c_double), ("beta_rec", C.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, FP64, no FMA contraction,
    OpenMP over loops of independent entities)."""
    if force or not os.path.exists(LIB) or \
            os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-fopenmp", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.POINTER
        L.orc_create.argtypes = [P(OrcParams), C.c_void_p, C.c_void_p,
                                 P(C.c_void_p)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_destroy.restype = None
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_regrid.argtypes = [C.c_void_p]
        L.orc_get_patch.argtypes = [C.c_void_p, P(C.c_int32)]
        L.orc_field_dims.argtypes = [C.c_void_p, C.c_int, C.c_int, P(C.c_int32)]
        L.orc_get_field.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        L.orc_set_field.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        L.orc_get_regrid.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, P(C.c_int32)]
        L.orc_time.argtypes = [C.c_void_p, P(C.c_double), P(C.c_int64)]
        L.orc_add_blocks.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_get_blocks.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_set_old_e.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_cfb_fill.argtypes = [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]
        L.orc_set_hz_halves.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_restrict.argtypes = [C.c_void_p]
        L.orc_transfer_density.argtypes = [C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.argtypes = []
        L.orc_derived.argtypes = [P(OrcParams), P(C.c_double), C.c_int]
        L.orc_nu_net.argtypes = [P(OrcParams), C.c_double]
        L.orc_nu_net.restype = C.c_double
        L.orc_r_ei.argtypes = [P(OrcParams)]
        L.orc_r_ei.restype = C.c_double
        L.orc_d_eff.argtypes = [P(OrcParams), C.c_double]
        L.orc_d_eff.restype = C.c_double
        L.orc_continuity_apply.argtypes = [
            P(OrcParams), C.c_int, C.c_int, C.c_double, C.c_double, C.c_int,
            C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def make_params(cfg: dict) -> OrcParams:
    p = OrcParams()
    for name, _ in OrcParams._fields_:
        if name in ("bc_x", "bc_y"):
            setattr(p, name, BC[cfg[name]])
        elif name == "mode":
            setattr(p, name, MODE[cfg["mode"]])
        elif name == "d_mode":
            setattr(p, name, DMODE[cfg["d_mode"]])
        elif name == "source_model":
            p.source_model = {"power": 0, "townsend": 1}[cfg.get("source_model", "power")]
        elif name == "regrid_rule":
            p.regrid_rule = {"blocks": 0, "lines": 1, "union": 2}[cfg.get("regrid_rule", "blocks")]
        elif name == "static_ext":
            for k, v in enumerate(cfg.get("static_ext", (0, 0, 0, 0))):
                p.static_ext[k] = int(v)
        elif name == "continuity_on":
            p.continuity_on = int(bool(cfg["continuity_on"]))
        else:
            setattr(p, name, cfg[name])
    return p


def set_threads(n: int) -> int:
    """OpenMP worker threads of the oracle (n <= 0: all processors); results
    do not depend on it.  Returns the count in use."""
    return lib().orc_set_threads(int(n))


def threads() -> int:
    return lib().orc_get_threads()


def derived(cfg: dict) -> dict:
    p = make_params(cfg)
    out = (C.c_double * len(DERIVED))()
    lib().orc_derived(C.byref(p), out, len(DERIVED))
    return dict(zip(DERIVED, list(out)))


def r_ei(cfg: dict) -> float:
    """Recombination coefficient of Eq. (4), m^3/s."""
    p = make_params(cfg)
    return lib().orc_r_ei(C.byref(p))


def nu_net(cfg: dict, erms2: float) -> float:
    p = make_params(cfg)
    return lib().orc_nu_net(C.byref(p), float(erms2))


def d_eff(cfg: dict, n: float) -> float:
    p = make_params(cfg)
    return lib().orc_d_eff(C.byref(p), float(n))


def continuity_apply(cfg: dict, n, erms2, dx, dtn, perx=False, pery=False):
    """One continuity step on node arrays [ny+1][nx+1]."""
    p = make_params(cfg)
    n = np.ascontiguousarray(n, np.float64)
    e = np.ascontiguousarray(np.broadcast_to(erms2, n.shape), np.float64)
    out = np.empty_like(n)
    ny, nx = n.shape[0] - 1, n.shape[1] - 1
    rc = lib().orc_continuity_apply(C.byref(p), nx, ny, float(dx), float(dtn),
                                    int(perx), int(pery), _ptr(n), _ptr(e),
                                    _ptr(out))
    if rc:
        raise RuntimeError("orc_continuity_apply failed: %d" % rc)
    return out


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Sim:
    """One oracle simulation (FP64)."""

    def __init__(self, cfg: dict, seed_base=None, seed_fine=None):
        self.cfg = dict(cfg)
        self._p = make_params(cfg)
        h = C.c_void_p()
        sb = None if seed_base is None else np.ascontiguousarray(seed_base, np.float64)
        sf = None if seed_fine is None else np.ascontiguousarray(seed_fine, np.float64)
        if sb is not None and sb.shape != (cfg["ny"] + 1, cfg["nx"] + 1):
            raise ValueError("seed_base shape %s" % (sb.shape,))
        rc = lib().orc_create(C.byref(self._p), _ptr(sb), _ptr(sf), C.byref(h))
        if rc:
            raise RuntimeError("orc_create failed: %d" % rc)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    __del__ = close

    def step(self, n: int):
        rc = lib().orc_step(self._h, int(n))
        if rc:
            raise RuntimeError("orc_step failed: %d" % rc)

    def regrid(self):
        rc = lib().orc_regrid(self._h)
        if rc:
            raise RuntimeError("orc_regrid failed: %d" % rc)

    def patch(self):
        e = (C.c_int32 * 4)()
        lib().orc_get_patch(self._h, e)
        return tuple(e)

    def dims(self, field: str, level: int = 0):
        d = (C.c_int32 * 2)()
        if lib().orc_field_dims(self._h, FIELD[field], level, d):
            raise ValueError("no such field/level")
        return (d[0], d[1])

    def get(self, field: str, level: int = 0) -> np.ndarray:
        r, c = self.dims(field, level)
        out = np.empty((r, c), np.float64)
        lib().orc_get_field(self._h, FIELD[field], level, _ptr(out))
        if field == "ring":
            out = out.reshape(8, r // 8, c)
        return out

    def set(self, field: str, level: int, arr):
        r, c = self.dims(field, level)
        a = np.ascontiguousarray(arr, np.float64).reshape(-1)
        if a.size != r * c:
            raise ValueError("size mismatch")
        if lib().orc_set_field(self._h, FIELD[field], level, _ptr(a)):
            raise RuntimeError("orc_set_field failed")

    def regrid_info(self):
        nbx = self.cfg["nx"] // self.cfg["block"]
        nby = self.cfg["ny"] // self.cfg["block"]
        flags = np.zeros((nby, nbx), np.uint8)
        scan = np.zeros(nbx * nby, np.int32)
        lst = np.zeros(nbx * nby, np.int32)
        cnt = C.c_int32()
        lib().orc_get_regrid(self._h, _ptr(flags), _ptr(scan), _ptr(lst),
                             C.byref(cnt))
        return flags, scan, lst[:cnt.value].copy(), cnt.value

    def blocks(self) -> np.ndarray:
        """Active blocks [NBy][NBx] of the union-of-blocks fine level."""
        nbx = self.cfg["nx"] // self.cfg["block"]
        nby = self.cfg["ny"] // self.cfg["block"]
        out = np.zeros((nby, nbx), np.uint8)
        if lib().orc_get_blocks(self._h, _ptr(out)):
            raise RuntimeError("orc_get_blocks failed")
        return out

    def add_blocks(self, mask):
        m = np.ascontiguousarray(mask, np.uint8)
        rc = lib().orc_add_blocks(self._h, _ptr(m))
        if rc:
            raise RuntimeError("orc_add_blocks failed: %d" % rc)

    def time(self):
        t = C.c_double()
        st = C.c_int64()
        lib().orc_time(self._h, C.byref(t), C.byref(st))
        return t.value, st.value

    # -- test hooks: the coarse/fine transfers of Sec. III.C on the current
    # layout (arrays in the field-call layout) --------------------------------
    def _arr(self, field, level, a):
        r, c = self.dims(field, level)
        a = np.ascontiguousarray(a, np.float64)
        if a.shape != (r, c):
            raise ValueError("%s level %d: shape %s, expected %s" % (field, level, a.shape, (r, c)))
        return a

    def set_old_e(self, ex, ey):
        """Coarse E^n that Eq. (5b) interpolates from (base-level EX, EY)."""
        ex, ey = self._arr("ex", 0, ex), self._arr("ey", 0, ey)
        if lib().orc_set_old_e(self._h, _ptr(ex), _ptr(ey)):
            raise RuntimeError("orc_set_old_e failed")

    def cfb_fill(self, frac):
        """Eq. (5b) values at time fraction frac on the fine level's boundary
        edges, NaN elsewhere: (EX, EY) of level 1."""
        ex = np.empty(self.dims("ex", 1))
        ey = np.empty(self.dims("ey", 1))
        if lib().orc_cfb_fill(self._h, float(frac), _ptr(ex), _ptr(ey)):
            raise RuntimeError("orc_cfb_fill failed")
        return ex, ey

    def set_hz_halves(self, lo, hi):
        """The two fine Hz half levels the fine -> coarse transfer averages."""
        lo, hi = self._arr("hz", 1, lo), self._arr("hz", 1, hi)
        if lib().orc_set_hz_halves(self._h, _ptr(lo), _ptr(hi)):
            raise RuntimeError("orc_set_hz_halves failed")

    def restrict(self):
        """Run the fine -> coarse transfer of the end of a base step."""
        if lib().orc_restrict(self._h):
            raise RuntimeError("orc_restrict failed")

    def transfer_density(self):
        """Run the density transfers of a sync point (no continuity step)."""
        if lib().orc_transfer_density(self._h):
            raise RuntimeError("orc_transfer_density failed")
