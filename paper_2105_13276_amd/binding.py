"""Thin ctypes binding of libdmr.so (include/dmr.h).

Argument marshalling only: every step of the update runs in the HIP kernels
of libdmr.so.  PyTorch provides the device workspace and the stream.  If the
library has not been built this module raises on use; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(PKG, "libdmr.so")

BC = {"mur": 0, "pec": 1}
MODE = {"uniform": 0, "static": 1, "dynamic": 2}
DMODE = {"blend": 0, "const": 1}
RULE = {"blocks": 0, "lines": 1, "union": 2}
SOURCE = {"power": 0, "townsend": 1}
FIELD = {"hz": 0, "ex": 1, "ey": 2, "jx": 3, "jy": 4, "n": 5, "acc": 6,
         "erms2": 7, "ring": 8}
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EUNSTABLE"}

SYMBOLS = ["dmr_workspace_bytes", "dmr_create", "dmr_destroy", "dmr_step",
           "dmr_regrid", "dmr_get_patch", "dmr_get_regrid", "dmr_field_dims",
           "dmr_read_field", "dmr_write_field", "dmr_time", "dmr_sync",
           "dmr_set_timing", "dmr_get_timing", "dmr_last_error",
           "dmr_batch_workspace_bytes", "dmr_batch_create", "dmr_batch_step",
           "dmr_batch_instance", "dmr_batch_sync", "dmr_batch_config",
           "dmr_batch_set_config", "dmr_batch_destroy", "dmr_batch_last_error",
           "dmr_adjoint_tape_bytes", "dmr_forward_record", "dmr_backward",
           "dmr_weighted_sum", "dmr_state_bytes", "dmr_save", "dmr_load",
           "dmr_get_blocks", "dmr_add_blocks", "dmr_derived",
           "dmr_weighted_sum_static", "dmr_adjoint_tape_bytes_rows"]

# the scalars dmr_derived returns, in its order
DERIVED = ["omega", "lambda", "dx", "dt", "nu_m", "n_c", "eeff_fac", "E_bd",
           "E0", "D_e", "D_a", "n_amb", "a", "b", "ktilde", "nu_att",
           "steps_per_period"]


class DmrParams(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("cells_per_lambda", C.c_int32), ("r", C.c_int32),
        ("block", C.c_int32), ("regrid_every", C.c_int32),
        ("tfsf_i", C.c_int32), ("ramp_periods", C.c_int32),
        ("bc_x", C.c_int32), ("bc_y", C.c_int32), ("mode", C.c_int32),
        ("static_ext", C.c_int32 * 4), ("d_mode", C.c_int32),
        ("continuity_on", C.c_int32), ("pad_", C.c_int32),
        ("freq_hz", C.c_double), ("erms_over_ebd", C.c_double),
        ("p_torr", C.c_double), ("A_ion", C.c_double),
        ("beta_ion", C.c_double), ("ecr_over_p", C.c_double),
        ("te_ev", C.c_double), ("ti_ev", C.c_double),
        ("mu_i_760", C.c_double), ("L_amb", C.c_double),
        ("d_const", C.c_double), ("n_thr_over_nc", C.c_double),
        ("grad_thr", C.c_double), ("n_floor_over_nc", C.c_double),
        ("courant", C.c_double), ("fine_filter", C.c_double),
        ("regrid_rule", C.c_int32), ("m_lx", C.c_int32), ("m_ly", C.c_int32),
        ("m_ex", C.c_int32), ("m_ey", C.c_int32), ("pad2_", C.c_int32),
        ("n_line", C.c_double), ("source_model", C.c_int32), ("pad3_", C.c_int32),
        ("A_town", C.c_double), ("B_town", C.c_double), ("nu_att", C.c_double),
        ("beta_rec", C.c_double),
    ]


class DmrError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libdmr.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(
                "libdmr.so is not built; run `python -m paper_2105_13276_amd.build` "
                "(or __graft_entry__.build()) first")
        # torch ships its own HIP runtime (same soname); load it first so that
        # libdmr.so binds to the runtime that owns the workspace and stream
        import torch  # noqa: F401
        L = C.CDLL(LIB)
        P, V = C.POINTER, C.c_void_p
        L.dmr_workspace_bytes.argtypes = [P(DmrParams), P(C.c_size_t)]
        L.dmr_derived.argtypes = [P(DmrParams), P(C.c_double), C.c_int]
        L.dmr_create.argtypes = [P(DmrParams), V, V, V, C.c_size_t, V, P(V)]
        L.dmr_destroy.argtypes = [V]
        L.dmr_destroy.restype = None
        L.dmr_step.argtypes = [V, C.c_int64]
        L.dmr_regrid.argtypes = [V]
        L.dmr_get_patch.argtypes = [V, P(C.c_int32)]
        L.dmr_get_regrid.argtypes = [V, V, V, V, P(C.c_int32)]
        L.dmr_field_dims.argtypes = [V, C.c_int, C.c_int, P(C.c_int32)]
        L.dmr_read_field.argtypes = [V, C.c_int, C.c_int, V, C.c_size_t, C.c_int]
        L.dmr_write_field.argtypes = [V, C.c_int, C.c_int, V, C.c_size_t, C.c_int]
        L.dmr_time.argtypes = [V, P(C.c_double), P(C.c_int64)]
        L.dmr_sync.argtypes = [V]
        L.dmr_set_timing.argtypes = [V, C.c_int]
        L.dmr_get_timing.argtypes = [V, P(C.c_double), P(C.c_int64)]
        L.dmr_last_error.argtypes = [V]
        L.dmr_last_error.restype = C.c_char_p
        L.dmr_batch_workspace_bytes.argtypes = [V, C.c_int, P(C.c_size_t)]
        L.dmr_batch_create.argtypes = [V, C.c_int, V, V, V, C.c_size_t, V, P(V)]
        L.dmr_batch_step.argtypes = [V, C.c_int64]
        L.dmr_batch_instance.argtypes = [V, C.c_int, P(V)]
        L.dmr_batch_sync.argtypes = [V]
        L.dmr_batch_config.argtypes = [V, P(C.c_int32)]
        L.dmr_batch_set_config.argtypes = [V, P(C.c_int32)]
        L.dmr_batch_destroy.argtypes = [V]
        L.dmr_batch_destroy.restype = None
        L.dmr_batch_last_error.argtypes = [V]
        L.dmr_batch_last_error.restype = C.c_char_p
        L.dmr_adjoint_tape_bytes.argtypes = [P(DmrParams), C.c_int64, C.c_int, P(C.c_size_t)]
        L.dmr_adjoint_tape_bytes_rows.argtypes = [P(DmrParams), C.c_int64, C.c_int, C.c_int32,
                                                  P(C.c_size_t)]
        L.dmr_forward_record.argtypes = [V, C.c_int64, C.c_int, V, C.c_size_t]
        L.dmr_backward.argtypes = [V, V, V, V, V, V, P(C.c_double)]
        L.dmr_weighted_sum.argtypes = [V, C.c_int, V, P(C.c_double)]
        L.dmr_weighted_sum_static.argtypes = [V, C.c_int, V, P(C.c_double)]
        L.dmr_state_bytes.argtypes = [V, P(C.c_size_t)]
        L.dmr_save.argtypes = [V, V, C.c_size_t, C.c_int]
        L.dmr_load.argtypes = [V, V, C.c_size_t, C.c_int]
        L.dmr_get_blocks.argtypes = [V, V]
        L.dmr_add_blocks.argtypes = [V, V]
        _lib = L
    return _lib


def make_params(cfg: dict) -> DmrParams:
    p = DmrParams()
    p.struct_size = C.sizeof(DmrParams)
    for name, _ in DmrParams._fields_:
        if name in ("struct_size", "pad_", "pad2_", "pad3_"):
            continue
        if name in ("bc_x", "bc_y"):
            setattr(p, name, BC[cfg[name]])
        elif name == "mode":
            p.mode = MODE[cfg["mode"]]
        elif name == "d_mode":
            p.d_mode = DMODE[cfg["d_mode"]]
        elif name == "regrid_rule":
            p.regrid_rule = RULE[cfg["regrid_rule"]]
        elif name == "source_model":
            p.source_model = SOURCE[cfg["source_model"]]
        elif name == "static_ext":
            for k, v in enumerate(cfg.get("static_ext", (0, 0, 0, 0))):
                p.static_ext[k] = int(v)
        elif name == "continuity_on":
            p.continuity_on = int(bool(cfg["continuity_on"]))
        else:
            setattr(p, name, cfg[name])
    return p


def derived(cfg: dict) -> dict:
    """The library's derived scalars for cfg (host only, no device call)."""
    p = make_params(cfg)
    out = (C.c_double * len(DERIVED))()
    rc = lib().dmr_derived(C.byref(p), out, len(DERIVED))
    if rc:
        raise DmrError("dmr_derived: %s" % ERRORS.get(rc, rc))
    return dict(zip(DERIVED, list(out)))


def adjoint_tape_bytes(cfg: dict, steps: int, ckpt_every: int, fine_rows: int = 0) -> int:
    """Bytes of the adjoint tape (dmr_adjoint_tape_bytes_rows)."""
    p = make_params(cfg)
    n = C.c_size_t()
    rc = lib().dmr_adjoint_tape_bytes_rows(C.byref(p), int(steps), int(ckpt_every),
                                           int(fine_rows), C.byref(n))
    if rc:
        raise DmrError("dmr_adjoint_tape_bytes_rows: %s" % ERRORS.get(rc, rc))
    return n.value


def workspace_bytes(cfg: dict) -> int:
    p = make_params(cfg)
    n = C.c_size_t()
    rc = lib().dmr_workspace_bytes(C.byref(p), C.byref(n))
    if rc:
        raise DmrError("dmr_workspace_bytes: %s" % ERRORS.get(rc, rc))
    return n.value


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _buffer(buf):
    """(on device, pointer, bytes) of a numpy array or a torch tensor."""
    if isinstance(buf, np.ndarray):
        return 0, buf.ctypes.data_as(C.c_void_p), buf.nbytes
    return (1 if buf.is_cuda else 0), C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()


class _Handle:
    """Methods shared by owned simulations and batch instances."""

    _h = None
    cfg: dict = {}
    device = None

    def _check(self, rc, what):
        if rc:
            msg = lib().dmr_last_error(self._h).decode()
            raise DmrError("%s: %s (%s)" % (what, ERRORS.get(rc, rc), msg))

    def sync(self):
        self._check(lib().dmr_sync(self._h), "dmr_sync")

    def patch(self):
        e = (C.c_int32 * 4)()
        self._check(lib().dmr_get_patch(self._h, e), "dmr_get_patch")
        return tuple(e)

    def blocks(self) -> np.ndarray:
        """Active blocks [NBy][NBx] of a union-of-blocks fine level."""
        out = np.zeros((self.cfg["ny"] // self.cfg["block"],
                        self.cfg["nx"] // self.cfg["block"]), np.uint8)
        self._check(lib().dmr_get_blocks(self._h, _ptr(out)), "dmr_get_blocks")
        return out

    def add_blocks(self, mask):
        m = np.ascontiguousarray(mask, np.uint8)
        if m.shape != (self.cfg["ny"] // self.cfg["block"], self.cfg["nx"] // self.cfg["block"]):
            raise ValueError("mask shape %s" % (m.shape,))
        self._check(lib().dmr_add_blocks(self._h, _ptr(m)), "dmr_add_blocks")

    def regrid_info(self):
        nbx = self.cfg["nx"] // self.cfg["block"]
        nby = self.cfg["ny"] // self.cfg["block"]
        flags = np.zeros((nby, nbx), np.uint8)
        scan = np.zeros(nbx * nby, np.int32)
        lst = np.zeros(nbx * nby, np.int32)
        cnt = C.c_int32()
        self._check(lib().dmr_get_regrid(self._h, _ptr(flags), _ptr(scan),
                                         _ptr(lst), C.byref(cnt)), "dmr_get_regrid")
        return flags, scan, lst[:cnt.value].copy(), cnt.value

    def dims(self, field: str, level: int = 0):
        d = (C.c_int32 * 2)()
        self._check(lib().dmr_field_dims(self._h, FIELD[field], level, d), "dmr_field_dims")
        return (d[0], d[1])

    def get(self, field: str, level: int = 0) -> np.ndarray:
        r, c = self.dims(field, level)
        out = np.empty((r, c), np.float32)
        self._check(lib().dmr_read_field(self._h, FIELD[field], level, _ptr(out),
                                         out.nbytes, 0), "dmr_read_field")
        if field == "ring":
            out = out.reshape(8, r // 8, c)
        return out

    def time(self):
        t = C.c_double()
        st = C.c_int64()
        self._check(lib().dmr_time(self._h, C.byref(t), C.byref(st)), "dmr_time")
        return t.value, st.value

    def state_bytes(self) -> int:
        n = C.c_size_t()
        self._check(lib().dmr_state_bytes(self._h, C.byref(n)), "dmr_state_bytes")
        return n.value

    def save(self, buf=None):
        """Checkpoint of the state: into `buf` (a host numpy uint8 array or a
        256-byte aligned CUDA uint8 tensor of state_bytes()) or a new host
        array, which is returned."""
        if buf is None:
            buf = np.empty(self.state_bytes(), np.uint8)
        dev, ptr, n = _buffer(buf)
        self._check(lib().dmr_save(self._h, ptr, n, dev), "dmr_save")
        return buf

    def load(self, buf):
        """Restore a state saved from a handle with the same parameters."""
        dev, ptr, n = _buffer(buf)
        self._check(lib().dmr_load(self._h, ptr, n, dev), "dmr_load")


class BatchInstance(_Handle):
    """Borrowed view of one instance of a Batch (reads only)."""

    def __init__(self, batch, k):
        h = C.c_void_p()
        rc = lib().dmr_batch_instance(batch._h, k, C.byref(h))
        if rc:
            raise DmrError("dmr_batch_instance: %s" % ERRORS.get(rc, rc))
        self._h = h
        self.cfg = batch.cfgs[k]
        self._batch = batch  # keeps the batch alive


class Batch:
    """Many independent simulations advanced in lockstep by batched launches
    (graph-replayed intervals, tuned launch shapes)."""

    def __init__(self, cfgs, seeds, device: str = "cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise DmrError("no HIP device available")
        self.cfgs = [dict(c) for c in cfgs]
        n = len(cfgs)
        self._params = (DmrParams * n)(*[make_params(c) for c in cfgs])
        nbytes = C.c_size_t()
        rc = lib().dmr_batch_workspace_bytes(self._params, n, C.byref(nbytes))
        if rc:
            raise DmrError("dmr_batch_workspace_bytes: %s" % ERRORS.get(rc, rc))
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        self._seed_arrays = []
        sb = (C.c_void_p * n)()
        sf = (C.c_void_p * n)()
        for k, (b, f) in enumerate(seeds):
            if b is not None:
                b = np.ascontiguousarray(b, np.float64)
                self._seed_arrays.append(b)
                sb[k] = b.ctypes.data
            if f is not None:
                f = np.ascontiguousarray(f, np.float64)
                self._seed_arrays.append(f)
                sf[k] = f.ctypes.data
        h = C.c_void_p()
        rc = lib().dmr_batch_create(self._params, n, sb, sf,
                                    C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc:
            raise DmrError("dmr_batch_create failed: %s" % ERRORS.get(rc, rc))
        self._h = h
        self.instances = [BatchInstance(self, k) for k in range(n)]

    def _check(self, rc, what):
        if rc:
            msg = lib().dmr_batch_last_error(self._h).decode()
            raise DmrError("%s: %s (%s)" % (what, ERRORS.get(rc, rc), msg))

    def step(self, n: int):
        self._check(lib().dmr_batch_step(self._h, int(n)), "dmr_batch_step")

    def sync(self):
        self._check(lib().dmr_batch_sync(self._h), "dmr_batch_sync")

    SCHEDULES = ("separate", "fused", "combined")

    def config(self):
        """(segment rows, load depth, fine tile rows, graph on, schedule)."""
        c = (C.c_int32 * 5)()
        self._check(lib().dmr_batch_config(self._h, c), "dmr_batch_config")
        return tuple(c[:4]) + (self.SCHEDULES[c[4]],)

    def set_config(self, seg, depth, ty, graph, schedule="separate"):
        c = (C.c_int32 * 5)(seg, depth, ty, int(graph), self.SCHEDULES.index(schedule))
        self._check(lib().dmr_batch_set_config(self._h, c), "dmr_batch_set_config")

    def close(self):
        if getattr(self, "_h", None):
            self.instances = []
            lib().dmr_batch_destroy(self._h)
            self._h = None

    __del__ = close


class Sim(_Handle):
    """One simulation on one GPU.  The workspace is a torch uint8 tensor and
    work is queued on torch's current stream of ``device``."""

    def __init__(self, cfg: dict, seed_base=None, seed_fine=None,
                 device: str = "cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise DmrError("no HIP device available")
        self.cfg = dict(cfg)
        self.device = torch.device(device)
        self._p = make_params(cfg)
        nbytes = workspace_bytes(cfg)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream or torch.cuda.current_stream(self.device)
        sb = None if seed_base is None else np.ascontiguousarray(seed_base, np.float64)
        sf = None if seed_fine is None else np.ascontiguousarray(seed_fine, np.float64)
        if sb is not None and sb.shape != (cfg["ny"] + 1, cfg["nx"] + 1):
            raise ValueError("seed_base shape %s" % (sb.shape,))
        if sf is not None and sf.shape != (cfg["r"] * cfg["ny"] + 1, cfg["r"] * cfg["nx"] + 1):
            raise ValueError("seed_fine shape %s" % (sf.shape,))
        h = C.c_void_p()
        rc = lib().dmr_create(C.byref(self._p), _ptr(sb), _ptr(sf),
                              C.c_void_p(self.workspace.data_ptr()), nbytes,
                              C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc:
            raise DmrError("dmr_create failed: %s" % ERRORS.get(rc, rc))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().dmr_destroy(self._h)
            self._h = None

    __del__ = close

    def step(self, n: int):
        self._check(lib().dmr_step(self._h, int(n)), "dmr_step")

    def regrid(self):
        self._check(lib().dmr_regrid(self._h), "dmr_regrid")

    def get_device(self, field: str, level: int = 0):
        import torch
        r, c = self.dims(field, level)
        out = torch.empty((r, c), dtype=torch.float32, device=self.device)
        self._check(lib().dmr_read_field(self._h, FIELD[field], level,
                                         C.c_void_p(out.data_ptr()),
                                         out.numel() * 4, 1), "dmr_read_field")
        return out

    def set(self, field: str, level: int, arr):
        r, c = self.dims(field, level)
        a = np.ascontiguousarray(arr, np.float32).reshape(-1)
        if a.size != r * c:
            raise ValueError("size mismatch")
        self._check(lib().dmr_write_field(self._h, FIELD[field], level, _ptr(a),
                                          a.nbytes, 0), "dmr_write_field")

    def set_timing(self, on: bool):
        self._check(lib().dmr_set_timing(self._h, int(on)), "dmr_set_timing")

    # ---- adjoint -----------------------------------------------------------
    def _dev_f32(self, a):
        import torch
        return torch.as_tensor(np.asarray(a, np.float32) if not torch.is_tensor(a) else a,
                               dtype=torch.float32, device=self.device).contiguous()

    def record(self, steps: int, ckpt_every: int = 45, fine_rows: int = 0):
        """Advance `steps` base steps from t = 0, recording for backward().
        fine_rows: the most fine node rows any patch of the run spans (the
        tape's fine slots hold only those); 0: all rows of the fine grid."""
        import torch
        n = C.c_size_t()
        rc = lib().dmr_adjoint_tape_bytes_rows(C.byref(self._p), int(steps), int(ckpt_every),
                                               int(fine_rows), C.byref(n))
        if rc:
            raise DmrError("dmr_adjoint_tape_bytes_rows: %s" % ERRORS.get(rc, rc))
        with torch.cuda.device(self.device):
            self.tape = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self._check(lib().dmr_forward_record(self._h, int(steps), int(ckpt_every),
                                             C.c_void_p(self.tape.data_ptr()), n.value),
                    "dmr_forward_record")

    def weighted_sum(self, w, level: int = 0) -> float:
        """sum of w * n over the nodes of a level (fine: full-domain grid)."""
        wd = self._dev_f32(w)
        out = C.c_double()
        self._check(lib().dmr_weighted_sum(self._h, level, C.c_void_p(wd.data_ptr()),
                                           C.byref(out)), "dmr_weighted_sum")
        return out.value

    def weighted_sum_static(self, w, level: int = 0) -> float:
        """weighted_sum through dmr_weighted_sum_static (no workspace scratch:
        a static device array of the library)."""
        wd = self._dev_f32(w)
        out = C.c_double()
        self._check(lib().dmr_weighted_sum_static(self._h, level, C.c_void_p(wd.data_ptr()),
                                                  C.byref(out)), "dmr_weighted_sum_static")
        return out.value

    def backward(self, w_coarse, w_fine=None):
        """Gradients of F = sum w_c n_c + sum w_f n_f at the recorded t_final:
        dict(seed=[ny+1][nx+1] device tensor, seed_fine=(full-domain fine
        grid or None), E0=dF/dE0, A=dF/dA, beta=dF/dbeta)."""
        import torch
        cfg = self.cfg
        wc = self._dev_f32(w_coarse)
        wf = None if w_fine is None else self._dev_f32(w_fine)
        g = torch.empty((cfg["ny"] + 1, cfg["nx"] + 1), dtype=torch.float32, device=self.device)
        gf = None
        if cfg["mode"] != "uniform":
            r = cfg["r"]
            gf = torch.empty((r * cfg["ny"] + 1, r * cfg["nx"] + 1), dtype=torch.float32,
                             device=self.device)
        out = (C.c_double * 3)()
        self._check(lib().dmr_backward(
            self._h, C.c_void_p(self.tape.data_ptr()), C.c_void_p(wc.data_ptr()),
            None if wf is None else C.c_void_p(wf.data_ptr()),
            C.c_void_p(g.data_ptr()), None if gf is None else C.c_void_p(gf.data_ptr()),
            out), "dmr_backward")
        return dict(seed=g, seed_fine=gf, E0=out[0], A=out[1], beta=out[2])

    def timing(self):
        ms = (C.c_double * 4)()
        n = (C.c_int64 * 4)()
        self._check(lib().dmr_get_timing(self._h, ms, n), "dmr_get_timing")
        return list(ms), list(n)
