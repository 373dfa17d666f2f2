"""Python binding of the batch calls of ``include/lbm_solid.h``.

Argument marshalling only; the batch arena, tables, graphs and kernels live
in ``liblbm_solid.so``. PyTorch provides the device workspace and stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import lbm
from .lbm import LbmError, lbm_diagnostics


class lbm_plate_desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("dx", ctypes.c_double),
        ("rho0", ctypes.c_double), ("lam", ctypes.c_double), ("mu", ctypes.c_double),
        ("tau_over_dt", ctypes.c_double),
        ("body", ctypes.c_double * 2),
        ("bc_ymin", ctypes.c_int), ("bc_ymax", ctypes.c_int),
        ("val_ymin", ctypes.c_double * 2), ("val_ymax", ctypes.c_double * 2),
        ("rounding", ctypes.c_int), ("seed", ctypes.c_uint64),
    ]


_configured = False


def _lib():
    global _configured
    lib = lbm.load_library()
    if not _configured:
        vp, dp, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.lbm_batch_plate_bytes.restype = sz
        lib.lbm_batch_plate_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.lbm_batch_plate_tiles.restype = ctypes.c_int
        lib.lbm_batch_plate_tiles.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.lbm_batch_workspace_bytes.restype = sz
        lib.lbm_batch_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int, sz]
        lib.lbm_batch_create.restype = ctypes.c_int
        lib.lbm_batch_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         vp, sz, vp, ctypes.POINTER(vp)]
        lib.lbm_batch_add.restype = ctypes.c_int
        lib.lbm_batch_add.argtypes = [vp, ctypes.POINTER(lbm_plate_desc), dp, dp, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int)]
        lib.lbm_batch_step.restype = ctypes.c_int
        lib.lbm_batch_step.argtypes = [vp, ctypes.c_int64]
        lib.lbm_batch_query.restype = ctypes.c_int
        lib.lbm_batch_query.argtypes = [vp, ctypes.c_int, i64p, i64p, ctypes.POINTER(ctypes.c_int)]
        lib.lbm_batch_read.restype = ctypes.c_int
        lib.lbm_batch_read.argtypes = [vp, ctypes.c_int, dp, dp, dp, ctypes.POINTER(lbm_diagnostics)]
        lib.lbm_batch_retire.restype = ctypes.c_int
        lib.lbm_batch_retire.argtypes = [vp, ctypes.c_int]
        lib.lbm_batch_info.restype = ctypes.c_int
        lib.lbm_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(sz), ctypes.POINTER(sz)]
        lib.lbm_batch_destroy.restype = None
        lib.lbm_batch_destroy.argtypes = [vp]
        ip = ctypes.POINTER(ctypes.c_int)
        lib.lbm_batch_read_derived.restype = ctypes.c_int
        lib.lbm_batch_read_derived.argtypes = [vp, ctypes.c_int, dp, dp, dp]
        lib.lbm_batch_sample.restype = ctypes.c_int
        lib.lbm_batch_sample.argtypes = [vp, ctypes.c_int, ctypes.c_int, ip, ip, dp]
        lib.lbm_batch_set_steps_per_launch.restype = ctypes.c_int
        lib.lbm_batch_set_steps_per_launch.argtypes = [vp, ctypes.c_int]
        lib.lbm_batch_get_steps_per_launch.restype = ctypes.c_int
        lib.lbm_batch_get_steps_per_launch.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        lib.lbm_batch_last_error.restype = ctypes.c_char_p
        lib.lbm_batch_last_error.argtypes = [vp]
        _configured = True
    return lib


def _check(status: int, handle) -> None:
    if status != lbm.LBM_OK:
        msg = _lib().lbm_batch_last_error(handle)
        raise LbmError(status, msg.decode() if msg else "")


def _dptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---- C names -------------------------------------------------------------

def lbm_batch_plate_bytes(nx, ny, precision):
    return int(_lib().lbm_batch_plate_bytes(nx, ny, precision))


def lbm_batch_plate_tiles(nx, ny, precision, scheme):
    return int(_lib().lbm_batch_plate_tiles(nx, ny, precision, scheme))


def lbm_batch_workspace_bytes(max_plates, max_tiles, arena_bytes):
    return int(_lib().lbm_batch_workspace_bytes(max_plates, max_tiles, arena_bytes))


def lbm_batch_create(max_plates, max_tiles, precision, scheme, walled, ws_ptr, ws_bytes, stream_ptr):
    h = ctypes.c_void_p()
    _check(_lib().lbm_batch_create(max_plates, max_tiles, precision, scheme, int(walled), ws_ptr, ws_bytes,
                                   stream_ptr, ctypes.byref(h)), None)
    return h


def lbm_batch_add(h, desc: lbm_plate_desc, u0, v0, nsteps):
    """Returns the slot, or None when the batch has no room (LBM_ERR_NOMEM)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    slot = ctypes.c_int(-1)
    st = _lib().lbm_batch_add(h, ctypes.byref(desc), _dptr(u0), _dptr(v0), int(nsteps), ctypes.byref(slot))
    if st == lbm.LBM_ERR_NOMEM:
        return None
    _check(st, h)
    return slot.value


def lbm_batch_step(h, nsteps):
    _check(_lib().lbm_batch_step(h, int(nsteps)), h)


def lbm_batch_set_steps_per_launch(h, k):
    _check(_lib().lbm_batch_set_steps_per_launch(h, int(k)), h)


def lbm_batch_get_steps_per_launch(h):
    k = ctypes.c_int()
    _check(_lib().lbm_batch_get_steps_per_launch(h, ctypes.byref(k)), h)
    return k.value


def lbm_batch_query(h, slot):
    done, left, bad = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
    _check(_lib().lbm_batch_query(h, slot, ctypes.byref(done), ctypes.byref(left), ctypes.byref(bad)), h)
    return done.value, left.value, bool(bad.value)


def lbm_batch_read(h, slot, u=None, v=None, P=None, diag=None) -> int:
    st = _lib().lbm_batch_read(h, slot, _dptr(u), _dptr(v), _dptr(P),
                               ctypes.byref(diag) if diag is not None else None)
    if st not in (lbm.LBM_OK, lbm.LBM_ERR_UNSTABLE):
        _check(st, h)
    return st


def lbm_batch_read_derived(h, slot, sigma=None, E=None, W=None):
    _check(_lib().lbm_batch_read_derived(h, slot, _dptr(sigma), _dptr(E), _dptr(W)), h)


def lbm_batch_sample(h, slot, xs, ys) -> np.ndarray:
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    out = np.empty((len(xs), 17))
    ip = ctypes.POINTER(ctypes.c_int)
    _check(_lib().lbm_batch_sample(h, slot, len(xs), xs.ctypes.data_as(ip), ys.ctypes.data_as(ip), _dptr(out)), h)
    return out


def lbm_batch_retire(h, slot):
    _check(_lib().lbm_batch_retire(h, slot), h)


def lbm_batch_info(h):
    n, free, big = ctypes.c_int(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib().lbm_batch_info(h, ctypes.byref(n), ctypes.byref(free), ctypes.byref(big)), h)
    return n.value, free.value, big.value


def lbm_batch_destroy(h):
    _lib().lbm_batch_destroy(h)


# ---- convenience wrapper -------------------------------------------------

@dataclass
class PlateSpec:
    nx: int
    ny: int
    dx: float = 1.0
    rho0: float = 1.0
    lam: float = 0.1
    mu: float = 0.05
    tau_over_dt: float = 0.8
    body: tuple = (0.0, 0.0)
    bc_ymin: int = lbm.LBM_BC_PERIODIC
    bc_ymax: int = lbm.LBM_BC_PERIODIC
    val_ymin: tuple = (0.0, 0.0)
    val_ymax: tuple = (0.0, 0.0)
    rounding: str = "nearest"
    seed: int = 0

    def c(self) -> lbm_plate_desc:
        d = lbm_plate_desc()
        d.nx, d.ny, d.dx = self.nx, self.ny, self.dx
        d.rho0, d.lam, d.mu, d.tau_over_dt = self.rho0, self.lam, self.mu, self.tau_over_dt
        d.body[0], d.body[1] = self.body
        d.bc_ymin, d.bc_ymax = self.bc_ymin, self.bc_ymax
        d.val_ymin[0], d.val_ymin[1] = self.val_ymin
        d.val_ymax[0], d.val_ymax[1] = self.val_ymax
        d.rounding = lbm.ROUNDINGS.get(self.rounding, self.rounding)
        d.seed = int(self.seed) & ((1 << 64) - 1)
        return d


class Batch:
    """A batch of plates on one GPU; the workspace is a torch uint8 tensor."""

    def __init__(self, max_plates: int, arena_bytes: int, precision: str = "fp16", scheme: str = "pc",
                 walled: bool = False, max_tiles: int = 1 << 18, device: str = "cuda:0", stream=None):
        import torch

        self.precision = lbm.PRECISIONS[precision]
        self.scheme = lbm.SCHEMES[scheme]
        nbytes = lbm_batch_workspace_bytes(max_plates, max_tiles, arena_bytes)
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = lbm_batch_create(max_plates, max_tiles, self.precision, self.scheme, walled,
                                  ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream))
        self.arena_bytes = arena_bytes
        self.max_tiles = max_tiles
        self.specs = {}

    def close(self):
        if getattr(self, "h", None) is not None:
            lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def plate_bytes(self, nx, ny):
        return lbm_batch_plate_bytes(nx, ny, self.precision)

    @staticmethod
    def plate_bytes_for(nx, ny, precision: str):
        return lbm_batch_plate_bytes(nx, ny, lbm.PRECISIONS[precision])

    def fits_empty(self, nx, ny) -> bool:
        """Whether a plate of nx x ny sites fits the batch when no other plate
        is resident (its arena bytes and tile-table entries)."""
        return (lbm_batch_plate_bytes(nx, ny, self.precision) <= self.arena_bytes
                and lbm_batch_plate_tiles(nx, ny, self.precision, self.scheme) <= self.max_tiles)

    def add(self, spec: PlateSpec, u0, v0, nsteps: int):
        for name, a in (("u0", u0), ("v0", v0)):
            if np.shape(a) != (2, spec.ny, spec.nx):
                raise ValueError(f"{name} of shape {np.shape(a)}; expected (2, {spec.ny}, {spec.nx})")
        slot = lbm_batch_add(self.h, spec.c(), u0, v0, nsteps)
        if slot is not None:
            self.specs[slot] = spec
        return slot

    def step(self, nsteps: int):
        lbm_batch_step(self.h, nsteps)

    def synchronize(self):
        """Wait for the work enqueued on the batch's stream."""
        self.stream.synchronize()

    def query(self, slot):
        return lbm_batch_query(self.h, slot)

    def set_steps_per_launch(self, k: int):
        lbm_batch_set_steps_per_launch(self.h, k)

    def steps_per_launch(self) -> int:
        return lbm_batch_get_steps_per_launch(self.h)

    def read(self, slot, want_fields: bool = True):
        sp = self.specs[slot]
        ny, nx = sp.ny, sp.nx
        u = np.empty((2, ny, nx)) if want_fields else None
        v = np.empty((2, ny, nx)) if want_fields else None
        P = np.empty((2, 2, ny, nx)) if want_fields else None
        d = lbm_diagnostics()
        st = lbm_batch_read(self.h, slot, u, v, P, d)
        diag = lbm.Diagnostics(np.array(d.momentum[:]), d.mass_moment, d.energy, d.min_J, d.max_strain,
                               bool(d.unstable), int(d.steps))
        return u, v, P, diag, st

    def read_derived(self, slot):
        sp = self.specs[slot]
        sig, E, W = np.empty((2, 2, sp.ny, sp.nx)), np.empty((2, 2, sp.ny, sp.nx)), np.empty((sp.ny, sp.nx))
        lbm_batch_read_derived(self.h, slot, sig, E, W)
        return sig, E, W

    def sample(self, slot, xs, ys):
        return lbm_batch_sample(self.h, slot, xs, ys)

    def retire(self, slot):
        lbm_batch_retire(self.h, slot)
        self.specs.pop(slot, None)

    def info(self):
        return lbm_batch_info(self.h)
