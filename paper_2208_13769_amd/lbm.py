"""Python binding of the C ABI in ``include/lbm_solid.h``.

Argument marshalling only: every step of the method runs in the HIP library
``liblbm_solid.so``. PyTorch provides the device workspace and the stream.
The functions keep the C names (``lbm_create``, ``lbm_step``, ...); the
``Solver`` class bundles them for one plate.

Loading fails loudly if the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_solid.so")

LBM_OK, LBM_ERR_ARG, LBM_ERR_NOMEM, LBM_ERR_HIP, LBM_ERR_STATE, LBM_ERR_UNSTABLE, LBM_ERR_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
LBM_FP64, LBM_FP32, LBM_FP16_STORE, LBM_BF16_STORE, LBM_FP32_U64 = 0, 1, 2, 3, 4
LBM_SCHEME_PC, LBM_SCHEME_EXPLICIT, LBM_SCHEME_EXTRAP = 0, 1, 2
LBM_EDGE_XMIN, LBM_EDGE_XMAX, LBM_EDGE_YMIN, LBM_EDGE_YMAX = 0, 1, 2, 3
LBM_BC_PERIODIC, LBM_BC_DIRICHLET_J, LBM_BC_NEUMANN_T = 0, 1, 2
LBM_ROUND_NEAREST, LBM_ROUND_STOCHASTIC = 0, 1

PRECISIONS = {"fp64": LBM_FP64, "fp32": LBM_FP32, "fp16": LBM_FP16_STORE, "bf16": LBM_BF16_STORE,
              "fp32u64": LBM_FP32_U64}
SCHEMES = {"pc": LBM_SCHEME_PC, "explicit": LBM_SCHEME_EXPLICIT, "extrap": LBM_SCHEME_EXTRAP}
ROUNDINGS = {"nearest": LBM_ROUND_NEAREST, "stochastic": LBM_ROUND_STOCHASTIC}

EXPORTED_EXTRA: list = []
EXPORTED = [
    "lbm_workspace_bytes", "lbm_create", "lbm_set_material", "lbm_set_body_force", "lbm_set_boundary",
    "lbm_set_fields", "lbm_step", "lbm_read_fields", "lbm_read_diagnostics_noalloc", "lbm_get_dt", "lbm_destroy",
    "lbm_last_error",
    "lbm_set_tiling", "lbm_get_tiling", "lbm_set_steps_per_launch", "lbm_get_steps_per_launch",
    "lbm_resident_blocks", "lbm_set_rounding", "lbm_read_derived", "lbm_sample", "lbm_batch_read_derived",
    "lbm_batch_sample", "lbm_workspace_bytes_walled", "lbm_set_general_path", "lbm_set_mask",
    "lbm_batch_plate_bytes", "lbm_batch_plate_tiles", "lbm_batch_workspace_bytes", "lbm_batch_create",
    "lbm_batch_add", "lbm_batch_step", "lbm_batch_query", "lbm_batch_read", "lbm_batch_retire", "lbm_batch_info",
    "lbm_batch_destroy", "lbm_batch_last_error", "lbm_batch_set_steps_per_launch",
    "lbm_batch_get_steps_per_launch",
]


class LbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"lbm status {status}: {message}")
        self.status = status


class lbm_diagnostics(ctypes.Structure):
    _fields_ = [
        ("momentum", ctypes.c_double * 2),
        ("mass_moment", ctypes.c_double),
        ("energy", ctypes.c_double),
        ("min_J", ctypes.c_double),
        ("max_strain", ctypes.c_double),
        ("unstable", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("steps", ctypes.c_int64),
    ]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the native library; raise if it is missing (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "or python paper_2208_13769_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, dp, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t
    lib.lbm_workspace_bytes.restype = sz
    lib.lbm_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.lbm_workspace_bytes_walled.restype = sz
    lib.lbm_workspace_bytes_walled.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.lbm_set_general_path.restype = ctypes.c_int
    lib.lbm_set_general_path.argtypes = [vp, ctypes.c_int]
    lib.lbm_set_mask.restype = ctypes.c_int
    lib.lbm_set_mask.argtypes = [vp, vp]
    lib.lbm_create.restype = ctypes.c_int
    lib.lbm_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                               vp, sz, vp, ctypes.POINTER(vp)]
    lib.lbm_set_material.restype = ctypes.c_int
    lib.lbm_set_material.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.lbm_set_body_force.restype = ctypes.c_int
    lib.lbm_set_body_force.argtypes = [vp, dp]
    lib.lbm_set_boundary.restype = ctypes.c_int
    lib.lbm_set_boundary.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp]
    lib.lbm_set_fields.restype = ctypes.c_int
    lib.lbm_set_fields.argtypes = [vp, dp, dp]
    lib.lbm_step.restype = ctypes.c_int
    lib.lbm_step.argtypes = [vp, ctypes.c_int64]
    lib.lbm_read_fields.restype = ctypes.c_int
    lib.lbm_read_fields.argtypes = [vp, dp, dp, dp, ctypes.POINTER(lbm_diagnostics)]
    lib.lbm_read_diagnostics_noalloc.restype = ctypes.c_int
    lib.lbm_read_diagnostics_noalloc.argtypes = [vp, ctypes.POINTER(lbm_diagnostics)]
    ip = ctypes.POINTER(ctypes.c_int)
    lib.lbm_read_derived.restype = ctypes.c_int
    lib.lbm_read_derived.argtypes = [vp, dp, dp, dp]
    lib.lbm_sample.restype = ctypes.c_int
    lib.lbm_sample.argtypes = [vp, ctypes.c_int, ip, ip, dp]
    lib.lbm_get_dt.restype = ctypes.c_int
    lib.lbm_get_dt.argtypes = [vp, dp]
    lib.lbm_destroy.restype = None
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_set_tiling.restype = ctypes.c_int
    lib.lbm_set_tiling.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.lbm_get_tiling.restype = ctypes.c_int
    lib.lbm_get_tiling.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.lbm_set_steps_per_launch.restype = ctypes.c_int
    lib.lbm_set_steps_per_launch.argtypes = [vp, ctypes.c_int]
    lib.lbm_get_steps_per_launch.restype = ctypes.c_int
    lib.lbm_get_steps_per_launch.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.lbm_set_rounding.restype = ctypes.c_int
    lib.lbm_set_rounding.argtypes = [vp, ctypes.c_int, ctypes.c_uint64]
    lib.lbm_resident_blocks.restype = ctypes.c_int
    lib.lbm_resident_blocks.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_last_error.argtypes = [vp]
    _lib = lib
    return lib


def _dptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(status: int, handle) -> None:
    if status != LBM_OK:
        msg = load_library().lbm_last_error(handle)
        raise LbmError(status, msg.decode() if msg else "")


# ---- C names -------------------------------------------------------------

def lbm_workspace_bytes(nx: int, ny: int, precision: int) -> int:
    return int(load_library().lbm_workspace_bytes(nx, ny, precision))


def lbm_workspace_bytes_walled(nx: int, ny: int, precision: int) -> int:
    return int(load_library().lbm_workspace_bytes_walled(nx, ny, precision))


def lbm_set_general_path(h, on: bool):
    _check(load_library().lbm_set_general_path(h, int(bool(on))), h)


def lbm_set_mask(h, solid):
    if solid is None:
        _check(load_library().lbm_set_mask(h, None), h)
        return
    m = np.ascontiguousarray(np.asarray(solid) != 0, dtype=np.uint8)
    _check(load_library().lbm_set_mask(h, m.ctypes.data_as(ctypes.c_void_p)), h)


def lbm_create(nx, ny, dx, precision, scheme, workspace_ptr, ws_bytes, stream_ptr):
    h = ctypes.c_void_p()
    _check(load_library().lbm_create(nx, ny, dx, precision, scheme, workspace_ptr, ws_bytes, stream_ptr,
                                     ctypes.byref(h)), None)
    return h


def lbm_set_material(h, rho0, lam, mu, tau_over_dt):
    _check(load_library().lbm_set_material(h, rho0, lam, mu, tau_over_dt), h)


def lbm_set_body_force(h, b):
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    if b.size != 2:
        raise ValueError(f"body force of {b.size} values; expected 2")
    _check(load_library().lbm_set_body_force(h, _dptr(b)), h)


def lbm_set_boundary(h, edge, bc, value=None):
    v = None if value is None else np.ascontiguousarray(value, dtype=np.float64).ravel()
    if v is not None and v.size != 2:
        raise ValueError(f"boundary value of {v.size} values; expected 2")
    _check(load_library().lbm_set_boundary(h, edge, bc, _dptr(v)), h)


def lbm_set_fields(h, u0, v0):
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    _check(load_library().lbm_set_fields(h, _dptr(u0), _dptr(v0)), h)


def lbm_step(h, nsteps: int):
    _check(load_library().lbm_step(h, int(nsteps)), h)


SAMPLE_FIELDS = ("u_x", "u_y", "v_x", "v_y", "P11", "P12", "P21", "P22", "sigma11", "sigma12", "sigma21",
                 "sigma22", "E11", "E12", "E21", "E22", "W")


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def lbm_read_derived(h, sigma=None, E=None, W=None):
    _check(load_library().lbm_read_derived(h, _dptr(sigma), _dptr(E), _dptr(W)), h)


def lbm_sample(h, xs, ys) -> np.ndarray:
    """[n][17] values at the nodes (xs[k], ys[k]); columns as SAMPLE_FIELDS."""
    xs = np.ascontiguousarray(xs, dtype=np.int32).ravel()
    ys = np.ascontiguousarray(ys, dtype=np.int32).ravel()
    if len(xs) != len(ys):
        raise ValueError(f"{len(xs)} x coordinates for {len(ys)} y coordinates")
    out = np.empty((len(xs), 17))
    _check(load_library().lbm_sample(h, len(xs), _iptr(xs), _iptr(ys), _dptr(out)), h)
    return out


def lbm_read_diagnostics_noalloc(h, diag: lbm_diagnostics) -> int:
    """Diagnostics through the entry point that allocates nothing (its scratch
    is a static device array); returns the status (LBM_ERR_UNSTABLE is
    returned, not raised)."""
    st = load_library().lbm_read_diagnostics_noalloc(h, ctypes.byref(diag))
    if st not in (LBM_OK, LBM_ERR_UNSTABLE):
        _check(st, h)
    return st


def lbm_read_fields(h, u=None, v=None, P=None, diag: lbm_diagnostics | None = None) -> int:
    """Fill the given arrays; returns the status (LBM_ERR_UNSTABLE is returned, not raised)."""
    st = load_library().lbm_read_fields(h, _dptr(u), _dptr(v), _dptr(P),
                                        ctypes.byref(diag) if diag is not None else None)
    if st not in (LBM_OK, LBM_ERR_UNSTABLE):
        _check(st, h)
    return st


def lbm_get_dt(h) -> float:
    out = ctypes.c_double()
    _check(load_library().lbm_get_dt(h, ctypes.byref(out)), h)
    return out.value


def lbm_set_tiling(h, block: int, n_segs: int):
    _check(load_library().lbm_set_tiling(h, int(block), int(n_segs)), h)


def lbm_get_tiling(h):
    b, n = ctypes.c_int(), ctypes.c_int()
    _check(load_library().lbm_get_tiling(h, ctypes.byref(b), ctypes.byref(n)), h)
    return b.value, n.value


def lbm_set_steps_per_launch(h, k: int):
    _check(load_library().lbm_set_steps_per_launch(h, int(k)), h)


def lbm_set_rounding(h, rounding: int, seed: int = 0):
    _check(load_library().lbm_set_rounding(h, int(rounding), int(seed) & ((1 << 64) - 1)), h)


def lbm_resident_blocks(h, block: int, steps_per_launch: int) -> int:
    out = ctypes.c_int()
    _check(load_library().lbm_resident_blocks(h, int(block), int(steps_per_launch), ctypes.byref(out)), h)
    return out.value


def lbm_get_steps_per_launch(h) -> int:
    out = ctypes.c_int()
    _check(load_library().lbm_get_steps_per_launch(h, ctypes.byref(out)), h)
    return out.value


def lbm_destroy(h):
    load_library().lbm_destroy(h)


def lbm_last_error(h) -> str:
    msg = load_library().lbm_last_error(h)
    return msg.decode() if msg else ""


# ---- convenience wrapper -------------------------------------------------

@dataclass
class Diagnostics:
    momentum: np.ndarray
    mass_moment: float
    energy: float
    min_J: float
    max_strain: float
    unstable: bool
    steps: int


class Solver:
    """One plate on one GPU; the workspace is a torch uint8 tensor."""

    def __init__(self, nx: int, ny: int, dx: float = 1.0, precision: str = "fp64", scheme: str = "pc",
                 device: str = "cuda:0", stream=None, walled: bool = False):
        """walled: size the workspace for walls on the x edges (the general
        step); always so for the "extrap" scheme."""
        import torch

        self.nx, self.ny, self.dx = nx, ny, dx
        self.precision = precision
        prec = PRECISIONS[precision]
        walled = walled or scheme == "extrap"
        nbytes = (lbm_workspace_bytes_walled if walled else lbm_workspace_bytes)(nx, ny, prec)
        if nbytes == 0:
            raise LbmError(LBM_ERR_ARG, "invalid size or precision")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = lbm_create(nx, ny, dx, prec, SCHEMES[scheme], ctypes.c_void_p(self.workspace.data_ptr()),
                            nbytes, ctypes.c_void_p(self.stream.cuda_stream))

    def close(self):
        if getattr(self, "h", None) is not None:
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_material(self, rho0: float, lam: float, mu: float, tau_over_dt: float):
        lbm_set_material(self.h, rho0, lam, mu, tau_over_dt)

    def set_body_force(self, b):
        lbm_set_body_force(self.h, b)

    def set_boundary(self, edge: int, bc: int, value=None):
        lbm_set_boundary(self.h, edge, bc, value)

    def set_general_path(self, on: bool):
        lbm_set_general_path(self.h, on)

    def set_mask(self, solid):
        """solid: [ny][nx] array, nonzero for material, 0 for holes; None removes it."""
        if solid is not None and np.shape(solid) != (self.ny, self.nx):
            raise ValueError(f"mask of shape {np.shape(solid)} for a {self.ny} x {self.nx} plate")
        lbm_set_mask(self.h, solid)

    def set_fields(self, u0, v0):
        """u0, v0: [2][ny][nx] start displacement and velocity (physical units)."""
        for name, a in (("u0", u0), ("v0", v0)):
            if np.shape(a) != (2, self.ny, self.nx):
                raise ValueError(f"{name} of shape {np.shape(a)}; expected (2, {self.ny}, {self.nx})")
        lbm_set_fields(self.h, u0, v0)

    def step(self, n: int):
        lbm_step(self.h, n)

    def set_tiling(self, block: int, n_segs: int):
        lbm_set_tiling(self.h, block, n_segs)

    def tiling(self):
        return lbm_get_tiling(self.h)

    def set_steps_per_launch(self, k: int):
        lbm_set_steps_per_launch(self.h, k)

    def steps_per_launch(self) -> int:
        return lbm_get_steps_per_launch(self.h)

    def set_rounding(self, rounding, seed: int = 0):
        """rounding: "nearest" / "stochastic" or LBM_ROUND_*."""
        lbm_set_rounding(self.h, ROUNDINGS.get(rounding, rounding), seed)

    def resident_blocks(self, block: int, steps_per_launch: int) -> int:
        return lbm_resident_blocks(self.h, block, steps_per_launch)

    @property
    def dt(self) -> float:
        return lbm_get_dt(self.h)

    def read_derived(self):
        """Return (sigma, E, W): Cauchy stress and Green-Lagrange strain
        [2][2][ny][nx] and strain-energy density [ny][nx]."""
        ny, nx = self.ny, self.nx
        sig, E, W = np.empty((2, 2, ny, nx)), np.empty((2, 2, ny, nx)), np.empty((ny, nx))
        lbm_read_derived(self.h, sig, E, W)
        return sig, E, W

    def sample(self, xs, ys) -> np.ndarray:
        return lbm_sample(self.h, xs, ys)

    def sample_series(self, xs, ys, nsteps: int, every: int):
        """Advance nsteps, sampling the nodes before the first step and after
        every `every` steps: returns (steps since the call [m], values
        [m][n][17])."""
        steps, vals = [], []
        done = 0
        while True:
            steps.append(done)
            vals.append(self.sample(xs, ys))
            if done >= nsteps:
                break
            k = min(every, nsteps - done)
            self.step(k)
            done += k
        return np.array(steps), np.array(vals)

    def read(self, want_fields: bool = True):
        """Return (u, v, P, Diagnostics, status)."""
        ny, nx = self.ny, self.nx
        u = np.empty((2, ny, nx)) if want_fields else None
        v = np.empty((2, ny, nx)) if want_fields else None
        P = np.empty((2, 2, ny, nx)) if want_fields else None
        d = lbm_diagnostics()
        st = lbm_read_fields(self.h, u, v, P, d)
        diag = Diagnostics(np.array(d.momentum[:]), d.mass_moment, d.energy, d.min_J, d.max_strain,
                           bool(d.unstable), int(d.steps))
        return u, v, P, diag, st
