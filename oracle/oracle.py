"""Python access to the FP64 CPU oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module. The HIP product path
never does, and this module imports nothing from that path.

The oracle works in physical units with the paper's own notation: lattice
spacing dX, reference density rho0, Lame parameters lam and mu of the
plane-strain neo-Hooke law (Sec. 7, eq. (27)), relaxation time tau given as
tau/dt, body force b. Fields are numpy arrays laid out as ``u[a, y, x]``,
``v[a, y, x]`` and ``P[a, b, y, x]``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

PERIODIC, DIRICHLET_J, NEUMANN_T = 0, 1, 2
PC, EXPLICIT, EXTRAP = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction of a*b+c into FMA)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-math-errno",
               "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("dx", ctypes.c_double), ("rho0", ctypes.c_double),
        ("lam", ctypes.c_double), ("mu", ctypes.c_double),
        ("tau_over_dt", ctypes.c_double),
        ("body", ctypes.c_double * 2),
        ("scheme", ctypes.c_int),
        ("bc_ymin", ctypes.c_int), ("bc_ymax", ctypes.c_int),
        ("val_ymin", ctypes.c_double * 2), ("val_ymax", ctypes.c_double * 2),
        ("bc_xmin", ctypes.c_int), ("bc_xmax", ctypes.c_int),
        ("val_xmin", ctypes.c_double * 2), ("val_xmax", ctypes.c_double * 2),
        ("solid", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        _lib.oracle_dt.restype = ctypes.c_double
        _lib.oracle_dt.argtypes = [pp]
        _lib.oracle_init.argtypes = [pp, dp, dp, dp, dp, dp]
        _lib.oracle_step.argtypes = [pp, dp, dp, dp, dp, ctypes.c_int]
        _lib.oracle_step_prev.argtypes = [pp, dp, dp, dp, dp, dp, ctypes.c_int]
        _lib.oracle_fields.argtypes = [pp, dp, dp, dp, dp, dp]
        _lib.oracle_diagnostics.argtypes = [pp, dp, dp, dp, dp, dp]
        _lib.oracle_piola.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp]
        _lib.oracle_poisson.argtypes = [ctypes.c_double, dp, dp]
        _lib.oracle_cauchy.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp]
        _lib.oracle_green_lagrange.argtypes = [dp, dp]
        _lib.oracle_derived.argtypes = [pp, dp, dp, dp, dp, dp]
        _lib.oracle_strain_energy.restype = ctypes.c_double
        _lib.oracle_strain_energy.argtypes = [ctypes.c_double, ctypes.c_double, dp]
        _lib.oracle_equilibrium.argtypes = [pp, ctypes.c_double, dp, dp, dp]
        _lib.oracle_source_pop.argtypes = [pp, dp, dp]
        _lib.oracle_velocity.argtypes = [pp, ctypes.c_int, dp]
        _lib.oracle_weight.restype = ctypes.c_double
        _lib.oracle_weight.argtypes = [ctypes.c_int]
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Params:
    nx: int
    ny: int
    dx: float = 1.0
    rho0: float = 1.0
    lam: float = 0.1
    mu: float = 0.05
    tau_over_dt: float = 0.8
    body: tuple = (0.0, 0.0)
    scheme: int = PC
    bc_ymin: int = PERIODIC
    bc_ymax: int = PERIODIC
    val_ymin: tuple = (0.0, 0.0)
    val_ymax: tuple = (0.0, 0.0)
    bc_xmin: int = PERIODIC
    bc_xmax: int = PERIODIC
    val_xmin: tuple = (0.0, 0.0)
    val_xmax: tuple = (0.0, 0.0)
    solid: object = None  # [ny][nx] 1 material / 0 hole (reading Q23), or None

    def c(self) -> _Params:
        p = _Params()
        p.nx, p.ny = self.nx, self.ny
        p.dx, p.rho0, p.lam, p.mu = self.dx, self.rho0, self.lam, self.mu
        p.tau_over_dt = self.tau_over_dt
        p.body[0], p.body[1] = self.body
        p.scheme = self.scheme
        p.bc_ymin, p.bc_ymax = self.bc_ymin, self.bc_ymax
        p.val_ymin[0], p.val_ymin[1] = self.val_ymin
        p.val_ymax[0], p.val_ymax[1] = self.val_ymax
        p.bc_xmin, p.bc_xmax = self.bc_xmin, self.bc_xmax
        p.val_xmin[0], p.val_xmin[1] = self.val_xmin
        p.val_xmax[0], p.val_xmax[1] = self.val_xmax
        if self.solid is not None:
            m = np.ascontiguousarray(self.solid, dtype=np.uint8)
            assert m.shape == (self.ny, self.nx)
            p._solid = m  # keeps the array alive with the structure
            p.solid = m.ctypes.data
        return p


def dt(params: Params) -> float:
    """Time step dt = dX / (sqrt(3) sqrt(mu / rho0))."""
    return lib().oracle_dt(ctypes.byref(params.c()))


class Solver:
    """State (f, u, j) of one plate, advanced by the oracle."""

    def __init__(self, params: Params, u0: np.ndarray, v0: np.ndarray):
        self.p = params
        ny, nx = params.ny, params.nx
        self.f = np.zeros((9, ny, nx))
        self.u = np.zeros((2, ny, nx))
        self.j = np.zeros((2, ny, nx))
        self.jprev = np.zeros((2, ny, nx))  # j one step back (the extrapolation variant)
        # displacement of each momentum wall (edges xmin, xmax, ymin, ymax),
        # zero at the start and advanced by the oracle with every step
        self.wall = np.zeros((4, 2))
        self.step_index = 0
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        assert u0.shape == (2, ny, nx) and v0.shape == (2, ny, nx)
        self._pc = params.c()
        rc = lib().oracle_init(ctypes.byref(self._pc), _ptr(u0), _ptr(v0),
                               _ptr(self.f), _ptr(self.u), _ptr(self.j))
        if rc != 0:
            raise ValueError("oracle_init rejected the parameters")
        self.jprev[...] = self.j

    @property
    def t(self) -> float:
        return self.step_index * dt(self.p)

    def step(self, n: int) -> None:
        rc = lib().oracle_step_prev(ctypes.byref(self._pc), _ptr(self.f), _ptr(self.u), _ptr(self.j),
                                    _ptr(self.jprev), _ptr(self.wall), int(n))
        if rc != 0:
            raise ValueError("oracle_step rejected the parameters")
        self.step_index += int(n)

    def set_boundary_value(self, edge: str, value):
        """New j* or T* of an edge ("xmin", "xmax", "ymin", "ymax") from the
        next step on (a load history applied step by step)."""
        self.p = dataclasses.replace(self.p, **{"val_" + edge: tuple(value)})
        self._pc = self.p.c()

    def fields(self):
        """Return (u, v, P) in physical units."""
        ny, nx = self.p.ny, self.p.nx
        v = np.zeros((2, ny, nx))
        P = np.zeros((2, 2, ny, nx))
        lib().oracle_fields(ctypes.byref(self._pc), _ptr(self.u), _ptr(self.j), _ptr(self.wall), _ptr(v), _ptr(P))
        return self.u.copy(), v, P

    def derived(self):
        """Return (sigma, E, W): Cauchy stress and Green-Lagrange strain
        [2][2][ny][nx] and strain-energy density [ny][nx], physical units."""
        ny, nx = self.p.ny, self.p.nx
        sig = np.zeros((2, 2, ny, nx))
        E = np.zeros((2, 2, ny, nx))
        W = np.zeros((ny, nx))
        lib().oracle_derived(ctypes.byref(self._pc), _ptr(self.u), _ptr(self.wall), _ptr(sig), _ptr(E), _ptr(W))
        return sig, E, W

    def diagnostics(self) -> dict:
        out = np.zeros(7)
        lib().oracle_diagnostics(ctypes.byref(self._pc), _ptr(self.f), _ptr(self.u), _ptr(self.j),
                                 _ptr(self.wall), _ptr(out))
        return {"momentum": out[0:2].copy(), "mass_moment": out[2], "energy": out[3],
                "min_J": out[4], "max_strain": out[5], "unstable": bool(out[6])}


def run(params: Params, u0, v0, nsteps: int):
    """Initialise, advance nsteps and return (u, v, P, diagnostics)."""
    s = Solver(params, u0, v0)
    s.step(nsteps)
    u, v, P = s.fields()
    return u, v, P, s.diagnostics()


# ---- single-point functions, for the unit pins ----

def piola(lam: float, mu: float, H) -> np.ndarray:
    H = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(4))
    P = np.zeros(4)
    lib().oracle_piola(lam, mu, _ptr(H), _ptr(P))
    return P.reshape(2, 2)


def poisson(mu: float, H) -> np.ndarray:
    H = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(4))
    P = np.zeros(4)
    lib().oracle_poisson(mu, _ptr(H), _ptr(P))
    return P.reshape(2, 2)


def cauchy(lam: float, mu: float, H) -> np.ndarray:
    H = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(4))
    out = np.zeros(4)
    lib().oracle_cauchy(lam, mu, _ptr(H), _ptr(out))
    return out.reshape(2, 2)


def green_lagrange(H) -> np.ndarray:
    H = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(4))
    out = np.zeros(4)
    lib().oracle_green_lagrange(_ptr(H), _ptr(out))
    return out.reshape(2, 2)


def strain_energy(lam: float, mu: float, H) -> float:
    H = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(4))
    return lib().oracle_strain_energy(lam, mu, _ptr(H))


def equilibrium(params: Params, r: float, j, Pb) -> np.ndarray:
    j = np.ascontiguousarray(np.asarray(j, dtype=np.float64).reshape(2))
    Pb = np.ascontiguousarray(np.asarray(Pb, dtype=np.float64).reshape(4))
    out = np.zeros(9)
    lib().oracle_equilibrium(ctypes.byref(params.c()), r, _ptr(j), _ptr(Pb), _ptr(out))
    return out


def source_populations(params: Params, S) -> np.ndarray:
    S = np.ascontiguousarray(np.asarray(S, dtype=np.float64).reshape(2))
    out = np.zeros(9)
    lib().oracle_source_pop(ctypes.byref(params.c()), _ptr(S), _ptr(out))
    return out


def velocities(params: Params) -> np.ndarray:
    out = np.zeros((9, 2))
    for i in range(9):
        c = np.zeros(2)
        lib().oracle_velocity(ctypes.byref(params.c()), i, _ptr(c))
        out[i] = c
    return out


def weights() -> np.ndarray:
    return np.array([lib().oracle_weight(i) for i in range(9)])
