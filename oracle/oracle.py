"""ctypes wrapper over the FP64 oracle library (test infrastructure only).

Arrays are numpy float64 (fields, populations) and uint8 (masks), C-ordered
with shapes (..., nz, ny, nx) so that x is fastest, matching the library's
``idx = x + nx*(y + ny*z)``.  Populations have shape (2, 19, nz, ny, nx).
"""
import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_LIB = None


class _CParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("half_force_shift", ctypes.c_int32),
        ("tau", ctypes.c_double * 2),
        ("G", ctypes.c_double),
        ("g", (ctypes.c_double * 3) * 2),
        ("open_x", ctypes.c_int32),
        ("rho_in", ctypes.c_double),
        ("rho_out", ctypes.c_double),
        ("frozen", ctypes.POINTER(ctypes.c_double)),
    ]


def _lib():
    global _LIB
    if _LIB is None:
        path = os.environ.get("MCLBM_ORACLE_LIB")   # a planted-mistake build (tests only)
        if path is None:
            path = _build.LIB
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
                _build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER(_CParams)
        dp = ctypes.POINTER(ctypes.c_double)
        bp = ctypes.POINTER(ctypes.c_uint8)
        ip = ctypes.POINTER(ctypes.c_int32)
        lib.orc_lattice.argtypes = [ip, dp, ip]
        lib.orc_viscosity.argtypes = [ctypes.c_double]
        lib.orc_viscosity.restype = ctypes.c_double
        lib.orc_mixture_tau.argtypes = [P, ctypes.c_double, ctypes.c_double]
        lib.orc_mixture_tau.restype = ctypes.c_double
        lib.orc_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        lib.orc_source.argtypes = [dp, dp, dp]
        lib.orc_densities.argtypes = [P, bp, dp, dp]
        lib.orc_pseudopotential.argtypes = [P, bp, dp, dp, dp]
        lib.orc_forces.argtypes = [P, bp, dp, dp, dp]
        lib.orc_velocity.argtypes = [P, bp, dp, dp, dp, dp]
        lib.orc_pressure.argtypes = [P, bp, dp, dp]
        lib.orc_fields.argtypes = [P, bp, dp, dp, dp, dp, dp, dp]
        lib.orc_init_equilibrium.argtypes = [P, bp, dp, dp]
        lib.orc_step.argtypes = [P, bp, dp, dp, dp, dp, dp, dp, dp]
        lib.orc_run.argtypes = [P, bp, dp, dp, dp, ctypes.c_int32, dp, dp, dp, dp]
        lib.orc_run.restype = ctypes.c_int32
        lib.orc_diagnostics.argtypes = [P, bp, dp, dp, dp, dp]
        lib.orc_loss_snw.argtypes = [P, bp, bp, dp]
        lib.orc_loss_snw.restype = ctypes.c_double
        lib.orc_num_threads.restype = ctypes.c_int32
        lib.orc_set_num_threads.argtypes = [ctypes.c_int32]
        lib.orc_open_rebuild.argtypes = [P, bp, dp]
        _LIB = lib
    return _LIB


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _b(a):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def num_threads() -> int:
    return int(_lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the lattice-wide loops from now on."""
    _lib().orc_set_num_threads(int(n))


def lattice_tables():
    """(e[19,3] int, w[19] float64, opposite[19] int) as the oracle holds them."""
    e = np.zeros(57, np.int32)
    w = np.zeros(19, np.float64)
    opp = np.zeros(19, np.int32)
    _lib().orc_lattice(e.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _d(w),
                       opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return e.reshape(19, 3), w, opp


@dataclass
class OracleParams:
    shape: tuple                      # (nx, ny, nz)
    tau: tuple = (1.0, 1.0)
    G: float = 3.5
    g: tuple = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    half_force_shift: bool = True

    def c(self):
        p = _CParams()
        p.nx, p.ny, p.nz = (int(v) for v in self.shape)
        p.half_force_shift = 1 if self.half_force_shift else 0
        p.tau[0], p.tau[1] = float(self.tau[0]), float(self.tau[1])
        p.G = float(self.G)
        for s in range(2):
            for a in range(3):
                p.g[s][a] = float(self.g[s][a])
        return p


class Oracle:
    """FP64 reference stepping of one lattice (two population buffers)."""

    def __init__(self, params: OracleParams, solid: np.ndarray, xi: np.ndarray = None):
        self.p = params
        self._cp = params.c()
        nx, ny, nz = params.shape
        self.dims = (nz, ny, nx)
        self.N = nx * ny * nz
        self.solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(self.dims)
        if xi is None:
            xi = np.zeros(self.dims)
        self.xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(self.dims)
        self.fa = np.zeros((2, 19) + self.dims)
        self.fb = np.zeros_like(self.fa)
        self.rho = np.zeros((2,) + self.dims)
        self.psi = np.zeros_like(self.rho)
        self.F = np.zeros((2, 3) + self.dims)
        self.u = np.zeros((3,) + self.dims)
        self.t = 0
        self.frozen = None

    @property
    def cp(self):
        return ctypes.byref(self._cp)

    # state ------------------------------------------------------------
    def init_equilibrium(self, rho: np.ndarray):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape((2,) + self.dims)
        _lib().orc_init_equilibrium(self.cp, _b(self.solid), _d(rho), _d(self.fa))
        self.t = 0

    def set_state(self, f: np.ndarray):
        self.fa[...] = f

    def set_open_x(self, rho_in: float, rho_out: float):
        """Open inlet (x = 0) and outlet (x = nx-1) planes from now on: component 1
        held at rho_in at the inlet, component 2 at rho_out at the outlet (NEEM);
        the entering populations of the other component keep the values they have
        now (the first call captures them)."""
        nz, ny, nx = self.dims
        if self.frozen is None:
            self.frozen = np.zeros((2, 19, nz, ny))
            self.frozen[0] = self.fa[1, :, :, :, 0]      # inlet: component 2
            self.frozen[1] = self.fa[0, :, :, :, nx - 1]  # outlet: component 1
        self._cp.open_x = 1
        self._cp.rho_in = float(rho_in)
        self._cp.rho_out = float(rho_out)
        self._cp.frozen = _d(self.frozen)

    @property
    def f(self):
        return self.fa

    def run(self, nsteps: int):
        which = _lib().orc_run(self.cp, _b(self.solid), _d(self.xi), _d(self.fa), _d(self.fb),
                               int(nsteps), _d(self.rho), _d(self.psi), _d(self.F), _d(self.u))
        if which == 1:
            self.fa, self.fb = self.fb, self.fa
        self.t += nsteps

    # readouts at the current time level --------------------------------
    def fields(self):
        """rho (2,...), psi-hat (2,...), F (2,3,...), u (3,...) of the current state."""
        _lib().orc_fields(self.cp, _b(self.solid), _d(self.xi), _d(self.fa), _d(self.rho),
                          _d(self.psi), _d(self.F), _d(self.u))
        return self.rho.copy(), self.psi.copy(), self.F.copy(), self.u.copy()

    def pressure(self):
        rho, _, _, _ = self.fields()
        P = np.zeros(self.dims)
        _lib().orc_pressure(self.cp, _b(self.solid), _d(rho), _d(P))
        return P

    def diagnostics(self):
        rho, _, _, u = self.fields()
        out = np.zeros(6)
        _lib().orc_diagnostics(self.cp, _b(self.solid), _d(self.fa), _d(rho), _d(u), _d(out))
        return out

    def loss_snw(self, region: np.ndarray):
        region = np.ascontiguousarray(region, dtype=np.uint8).reshape(self.dims)
        return _lib().orc_loss_snw(self.cp, _b(self.solid), _b(region), _d(self.fa))


# per-node building blocks ------------------------------------------------
def equilibrium(rho: float, u) -> np.ndarray:
    out = np.zeros(19)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    _lib().orc_equilibrium(float(rho), _d(uu), _d(out))
    return out


def source(u, F) -> np.ndarray:
    out = np.zeros(19)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    FF = np.ascontiguousarray(F, dtype=np.float64)
    _lib().orc_source(_d(uu), _d(FF), _d(out))
    return out


def viscosity(tau: float) -> float:
    return _lib().orc_viscosity(float(tau))


def mixture_tau(params: OracleParams, rho1: float, rho2: float) -> float:
    cp = params.c()
    return _lib().orc_mixture_tau(ctypes.byref(cp), float(rho1), float(rho2))
