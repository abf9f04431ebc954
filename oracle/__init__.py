"""CPU oracle for the Chemora right-hand-side path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it.
It shares no code with the HIP path.

The arithmetic lives in ``oracle.c`` (plain FP64 C, no FMA contraction,
OpenMP over z-planes).  This module only compiles it, loads it with ctypes and
marshals numpy arrays in the oracle's own unpadded layout
``(nvar, n_z+2g, n_y+2g, n_x+2g)``, x fastest, point index i in [-g, n+g).

What each routine follows in the paper (arXiv:1410.1764):
  * ``wave_rhs``: eq. (1), two-variable reading (du/dt = rho, drho/dt = Lap u),
    4th-order centred differences (Sec. III.B.2, Discretisation description).
  * ``wave5_rhs`` / ``wave5_energy``: eq. (1) in the paper's own first-order
    five-variable form and Fig. 1's Energy calculation.
  * ``bssn_rhs``: the Einstein equations in BSSN form that Sec. III.D evolves
    (chi variant; 1+log or harmonic slicing; Gamma-driver or frozen shift;
    lopsided stencils for advection).
  * ``fill_periodic`` / ``fill_gaugewave``: ghost zones owned by the driver
    (Sec. II).
  * ``rk4``: classical RK4 method of lines, as scheduled by a time-integrator
    thorn (Sec. II).
  * ``constraints``: Hamiltonian and momentum constraints of the physics
    system (Sec. III.B.1) with RMS norms.
  * ``prolong`` / ``restrict``: coupling of two refinement levels at ratio 2
    (Sec. IV, the mesh-refinement driver): degree-5 tensor-product Lagrange
    interpolation into fine ghost zones; injection back onto the coarse level.

Parity status of each routine (pins in ``tests/test_oracle_*.py``): all are
pinned to closed forms, convergence orders or invariants.  The 1+log /
harmonic lapse and Gamma-driver shift right-hand sides are pinned on data
with closed-form derivatives (sheared moving coordinates and a constant
shift, with smooth lapse, K and B^i): 4th-order convergence to the
definitions evaluated with exact derivatives, and every plausible sign,
coefficient or missing-term mistake misses them by far more than that
(``tests/test_oracle_gauge.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c11",
          "-Wall", "-shared", "-fPIC"]

WAVE, BSSN, WAVE5 = 1, 2, 3
BC_PERIODIC, BC_GAUGEWAVE = 0, 1
NVAR = {WAVE: 2, BSSN: 24, WAVE5: 5}


def build() -> str:
    """Compile liboracle.so next to its source (always recompiles)."""
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("g", ctypes.c_int),
                ("h", ctypes.c_double * 3), ("origin", ctypes.c_double * 3),
                ("slicing", ctypes.c_int), ("shift", ctypes.c_int),
                ("shift_F", ctypes.c_double), ("eta", ctypes.c_double),
                ("gw_amp", ctypes.c_double), ("gw_d", ctypes.c_double),
                ("gw_axis", ctypes.c_int), ("ko_sigma", ctypes.c_double),
                ("enforce", ctypes.c_int), ("fd_order", ctypes.c_int)]


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(LIB)
    P = ctypes.POINTER(_Params)
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_fill_periodic.argtypes = [P, ctypes.c_int, _DP]
    lib.orc_fill_gaugewave.argtypes = [P, ctypes.c_double, _DP]
    lib.orc_wave_rhs.argtypes = [P, _DP, _DP]
    lib.orc_bssn_rhs.argtypes = [P, _DP, _DP]
    lib.orc_wave5_rhs.argtypes = [P, _DP, _DP]
    lib.orc_wave5_energy.argtypes = [P, _DP, _DP]
    lib.orc_wave5_energy.restype = ctypes.c_double
    lib.orc_rk4.argtypes = [P, ctypes.c_int, ctypes.c_int, _DP, ctypes.c_double,
                            ctypes.c_double, ctypes.c_int]
    lib.orc_rk4.restype = ctypes.c_int
    lib.orc_bssn_constraints.argtypes = [P, _DP, _DP, _DP]
    lib.orc_stencil.argtypes = [P, _DP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _DP, _DP]
    lib.orc_bssn_enforce.argtypes = [P, _DP]
    lib.orc_prolong.argtypes = [P, ctypes.POINTER(_DP), _DP, ctypes.c_int, ctypes.c_double, P,
                                _DP, ctypes.c_int]
    lib.orc_prolong.restype = ctypes.c_int
    lib.orc_rk4_prolong.argtypes = [P, ctypes.c_int, _DP, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, P, ctypes.POINTER(_DP), _DP, ctypes.c_int]
    lib.orc_rk4_prolong.restype = ctypes.c_int
    lib.orc_restrict.argtypes = [P, _DP, P, _DP, ctypes.c_int]
    lib.orc_restrict.restype = ctypes.c_int
    _lib = lib
    return lib


def num_threads() -> int:
    return _load().orc_num_threads()


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


class Block:
    """A uniform block: n interior points per axis, g ghosts, spacing h.

    Coordinates of point (i, j, k) are origin + (i, j, k) * h.  Gauge and
    gauge-wave parameters only matter for BSSN.
    """

    def __init__(self, n, g, h, origin=(0.0, 0.0, 0.0), slicing=0, shift=1,
                 shift_F=0.75, eta=2.0, gw_amp=0.1, gw_d=1.0, gw_axis=0, ko_sigma=0.0,
                 enforce=0, fd_order=4):
        self.n = tuple(int(v) for v in n)
        self.g = int(g)
        self.h = tuple(float(v) for v in (h if np.ndim(h) else (h, h, h)))
        self.origin = tuple(float(v) for v in origin)
        self.slicing, self.shift = int(slicing), int(shift)
        self.shift_F, self.eta = float(shift_F), float(eta)
        self.gw_amp, self.gw_d, self.gw_axis = float(gw_amp), float(gw_d), int(gw_axis)
        p = _Params()
        p.n[:] = self.n
        p.g = self.g
        p.h[:] = self.h
        p.origin[:] = self.origin
        p.slicing, p.shift, p.shift_F, p.eta = self.slicing, self.shift, self.shift_F, self.eta
        p.gw_amp, p.gw_d, p.gw_axis = self.gw_amp, self.gw_d, self.gw_axis
        self.ko_sigma, self.enforce = float(ko_sigma), int(enforce)
        p.ko_sigma, p.enforce = self.ko_sigma, self.enforce
        self.fd_order = int(fd_order)
        p.fd_order = self.fd_order
        self._p = p

    @property
    def ext(self):
        """array shape of one grid function, (z, y, x) with ghosts"""
        g = self.g
        return (self.n[2] + 2 * g, self.n[1] + 2 * g, self.n[0] + 2 * g)

    def zeros(self, nvar: int) -> np.ndarray:
        return np.zeros((nvar, *self.ext))

    def interior(self, a: np.ndarray) -> np.ndarray:
        g = self.g
        return a[..., g:g + self.n[2], g:g + self.n[1], g:g + self.n[0]]

    def embed(self, interior: np.ndarray) -> np.ndarray:
        """interior data (nvar, n_z, n_y, n_x) -> array with zero ghosts"""
        a = self.zeros(interior.shape[0])
        self.interior(a)[...] = interior
        return a

    def coords(self, with_ghosts: bool = True):
        """1-D coordinate arrays (x, y, z)"""
        g = self.g if with_ghosts else 0
        return tuple(self.origin[d] + self.h[d] * np.arange(-g, self.n[d] + g)
                     for d in range(3))


def fill_periodic(b: Block, y: np.ndarray) -> None:
    _load().orc_fill_periodic(ctypes.byref(b._p), y.shape[0], _ptr(y))


def fill_gaugewave(b: Block, y: np.ndarray, t: float) -> None:
    assert y.shape[0] == 24
    _load().orc_fill_gaugewave(ctypes.byref(b._p), float(t), _ptr(y))


def wave_rhs(b: Block, y: np.ndarray) -> np.ndarray:
    r = np.zeros_like(y)
    _load().orc_wave_rhs(ctypes.byref(b._p), _ptr(y), _ptr(r))
    return r


def wave5_rhs(b: Block, y: np.ndarray) -> np.ndarray:
    assert y.shape[0] == 5
    r = np.zeros_like(y)
    _load().orc_wave5_rhs(ctypes.byref(b._p), _ptr(y), _ptr(r))
    return r


def wave5_energy(b: Block, y: np.ndarray, want_field: bool = False):
    """(total energy, eps field or None): Fig. 1's Energy calculation"""
    eps = b.zeros(1) if want_field else None
    e = _load().orc_wave5_energy(ctypes.byref(b._p), _ptr(y), _ptr(eps))
    return e, eps


def bssn_rhs(b: Block, y: np.ndarray) -> np.ndarray:
    assert y.shape[0] == 24 and b.g >= 3
    r = np.zeros_like(y)
    _load().orc_bssn_rhs(ctypes.byref(b._p), _ptr(y), _ptr(r))
    return r


def rk4(b: Block, system: int, bc: int, y: np.ndarray, t: float, dt: float,
        nsteps: int) -> None:
    """Advance y in place by nsteps classical RK4 steps; ghosts refilled."""
    assert y.shape[0] == NVAR[system]
    rc = _load().orc_rk4(ctypes.byref(b._p), system, bc, _ptr(y), float(t), float(dt),
                         int(nsteps))
    if rc != 0:
        raise MemoryError("oracle rk4: allocation failed")


def constraints(b: Block, y: np.ndarray, want_fields: bool = True):
    """(hm, norms): H, M^1..3 at interior points and their RMS norms."""
    hm = b.zeros(4) if want_fields else None
    norms = np.zeros(4)
    _load().orc_bssn_constraints(ctypes.byref(b._p), _ptr(y), _ptr(hm), _ptr(norms))
    return hm, norms


def stencil(b: Block, f: np.ndarray, kind: int, a: int, bdir: int = 0,
            sgn: np.ndarray | None = None) -> np.ndarray:
    """kind 1: centred d_a; 2: centred d_a d_b; 3: lopsided d_a (side by sign of sgn);
    4: sixth difference along a (Kreiss-Oliger stencil, unscaled)"""
    out = np.zeros_like(f)
    _load().orc_stencil(ctypes.byref(b._p), _ptr(f), kind, a, bdir, _ptr(sgn), _ptr(out))
    return out


def enforce(b: Block, y: np.ndarray) -> None:
    """In place at interior points: det gt = 1 (gt scaled by det^-1/3), then
    tr At = 0 with respect to the rescaled metric."""
    assert y.shape[0] == NVAR[BSSN]
    _load().orc_bssn_enforce(ctypes.byref(b._p), _ptr(y))


def prolong(coarse: Block, yc, fine: Block, yf: np.ndarray, times=None, t=0.0) -> None:
    """Fill every ghost point of yf (fine block) from the coarse block (valid
    ghosts) by degree-5 tensor-product Lagrange interpolation, ratio 2.

    yc is one coarse state, or a list of 1-3 coarse states at ``times``,
    combined with Lagrange weights in time at ``t``."""
    levels = [yc] if isinstance(yc, np.ndarray) else list(yc)
    times = [0.0] * len(levels) if times is None else list(times)
    assert len(times) == len(levels) and all(a.shape[0] == yf.shape[0] for a in levels)
    arr = (_DP * len(levels))(*[_ptr(a) for a in levels])
    tt = np.ascontiguousarray(times, dtype=np.float64)
    if _load().orc_prolong(ctypes.byref(coarse._p), arr, _ptr(tt), len(levels), float(t),
                           ctypes.byref(fine._p), _ptr(yf), yf.shape[0]):
        raise ValueError("oracle prolong: levels not in ratio 2, misaligned, out of reach, "
                         "or bad time levels")


def rk4_prolong(b: Block, system: int, y: np.ndarray, t: float, dt: float, nsteps: int,
                coarse: Block, yc, times) -> None:
    """Advance y (a refined block) in place by nsteps RK4 steps; the ghost
    zones of every stage (and of the result) are prolongated from the coarse
    levels yc at ``times`` at the stage's time (see prolong)."""
    levels = list(yc)
    assert len(levels) == len(times) and all(a.shape[0] == y.shape[0] for a in levels)
    arr = (_DP * len(levels))(*[_ptr(a) for a in levels])
    tt = np.ascontiguousarray(times, dtype=np.float64)
    if _load().orc_rk4_prolong(ctypes.byref(b._p), system, _ptr(y), float(t), float(dt),
                               int(nsteps), ctypes.byref(coarse._p), arr, _ptr(tt), len(levels)):
        raise ValueError("oracle rk4_prolong: a stage's prolongation failed (levels, reach or "
                         "time levels) or allocation failed")


def restrict(coarse: Block, yc: np.ndarray, fine: Block, yf: np.ndarray) -> None:
    """Copy fine interior values into the coarse interior points they coincide with."""
    assert yc.shape[0] == yf.shape[0]
    if _load().orc_restrict(ctypes.byref(coarse._p), _ptr(yc), ctypes.byref(fine._p), _ptr(yf),
                            yc.shape[0]):
        raise ValueError("oracle restrict: levels not in ratio 2 or misaligned")
