"""Thin ctypes binding of libchemora (include/chemora.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  The
library must have been built (``__graft_entry__.build()``); if it is missing
every call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchemora.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "chemora.h")

OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_DEVICE, ERR_HOST_NOMEM = 0, 1, 2, 3, 4
WAVE, BSSN, WAVE5 = 1, 2, 3
FP64, MIXED = 0, 1
BC_PERIODIC, BC_GAUGEWAVE, BC_CALLER = 0, 1, 2
SLICING_1PLUSLOG, SLICING_HARMONIC = 0, 1
SHIFT_FROZEN, SHIFT_GAMMADRIVER = 0, 1


class ChemoraError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"chemora status {status}: {msg}")
        self.status = status


class GridDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ghost", ctypes.c_int32),
                ("h", ctypes.c_double * 3), ("origin", ctypes.c_double * 3),
                ("system", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("boundary", ctypes.c_int32), ("slicing", ctypes.c_int32),
                ("shift", ctypes.c_int32), ("shift_F", ctypes.c_double),
                ("eta", ctypes.c_double), ("gw_amp", ctypes.c_double),
                ("gw_wavelength", ctypes.c_double), ("gw_axis", ctypes.c_int32),
                ("enforce", ctypes.c_int32), ("ko_sigma", ctypes.c_double),
                ("fd_order", ctypes.c_int32)]


class Patch(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_void_p), ("state", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p)]


class Parent(ctypes.Structure):
    _fields_ = [("coarse", ctypes.c_void_p), ("levels", ctypes.c_void_p * 3),
                ("times", ctypes.c_double * 3), ("ntimes", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "chemora_grid_create": (ctypes.c_int, [ctypes.POINTER(GridDesc), ctypes.POINTER(_vp)]),
        "chemora_grid_destroy": (ctypes.c_int, [_vp]),
        "chemora_grid_layout": (ctypes.c_int, [_vp, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                               ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "chemora_workspace_bytes": (i64, [_vp]),
        "chemora_fill_ghosts": (ctypes.c_int, [_vp, _vp, dbl, _vp]),
        "chemora_rhs": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
        "chemora_rk4_step": (ctypes.c_int, [_vp, _vp, _vp, dbl, dbl, i32, _vp]),
        "chemora_constraints_workspace_bytes": (i64, [_vp]),
        "chemora_constraints": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "chemora_constraints_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
        "chemora_energy_workspace_bytes": (i64, [_vp]),
        "chemora_energy": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "chemora_batch_meta_bytes": (i64, [i32]),
        "chemora_batch_step": (ctypes.c_int, [ctypes.POINTER(Patch), i32, _vp, dbl, dbl, i32,
                                              _vp]),
        "chemora_batch_step_levels": (ctypes.c_int, [ctypes.POINTER(Patch), ctypes.POINTER(Parent),
                                                     i32, _vp, dbl, dbl, i32, _vp]),
        "chemora_batch_release": (ctypes.c_int, [_vp]),
        "chemora_autotune": (ctypes.c_int, [ctypes.POINTER(Patch), i32, _vp, ctypes.c_char_p]),
        "chemora_batch_tile": (ctypes.c_int, [ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]),
        "chemora_batch_model": (ctypes.c_int, [ctypes.POINTER(i32), ctypes.POINTER(i32), i32, i32,
                                               i32, i32, i32, i32, i32, ctypes.POINTER(dbl)]),
        "chemora_probe_copy": (ctypes.c_int, [_vp, _vp, i64, _vp]),
        "chemora_probe_fma_bytes": (i64, []),
        "chemora_probe_fma": (ctypes.c_int, [i32, _vp, i32, ctypes.POINTER(dbl), _vp]),
        "chemora_prolong": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(dbl), i32,
                                           dbl, _vp, _vp, _vp]),
        "chemora_restrict": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
        "chemora_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of every function declared in include/chemora.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(chemora_\w+)\s*\(", text)))


def last_error() -> str:
    return lib().chemora_last_error().decode()


def check(status: int) -> None:
    if status != OK:
        raise ChemoraError(status, last_error())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Grid:
    """A grid object (host metadata) plus helpers to move states in and out of
    the library's padded device layout."""

    def __init__(self, n, ghost, h, origin=(0.0, 0.0, 0.0), system=WAVE, precision=FP64,
                 boundary=BC_PERIODIC, slicing=SLICING_1PLUSLOG, shift=SHIFT_GAMMADRIVER,
                 shift_F=0.75, eta=2.0, gw_amp=0.1, gw_wavelength=1.0, gw_axis=0,
                 enforce=0, ko_sigma=0.0, fd_order=0):
        d = GridDesc()
        d.n[:] = [int(v) for v in n]
        d.ghost = int(ghost)
        d.h[:] = [float(v) for v in (h if np.ndim(h) else (h, h, h))]
        d.origin[:] = [float(v) for v in origin]
        d.system, d.precision, d.boundary = system, precision, boundary
        d.slicing, d.shift, d.shift_F, d.eta = slicing, shift, float(shift_F), float(eta)
        d.gw_amp, d.gw_wavelength, d.gw_axis = float(gw_amp), float(gw_wavelength), gw_axis
        d.enforce, d.ko_sigma = int(enforce), float(ko_sigma)
        d.fd_order = int(fd_order)
        self.desc = d
        h_ = ctypes.c_void_p()
        check(lib().chemora_grid_create(ctypes.byref(d), ctypes.byref(h_)))
        self.handle = h_
        nv = ctypes.c_int32()
        st = (ctypes.c_int64 * 4)()
        off = ctypes.c_int64()
        el = ctypes.c_int64()
        check(lib().chemora_grid_layout(h_, ctypes.byref(nv), st, ctypes.byref(off),
                                        ctypes.byref(el)))
        self.nvars = nv.value
        self.strides = tuple(st)
        self.interior_offset = off.value
        self.state_elems = el.value
        self.n = tuple(d.n)
        self.g = d.ghost

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.chemora_grid_destroy(h)
            self.handle = None

    # ---- memory
    def workspace_bytes(self) -> int:
        return lib().chemora_workspace_bytes(self.handle)

    def new_state(self, device="cuda"):
        import torch
        return torch.zeros(self.state_elems, dtype=torch.float64, device=device)

    def new_workspace(self, device="cuda"):
        import torch
        return torch.empty(self.workspace_bytes() // 8, dtype=torch.float64, device=device)

    def view(self, state, var: int, ghosts: bool = True):
        """(z, y, x) strided view of one grid function of a flat state tensor"""
        import torch
        g = self.g if ghosts else 0
        _, sy, sz, sv = self.strides
        off = self.interior_offset + var * sv - g * (1 + sy + sz)
        shape = (self.n[2] + 2 * g, self.n[1] + 2 * g, self.n[0] + 2 * g)
        return torch.as_strided(state, shape, (sz, sy, 1), off)

    def upload(self, interior: np.ndarray, state=None, device="cuda"):
        """interior values (nvar, n_z, n_y, n_x) -> state tensor (ghosts zero)"""
        import torch
        assert interior.shape == (self.nvars, self.n[2], self.n[1], self.n[0]), interior.shape
        if state is None:
            state = self.new_state(device)
        for v in range(self.nvars):
            self.view(state, v, ghosts=False).copy_(torch.from_numpy(np.ascontiguousarray(interior[v])))
        return state

    def upload_full(self, full: np.ndarray, state=None, device="cuda"):
        """values including ghosts (nvar, n_z+2g, n_y+2g, n_x+2g) -> state tensor"""
        import torch
        if state is None:
            state = self.new_state(device)
        for v in range(self.nvars):
            self.view(state, v).copy_(torch.from_numpy(np.ascontiguousarray(full[v])))
        return state

    def download(self, state, ghosts: bool = False, nvars: int | None = None) -> np.ndarray:
        nv = self.nvars if nvars is None else nvars
        return np.stack([self.view(state, v, ghosts).cpu().numpy() for v in range(nv)])

    # ---- compute (asynchronous on the current stream)
    def fill_ghosts(self, state, t: float = 0.0, stream=None):
        check(lib().chemora_fill_ghosts(self.handle, _ptr(state), float(t), _stream(stream)))

    def rhs(self, state, out=None, stream=None):
        if out is None:
            out = self.new_state(state.device)
        check(lib().chemora_rhs(self.handle, _ptr(state), _ptr(out), _stream(stream)))
        return out

    def rk4_step(self, state, workspace, t: float, dt: float, nsteps: int = 1, stream=None):
        check(lib().chemora_rk4_step(self.handle, _ptr(state), _ptr(workspace), float(t),
                                     float(dt), int(nsteps), _stream(stream)))

    def constraints(self, state, hm=None, norms=None, workspace=None, stream=None):
        import torch
        if norms is None:
            norms = torch.zeros(4, dtype=torch.float64, device=state.device)
        if workspace is None:
            nb = lib().chemora_constraints_workspace_bytes(self.handle)
            workspace = torch.empty(max(nb // 8, 1), dtype=torch.float64, device=state.device)
        check(lib().chemora_constraints(self.handle, _ptr(state), _ptr(hm), _ptr(norms),
                                        _ptr(workspace), _stream(stream)))
        return norms


    def constraints_noalloc(self, state, norms, hm=None, stream=None):
        """chemora_constraints_noalloc: norms (device double[4]) is the caller's"""
        check(lib().chemora_constraints_noalloc(self.handle, _ptr(state), _ptr(hm), _ptr(norms),
                                                _stream(stream)))
        return norms

    def energy(self, state, eps=None, total=None, workspace=None, stream=None):
        """Fig. 1's Energy calculation (WAVE5): total = sum(eps) h^3 (device)"""
        import torch
        if total is None:
            total = torch.zeros(1, dtype=torch.float64, device=state.device)
        if workspace is None:
            nb = lib().chemora_energy_workspace_bytes(self.handle)
            workspace = torch.empty(max(nb // 8, 1), dtype=torch.float64, device=state.device)
        check(lib().chemora_energy(self.handle, _ptr(state), _ptr(eps), _ptr(total),
                                   _ptr(workspace), _stream(stream)))
        return total


def probe_fma(precision: int, out, iters: int, stream=None) -> float:
    """launch the FMA throughput probe; returns the launch's flop count"""
    fl = ctypes.c_double()
    check(lib().chemora_probe_fma(int(precision), _ptr(out), int(iters), ctypes.byref(fl),
                                  _stream(stream)))
    return fl.value


def probe_copy(dst, src, nbytes: int, stream=None):
    check(lib().chemora_probe_copy(_ptr(dst), _ptr(src), int(nbytes), _stream(stream)))


def prolong(coarse: "Grid", coarse_states, fine: "Grid", fine_state, times=None, t=0.0,
            stream=None):
    """Fill fine_state's ghost zones from one to three coarse states (at
    ``times``, combined at time ``t``); see chemora_prolong."""
    levels = [coarse_states] if hasattr(coarse_states, "data_ptr") else list(coarse_states)
    times = [0.0] * len(levels) if times is None else list(times)
    ptrs = (_vp * len(levels))(*[s.data_ptr() for s in levels])
    tt = (ctypes.c_double * len(times))(*[float(v) for v in times])
    check(lib().chemora_prolong(coarse.handle, ptrs, tt, len(levels), float(t), fine.handle,
                                _ptr(fine_state), _stream(stream)))


def restrict(coarse: "Grid", coarse_state, fine: "Grid", fine_state, stream=None):
    """Inject fine interior values into the coinciding coarse interior points."""
    check(lib().chemora_restrict(coarse.handle, _ptr(coarse_state), fine.handle,
                                 _ptr(fine_state), _stream(stream)))


def batch_meta_bytes(npatches: int) -> int:
    return lib().chemora_batch_meta_bytes(int(npatches))


def _patch_array(grids, states, workspaces):
    arr = (Patch * len(grids))()
    for q, (g, s, w) in enumerate(zip(grids, states, workspaces)):
        arr[q].grid = g.handle.value
        arr[q].state = s.data_ptr()
        arr[q].workspace = w.data_ptr()
    return arr


def batch_step(grids, states, workspaces, meta, t: float, dt: float, nsteps: int = 1,
               stream=None, parents=None):
    """parents: None, or one entry per patch: None (analytic ghosts) or
    (coarse Grid, [coarse level states], [times])"""
    arr = _patch_array(grids, states, workspaces)
    if parents is None:
        check(lib().chemora_batch_step(arr, len(grids), _ptr(meta), float(t), float(dt),
                                       int(nsteps), _stream(stream)))
        return
    par = (Parent * len(grids))()
    for q, pr in enumerate(parents):
        if pr is None:
            continue
        coarse, levels, times = pr
        par[q].coarse = coarse.handle.value
        for l, (lv, tt) in enumerate(zip(levels, times)):
            par[q].levels[l] = lv.data_ptr()
            par[q].times[l] = float(tt)
        par[q].ntimes = len(levels)
    check(lib().chemora_batch_step_levels(arr, par, len(grids), _ptr(meta), float(t), float(dt),
                                          int(nsteps), _stream(stream)))


def batch_release(meta):
    check(lib().chemora_batch_release(_ptr(meta)))


def autotune(grids, states, workspaces, meta, table_path: str | None = None):
    arr = _patch_array(grids, states, workspaces)
    path = table_path.encode() if table_path else None
    check(lib().chemora_autotune(arr, len(grids), _ptr(meta), path))


def batch_model(dims, tiles, kind: int, fd_order: int = 4, per_cu: int = 1, grid: int = 256,
                ghost_width: int = 0, per_item: bool = False) -> float:
    """the autotuner's model: predicted launch duration (wavefront-plane units)"""
    np_ = len(dims)
    d = (ctypes.c_int32 * (3 * np_))(*[int(v) for n in dims for v in n])
    t = (ctypes.c_int32 * (3 * np_))(*[int(v) for tl in tiles for v in tl])
    out = ctypes.c_double()
    check(lib().chemora_batch_model(d, t, np_, int(kind), int(fd_order), int(per_cu), int(grid),
                                    int(ghost_width), int(bool(per_item)), ctypes.byref(out)))
    return out.value


def batch_tile(n, precision=FP64):
    nn = (ctypes.c_int32 * 3)(*[int(v) for v in n])
    out = (ctypes.c_int32 * 3)()
    check(lib().chemora_batch_tile(nn, int(precision), out))
    return tuple(out)
