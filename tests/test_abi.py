"""The C ABI without a GPU: the library loads, exports every function that
include/chemora.h declares, and rejects bad arguments with the documented
status before touching the device."""
import ctypes

import pytest

from paper_1410_1764_amd import chemora as C


def test_library_exports_every_declared_function():
    L = C.lib()
    names = C.header_functions()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def _create(**kw):
    base = dict(n=(8, 8, 8), ghost=3, h=0.1, system=C.BSSN)
    base.update(kw)
    return C.Grid(**base)


@pytest.mark.parametrize("kw,msg", [
    (dict(n=(0, 8, 8)), "n[0]"),
    (dict(ghost=2), "ghost"),
    (dict(system=C.WAVE, ghost=1), "ghost"),
    (dict(ghost=9), "ghost"),
    (dict(h=(0.1, 0.0, 0.1)), "h[1]"),
    (dict(h=(0.1, 0.1, float("nan"))), "h[2]"),
    (dict(system=4), "system"),
    (dict(precision=2), "precision"),
    (dict(boundary=7), "boundary"),
    (dict(n=(8, 2, 8)), "periodic"),
    (dict(system=C.WAVE, ghost=2, boundary=C.BC_GAUGEWAVE), "BSSN"),
    (dict(boundary=C.BC_GAUGEWAVE, gw_amp=1.5), "amplitude"),
    (dict(boundary=C.BC_GAUGEWAVE, gw_axis=3), "axis"),
    (dict(boundary=C.BC_GAUGEWAVE, gw_wavelength=0.0), "wavelength"),
    (dict(slicing=5), "slicing"),
    (dict(shift=5), "shift"),
    (dict(enforce=2), "enforce"),
    (dict(ko_sigma=-0.1), "ko_sigma"),
    (dict(ko_sigma=float("inf")), "ko_sigma"),
    (dict(system=C.WAVE, ghost=2, ko_sigma=0.1), "BSSN system only"),
    (dict(system=C.WAVE, ghost=2, enforce=1), "BSSN system only"),
    (dict(fd_order=5), "fd_order"),
    (dict(fd_order=6), "ghost >= 4"),
    (dict(ghost=4, fd_order=8), "ghost >= 5"),
    (dict(ghost=4, fd_order=6, ko_sigma=0.1), "fd_order 4"),
    (dict(system=C.WAVE, ghost=4, fd_order=6), "BSSN system only"),
])
def test_grid_create_rejects(kw, msg):
    with pytest.raises(C.ChemoraError) as e:
        _create(**kw)
    assert e.value.status == C.ERR_INVALID
    assert msg in str(e.value)


def test_null_arguments():
    L = C.lib()
    assert L.chemora_grid_create(None, None) == C.ERR_INVALID
    h = ctypes.c_void_p()
    assert L.chemora_grid_create(None, ctypes.byref(h)) == C.ERR_INVALID
    assert "NULL" in C.last_error()
    assert L.chemora_workspace_bytes(None) == -1
    assert L.chemora_rhs(None, None, None, None) == C.ERR_INVALID
    g = _create()
    assert L.chemora_rhs(g.handle, None, None, None) == C.ERR_INVALID
    assert L.chemora_rk4_step(g.handle, None, None, 0.0, 0.1, 1, None) == C.ERR_INVALID
    # misaligned pointers are rejected before any launch
    assert L.chemora_rhs(g.handle, ctypes.c_void_p(8), ctypes.c_void_p(4096), None) == C.ERR_INVALID
    assert "aligned" in C.last_error()
    # overlapping state / rhs
    assert L.chemora_rhs(g.handle, ctypes.c_void_p(4096), ctypes.c_void_p(4096), None) == C.ERR_INVALID
    assert "overlap" in C.last_error()
    assert L.chemora_rk4_step(g.handle, ctypes.c_void_p(4096), ctypes.c_void_p(1 << 40), 0.0,
                              0.1, -1, None) == C.ERR_INVALID
    assert L.chemora_rk4_step(g.handle, ctypes.c_void_p(4096), ctypes.c_void_p(1 << 40), 0.0,
                              float("inf"), 1, None) == C.ERR_INVALID


def test_caller_boundary_rejected_by_rk4():
    g = _create(boundary=C.BC_CALLER)
    assert C.lib().chemora_rk4_step(g.handle, ctypes.c_void_p(4096), ctypes.c_void_p(1 << 40),
                                    0.0, 0.1, 1, None) == C.ERR_INVALID
    assert C.lib().chemora_fill_ghosts(g.handle, ctypes.c_void_p(4096), 0.0, None) == C.OK


def test_constraints_unsupported_for_wave():
    g = C.Grid((8, 8, 8), 2, 0.1, system=C.WAVE)
    st = C.lib().chemora_constraints(g.handle, ctypes.c_void_p(4096), None,
                                     ctypes.c_void_p(8192), ctypes.c_void_p(1 << 20), None)
    assert st == C.ERR_UNSUPPORTED


@pytest.mark.parametrize("n,g,system", [((128, 128, 128), 3, C.BSSN), ((37, 29, 19), 2, C.WAVE),
                                        ((5, 3, 4), 3, C.BSSN)])
def test_layout(n, g, system):
    gr = C.Grid(n, g, 0.1, system=system, boundary=C.BC_CALLER)
    nv = 24 if system == C.BSSN else 2
    assert gr.nvars == nv
    sx, sy, sz, sv = gr.strides
    assert sx == 1
    # interior x = 0 on a 128-byte boundary, rows 128-byte multiples
    assert gr.interior_offset % 16 == 0 and sy % 16 == 0
    assert sy >= n[0] + 2 * g + 16 - g
    assert sz == sy * (n[1] + 2 * g)
    assert sv == sz * (n[2] + 2 * g)
    assert gr.state_elems == nv * sv
    # the lowest ghost point is still inside the array
    assert gr.interior_offset - g * (1 + sy + sz) >= 0
    assert gr.workspace_bytes() == 3 * gr.state_elems * 8


def test_batch_meta_bytes_rejects_empty():
    assert C.batch_meta_bytes(0) == -1


def _bssn_gw(n=(24, 24, 24), precision=C.FP64):
    return C.Grid(n, 3, 1 / 64, system=C.BSSN, precision=precision, boundary=C.BC_GAUGEWAVE,
                  slicing=C.SLICING_HARMONIC, shift=C.SHIFT_FROZEN)


def test_batch_argument_validation():
    L = C.lib()
    g1, g2 = _bssn_gw(), _bssn_gw(precision=C.MIXED)
    arr = (C.Patch * 2)()
    for q, g in enumerate((g1, g2)):
        arr[q].grid = g.handle.value
        arr[q].state = 4096 * (q + 1) * 1024
        arr[q].workspace = 4096 * (q + 5) * 1024
    meta = ctypes.c_void_p(1 << 30)
    assert L.chemora_batch_step(None, 2, meta, 0.0, 0.1, 1, None) == C.ERR_INVALID
    assert L.chemora_batch_step(arr, 0, meta, 0.0, 0.1, 1, None) == C.ERR_INVALID
    assert L.chemora_batch_step(arr, 2, meta, 0.0, 0.1, 1, None) == C.ERR_INVALID
    assert "precision" in C.last_error()
    assert L.chemora_batch_step(arr, 1, None, 0.0, 0.1, 1, None) == C.ERR_INVALID
    assert L.chemora_batch_step(arr, 1, meta, 0.0, 0.1, -1, None) == C.ERR_INVALID
    wave = C.Grid((8, 8, 8), 2, 0.1, system=C.WAVE)
    arr[1].grid = wave.handle.value
    assert L.chemora_batch_step(arr, 2, meta, 0.0, 0.1, 1, None) == C.ERR_INVALID
    assert "gauge-wave" in C.last_error()
    arr[1].state = 0
    assert L.chemora_batch_step(arr, 2, meta, 0.0, 0.1, 1, None) == C.ERR_INVALID
    assert L.chemora_autotune(arr, 0, meta, None) == C.ERR_INVALID
    # one fd_order per batch
    g6 = C.Grid((24, 24, 24), 4, 1 / 64, system=C.BSSN, boundary=C.BC_GAUGEWAVE,
                slicing=C.SLICING_HARMONIC, shift=C.SHIFT_FROZEN, fd_order=6)
    arr[0].grid, arr[1].grid = g1.handle.value, g6.handle.value
    arr[0].state, arr[1].state = 4096 * 1024, 8192 * 1024
    assert L.chemora_batch_step(arr, 2, meta, 0.0, 0.1, 1, None) == C.ERR_INVALID
    assert "fd_order" in C.last_error()
    # FP64 batches of 6th-order patches are switched off
    arr[0].grid = g6.handle.value
    assert L.chemora_batch_step(arr, 1, meta, 0.0, 0.1, 1, None) == C.ERR_UNSUPPORTED
    assert C.batch_meta_bytes(64) > 64 * 200
    assert C.batch_meta_bytes(64) % 256 == 0


def test_batch_tile_model():
    t = C.batch_tile((96, 90, 80))
    assert t[0] * t[1] == 256 and t[2] >= 1
    assert C.batch_tile((24, 30, 40))[0] <= 32  # narrow patches get narrow tiles


def test_energy_unsupported_for_other_systems():
    g = C.Grid((8, 8, 8), 2, 0.1, system=C.WAVE)
    st = C.lib().chemora_energy(g.handle, ctypes.c_void_p(4096), None, ctypes.c_void_p(8192),
                                ctypes.c_void_p(1 << 20), None)
    assert st == C.ERR_UNSUPPORTED
    g5 = C.Grid((8, 8, 8), 2, 0.1, system=C.WAVE5)
    assert g5.nvars == 5
    assert C.lib().chemora_energy(g5.handle, None, None, None, None, None) == C.ERR_INVALID


def test_level_pair_validation():
    L = C.lib()
    co = C.Grid((16, 16, 16), 3, 0.1, system=C.BSSN, boundary=C.BC_CALLER)
    fi = C.Grid((12, 12, 12), 3, 0.05, origin=(0.3, 0.3, 0.3), system=C.BSSN,
                boundary=C.BC_CALLER)
    cs = (ctypes.c_void_p * 3)(1 << 30, 2 << 30, 3 << 30)
    tt = (ctypes.c_double * 3)(0.0, 0.1, 0.2)
    fs = ctypes.c_void_p(8 << 30)

    def pro(c=co, f=fi, states=cs, times=tt, n=1, t=0.0, out=fs):
        return L.chemora_prolong(c.handle, states, times, n, t, f.handle, out, None)

    assert pro(n=0) == C.ERR_INVALID and "ntimes" in C.last_error()
    assert pro(n=4) == C.ERR_INVALID
    assert pro(out=None) == C.ERR_INVALID
    assert pro(out=ctypes.c_void_p((8 << 30) + 8)) == C.ERR_INVALID
    assert "aligned" in C.last_error()
    assert pro(t=float("nan")) == C.ERR_INVALID
    same = (ctypes.c_double * 3)(0.0, 0.0, 0.2)
    assert pro(times=same, n=2) == C.ERR_INVALID and "distinct" in C.last_error()
    over = (ctypes.c_void_p * 1)(8 << 30)
    assert pro(states=over) == C.ERR_INVALID and "overlap" in C.last_error()
    ratio = C.Grid((12, 12, 12), 3, 0.04, origin=(0.32, 0.32, 0.32), system=C.BSSN,
                   boundary=C.BC_CALLER)
    assert pro(f=ratio) == C.ERR_INVALID and "twice" in C.last_error()
    shifted = C.Grid((12, 12, 12), 3, 0.05, origin=(0.31, 0.3, 0.3), system=C.BSSN,
                     boundary=C.BC_CALLER)
    assert pro(f=shifted) == C.ERR_INVALID and "whole number" in C.last_error()
    wave = C.Grid((12, 12, 12), 3, 0.05, origin=(0.3, 0.3, 0.3), system=C.WAVE,
                  boundary=C.BC_CALLER)
    assert pro(f=wave) == C.ERR_INVALID and "systems" in C.last_error()
    # the fine ghosts would need coarse points beyond the coarse ghost zones
    far = C.Grid((12, 12, 12), 3, 0.05, origin=(-0.05, 0.3, 0.3), system=C.BSSN,
                 boundary=C.BC_CALLER)
    assert pro(f=far) == C.ERR_INVALID and "outside the coarse extended range" in C.last_error()
    assert L.chemora_restrict(co.handle, None, fi.handle, fs, None) == C.ERR_INVALID
    assert L.chemora_restrict(co.handle, ctypes.c_void_p(8 << 30), fi.handle, fs,
                              None) == C.ERR_INVALID
    assert "overlap" in C.last_error()
    assert L.chemora_restrict(co.handle, ctypes.c_void_p(1 << 30), ratio.handle, fs,
                              None) == C.ERR_INVALID
    # no coinciding interior points: nothing is enqueued
    away = C.Grid((4, 4, 4), 3, 0.05, origin=(5.0, 5.0, 5.0), system=C.BSSN,
                  boundary=C.BC_CALLER)
    assert L.chemora_restrict(co.handle, ctypes.c_void_p(1 << 30), away.handle, fs,
                              None) == C.OK


def test_constraints_noalloc_refuses_grids_beyond_its_buffer():
    """checked on the host before any device call: a grid whose partial sums
    exceed the static buffer (2^20 doubles) is refused with INVALID"""
    n = (1024, 1024, 1024)
    g = C.Grid(n, 3, 1.0 / 1024, system=C.BSSN)
    need = C.lib().chemora_constraints_workspace_bytes(g.handle)
    assert need > 8 * (1 << 20)
    st = ctypes.c_void_p(1 << 20)  # aligned, never dereferenced
    nrm = ctypes.c_void_p(1 << 21)
    rc = C.lib().chemora_constraints_noalloc(g.handle, st, None, nrm, None)
    assert rc == C.ERR_INVALID
    assert b"static buffer" in C.lib().chemora_last_error()


def test_probe_fma_validation():
    L = C.lib()
    fl = ctypes.c_double()
    assert L.chemora_probe_fma_bytes() == 8192 * 256 * 8
    assert L.chemora_probe_fma(C.FP64, None, 4, ctypes.byref(fl), None) == C.ERR_INVALID
    assert L.chemora_probe_fma(C.FP64, ctypes.c_void_p(8), 4, ctypes.byref(fl), None) \
        == C.ERR_INVALID
    assert "aligned" in C.last_error()
    assert L.chemora_probe_fma(7, ctypes.c_void_p(4096), 4, ctypes.byref(fl), None) \
        == C.ERR_INVALID
    assert L.chemora_probe_fma(C.FP64, ctypes.c_void_p(4096), 0, ctypes.byref(fl), None) \
        == C.ERR_INVALID


def test_batch_model_wave_quantisation_and_schedule():
    """The autotuner's model on cases whose answer follows from its
    definition: a ragged tile costs its whole waves; the XCD shares and the
    round robin over the persistent grid decide the makespan; more resident
    workgroups per CU than two stretch it."""
    one = C.batch_model([(64, 64, 8)], [(32, 8, 1)], kind=1, grid=8)
    # 128 equal items, 8 XCD shares of 16, one workgroup per XCD
    item = one / 16
    assert C.batch_model([(64, 64, 8)], [(32, 8, 1)], kind=1, grid=128) == pytest.approx(item)
    assert C.batch_model([(64, 64, 8)], [(32, 8, 1)], kind=1, grid=1024) == pytest.approx(item)
    # wave quantisation: 33 points wide needs as many 32-wide tiles as 64
    assert C.batch_model([(33, 64, 8)], [(32, 8, 1)], kind=1, grid=8) == pytest.approx(one)
    assert C.batch_model([(32, 64, 8)], [(32, 8, 1)], kind=1, grid=8) == pytest.approx(one / 2)
    # 9 items over 8 shares: one share holds two
    assert C.batch_model([(32, 8, 9)], [(32, 8, 1)], kind=1, grid=8) == pytest.approx(2 * item)
    # per-CU occupancy beyond two waves per SIMD does not speed a workgroup up
    assert C.batch_model([(64, 64, 8)], [(32, 8, 1)], kind=1, grid=8, per_cu=4) \
        == pytest.approx(2 * one)
    # ghost items only add
    assert C.batch_model([(64, 64, 8)], [(32, 8, 1)], kind=1, grid=8, ghost_width=3) > one
    # the cached-load kind is priced above the staged kinds per point
    assert C.batch_model([(64, 64, 8)], [(32, 8, 1)], kind=0, grid=8) > one
    # one item per workgroup: the greedy hand-out balances what the static
    # stride cannot (a long item first, then short ones)
    mixed = [(32, 8, 16), (32, 8, 1), (32, 8, 1), (32, 8, 1)]
    tiles = [(32, 8, 1)] * 4
    stat = C.batch_model(mixed, tiles, kind=1, grid=16)
    dyn = C.batch_model(mixed, tiles, kind=1, grid=16, per_item=True)
    assert dyn <= stat
    assert C.batch_model([(64, 64, 8)], [(32, 8, 1)], kind=1, grid=8, per_item=True) \
        == pytest.approx(one)
    with pytest.raises(C.ChemoraError):
        C.batch_model([(64, 64, 8)], [(32, 8, 1)], kind=8)


def test_batch_parent_validation_without_a_device():
    """chemora_batch_step_levels refuses bad parents before touching the
    device: ratio and reach (INVALID), a time level inside a patch's state
    (INVALID), parents for high-order batches or wide ghost zones
    (UNSUPPORTED)."""
    L = C.lib()
    fine = C.Grid((16, 16, 16), 3, 1 / 64, origin=(4 / 64, 4 / 64, 4 / 64), system=C.BSSN,
                  boundary=C.BC_GAUGEWAVE, slicing=C.SLICING_HARMONIC, shift=C.SHIFT_FROZEN)
    coarse = C.Grid((24, 24, 24), 3, 1 / 32, system=C.BSSN, boundary=C.BC_CALLER)
    arr = (C.Patch * 1)()
    arr[0].grid = fine.handle.value
    arr[0].state = 1 << 32
    arr[0].workspace = 1 << 33
    meta = ctypes.c_void_p(1 << 30)
    par = (C.Parent * 1)()

    def step():
        return L.chemora_batch_step_levels(arr, par, 1, meta, 0.0, 0.001, 1, None)

    def parent(grid, levels, times):
        par[0].coarse = grid.handle.value
        for l, (lv, t) in enumerate(zip(levels, times)):
            par[0].levels[l] = lv
            par[0].times[l] = t
        par[0].ntimes = len(levels)

    lv = [1 << 36, (1 << 36) + (1 << 31), (1 << 36) + (1 << 32)]
    # spacing not in ratio 2
    parent(C.Grid((24, 24, 24), 3, 1 / 48, system=C.BSSN, boundary=C.BC_CALLER), lv,
           [0.0, 0.5, 1.0])
    assert step() == C.ERR_INVALID and "twice" in C.last_error()
    # a coarse block too small for the fine ghosts' stencils
    parent(C.Grid((8, 8, 8), 3, 1 / 32, system=C.BSSN, boundary=C.BC_CALLER), lv,
           [0.0, 0.5, 1.0])
    assert step() == C.ERR_INVALID and "outside the coarse extended range" in C.last_error()
    # a time level inside the patch's own state
    parent(coarse, [lv[0], arr[0].state, lv[2]], [0.0, 0.5, 1.0])
    assert step() == C.ERR_INVALID and "overlaps" in C.last_error()
    parent(coarse, lv, [0.0, 0.5, 0.5])
    assert step() == C.ERR_INVALID and "distinct" in C.last_error()
    # ghost zones wider than the batch's prolongation boxes allow
    wide = C.Grid((16, 16, 16), 6, 1 / 64, origin=(8 / 64, 8 / 64, 8 / 64), system=C.BSSN,
                  boundary=C.BC_GAUGEWAVE, slicing=C.SLICING_HARMONIC, shift=C.SHIFT_FROZEN)
    arr[0].grid = wide.handle.value
    parent(coarse, lv, [0.0, 0.5, 1.0])
    assert step() == C.ERR_UNSUPPORTED and "ghost width" in C.last_error()
    # parents in a 6th-order batch
    g6 = C.Grid((16, 16, 16), 4, 1 / 64, origin=(8 / 64, 8 / 64, 8 / 64), system=C.BSSN,
                boundary=C.BC_GAUGEWAVE, slicing=C.SLICING_HARMONIC, shift=C.SHIFT_FROZEN,
                fd_order=6, precision=C.MIXED)
    arr[0].grid = g6.handle.value
    assert step() == C.ERR_UNSUPPORTED and "fd_order 4" in C.last_error()
