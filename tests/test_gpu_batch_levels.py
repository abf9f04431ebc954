"""Batches with refined patches (Sec. IV: a refined patch's ghost zones come
from the next coarser level): the ghosts of such a patch's state and of every
RK stage output are prolongated inside the batch's persistent launch, one
ghost item per box of its ghost shell, from three time levels of a coarse
parent, at the stage's time.  Each patch against the oracle's RK4 with the
same prolongated ghosts (orc_rk4_prolong), interior and ghosts; patches with
analytic ghosts in the same batch against the oracle's analytic RK4; both
precisions, the 4th-order kernel kinds, plan reuse and graph replays
across calls; argument checks."""
import numpy as np
import pytest
import torch

import oracle
from paper_1410_1764_amd import chemora as C
from paper_1410_1764_amd import inputs as I
from tests.helpers import parity
from tests.test_oracle_bssn import _smooth_random

pytestmark = pytest.mark.gpu

HC = 1 / 48                       # coarse spacing
NC = (24, 20, 20)                 # coarse interior
OC = (0.05, 0.1, 0.15)            # coarse origin
FINE = [((20, 14, 12), (5, 6, 7)),    # (interior, offset in fine spacings): odd offsets
        ((16, 16, 10), (10, 4, 8))]   # start half-way between coarse points
KW = dict(slicing=C.SLICING_HARMONIC, shift=C.SHIFT_FROZEN, gw_amp=0.1, gw_wavelength=1.0,
          gw_axis=0)
BKW = dict(slicing=1, shift=0, gw_amp=0.1, gw_d=1.0, gw_axis=0)


def _coarse_levels(times, seed):
    """the coarse parent: gauge wave plus a smooth perturbation, every point,
    at each of the three times (the perturbation drifts linearly in time)"""
    cb = oracle.Block(NC, 3, HC, OC, **BKW)
    gc = C.Grid(NC, 3, HC, origin=OC, system=C.BSSN, boundary=C.BC_CALLER, **KW)
    pert = cb.embed(_smooth_random(NC, seed) - I.minkowski(NC))
    levels = []
    for t in times:
        y = cb.embed(I.gaugewave(NC, HC, OC, 0.1, 1.0, 0, t))
        oracle.fill_gaugewave(cb, y, t)
        y = y + (1.0 + 3.0 * t) * pert
        levels.append(y)
    return cb, gc, levels


def _setup(precision, seed=5):
    t0, dtc = 0.2, 0.25 * HC
    times = [t0 - dtc, t0, t0 + dtc]
    cb, gc, levels = _coarse_levels(times, seed)
    dlev = [gc.upload_full(y) for y in levels]
    rng = np.random.default_rng(seed)
    grids, blocks, states, wss, y0s, parents = [], [], [], [], [], []
    hf = HC / 2
    for n, off in FINE:
        origin = tuple(OC[d] + off[d] * hf for d in range(3))
        g = C.Grid(n, 3, hf, origin=origin, system=C.BSSN, precision=precision,
                   boundary=C.BC_GAUGEWAVE, **KW)
        b = oracle.Block(n, 3, hf, origin, **BKW)
        y0 = I.gaugewave(n, hf, origin, 0.1, 1.0, 0, t0) + (
            _smooth_random(n, int(rng.integers(1 << 30))) - I.minkowski(n))
        grids.append(g), blocks.append(b), states.append(g.upload(y0))
        wss.append(g.new_workspace()), y0s.append(y0)
        parents.append((gc, dlev, times))
    # a patch with analytic ghosts in the same batch
    n, h, origin = (21, 17, 13), 1 / 64, (0.3, 0.2, 0.1)
    g = C.Grid(n, 3, h, origin=origin, system=C.BSSN, precision=precision,
               boundary=C.BC_GAUGEWAVE, **KW)
    b = oracle.Block(n, 3, h, origin, **BKW)
    y0 = I.gaugewave(n, h, origin, 0.1, 1.0, 0, t0) + (
        _smooth_random(n, int(rng.integers(1 << 30))) - I.minkowski(n))
    grids.append(g), blocks.append(b), states.append(g.upload(y0))
    wss.append(g.new_workspace()), y0s.append(y0)
    parents.append(None)
    return dict(t0=t0, dtc=dtc, times=times, cb=cb, gc=gc, levels=levels, dlev=dlev,
                grids=grids, blocks=blocks, states=states, wss=wss, y0s=y0s, parents=parents)


def _check(S, nsteps, dt, tol, label):
    for q, (g, b, st, y0, par) in enumerate(zip(S["grids"], S["blocks"], S["states"], S["y0s"],
                                               S["parents"])):
        yo = b.embed(y0)
        if par is None:
            oracle.rk4(b, oracle.BSSN, oracle.BC_GAUGEWAVE, yo, S["t0"], dt, nsteps)
        else:
            oracle.rk4_prolong(b, oracle.BSSN, yo, S["t0"], dt, nsteps, S["cb"], S["levels"],
                               S["times"])
        got = g.download(st, ghosts=True)
        e = parity(g.download(st), b.interior(yo))
        m = np.ones(b.ext, dtype=bool)
        m[3:-3, 3:-3, 3:-3] = False
        eg = float(np.abs(got[:, m] - yo[:, m]).max() / np.abs(yo[:, m]).max())
        print(label, "patch", q, "parent" if par else "analytic", "interior", e.max(),
              I.BSSN_NAMES[int(np.argmax(e))], "ghosts", eg, flush=True)
        assert e.max() <= tol
        assert eg <= max(tol, 1e-14)


@pytest.mark.parametrize("kind", ["0", "1", "2", "3"])
@pytest.mark.parametrize("precision,tol", [(C.FP64, 1e-12), (C.MIXED, 1e-5)])
def test_batch_with_parents_matches_oracle(kind, precision, tol, monkeypatch):
    monkeypatch.setenv("CHEMORA_BATCH_KIND", kind)
    S = _setup(precision)
    meta = torch.empty(C.batch_meta_bytes(len(S["grids"])) // 8, dtype=torch.float64,
                       device="cuda")
    dt = S["dtc"] / 2
    # two calls of one step each: the plan and its graph are reused
    C.batch_step(S["grids"], S["states"], S["wss"], meta, S["t0"], dt, 1, parents=S["parents"])
    C.batch_step(S["grids"], S["states"], S["wss"], meta, S["t0"] + dt, dt, 1,
                 parents=S["parents"])
    torch.cuda.synchronize()
    _check(S, 2, dt, tol, f"kind {kind}")
    C.batch_release(meta)


def test_batch_parent_levels_are_read_only_and_times_matter():
    """the coarse levels are left alone; shifting the level times changes the
    prolongated ghosts (a new plan is built for them)"""
    S = _setup(C.FP64, seed=9)
    before = [lv.clone() for lv in S["dlev"]]
    meta = torch.empty(C.batch_meta_bytes(len(S["grids"])) // 8, dtype=torch.float64,
                       device="cuda")
    dt = S["dtc"] / 2
    C.batch_step(S["grids"], S["states"], S["wss"], meta, S["t0"], dt, 1, parents=S["parents"])
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(before, S["dlev"]))
    g0 = S["grids"][0].download(S["states"][0], ghosts=True)
    shifted = [(p[0], p[1], [t + 0.5 * S["dtc"] for t in p[2]]) if p else None
               for p in S["parents"]]
    st = S["grids"][0].upload(S["y0s"][0])
    states = [st] + S["states"][1:]
    C.batch_step(S["grids"], states, S["wss"], meta, S["t0"], dt, 1, parents=shifted)
    torch.cuda.synchronize()
    g1 = S["grids"][0].download(st, ghosts=True)
    assert np.abs(g1 - g0).max() > 1e-8
    C.batch_release(meta)


def test_batch_parent_argument_checks():
    S = _setup(C.FP64, seed=11)
    meta = torch.empty(C.batch_meta_bytes(len(S["grids"])) // 8, dtype=torch.float64,
                       device="cuda")
    gc, dlev, times = S["parents"][0]
    bad = [
        # a time level that is a patch's own state: the batch writes it
        ((gc, [S["states"][1], dlev[1], dlev[2]], times), C.ERR_INVALID),
        ((gc, dlev, [0.0, 0.0, 1.0]), C.ERR_INVALID),  # times not distinct
    ]
    for par, status in bad:
        parents = [par] + S["parents"][1:]
        with pytest.raises(C.ChemoraError) as e:
            C.batch_step(S["grids"], S["states"], S["wss"], meta, S["t0"], 0.001, 1,
                         parents=parents)
        assert e.value.status == status
    # a parent whose extended block does not reach the patch's ghost stencils
    small = C.Grid((8, 8, 8), 3, HC, origin=OC, system=C.BSSN, boundary=C.BC_CALLER, **KW)
    sm = [small.new_state() for _ in range(3)]
    with pytest.raises(C.ChemoraError) as e:
        C.batch_step(S["grids"], S["states"], S["wss"], meta, S["t0"], 0.001, 1,
                     parents=[(small, sm, times)] + S["parents"][1:])
    assert e.value.status == C.ERR_INVALID
