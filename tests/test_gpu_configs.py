"""The two larger workloads as parity cases, at their full sizes:

* BSSN at 192^3 + 3 ghosts, gauge-wave data (A = 0.1), 1+log / Gamma-driver,
  periodic, 50 RK4 steps in mixed precision: one FP64 step against the
  oracle, then the mixed evolution against the FP64 one after all 50 steps
  (<= 1e-5 per grid function), with the FP64 constraint norms of both;
* 64 uneven patches (sizes 24..96 per axis, three refinement levels,
  analytic gauge-wave ghosts at every substage) advanced by the batched,
  graph-captured path with autotuned tiles, FP64 and mixed: every patch
  against an oracle run of that patch alone after 2 steps, then mixed
  against FP64 after 20 steps.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1410_1764_amd import chemora as C
from paper_1410_1764_amd import inputs as I
from tests.helpers import pair, parity
from tests.test_gpu_batch import _patches

pytestmark = pytest.mark.gpu


def test_bssn_192_mixed_50_steps():
    n = (192, 192, 192)
    h = (1 / 192,) * 3
    kw = dict(slicing=0, shift=1)
    g64, b = pair(n, 3, h, C.BSSN, precision=C.FP64, **kw)
    gmx = C.Grid(n, 3, h, system=C.BSSN, precision=C.MIXED, **kw)
    y0 = I.gaugewave(n, h, A=0.1, d=1.0, axis=0)
    dt = 0.25 / 192
    s64, smx = g64.upload(y0), gmx.upload(y0)
    ws = g64.new_workspace()
    # one FP64 step against the oracle
    g64.rk4_step(s64, ws, 0.0, dt, 1)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.rk4(b, oracle.BSSN, oracle.BC_PERIODIC, yo, 0.0, dt, 1)
    e = parity(g64.download(s64), b.interior(yo))
    print("c3 fp64 step 1 vs oracle", e.max(), I.BSSN_NAMES[int(np.argmax(e))], flush=True)
    assert e.max() <= 1e-12
    del yo
    # 50 steps: FP64 and mixed
    g64.rk4_step(s64, ws, dt, dt, 49)
    gmx.rk4_step(smx, ws, 0.0, dt, 50)
    torch.cuda.synchronize()
    e = parity(gmx.download(smx), g64.download(s64))
    print("c3 mixed vs fp64 after 50 steps, per grid function:",
          {I.BSSN_NAMES[v]: float(e[v]) for v in range(len(e))}, flush=True)
    assert e.max() <= 1e-5
    # FP64 constraint norms of both evolutions (the mixed state is FP64)
    g64.fill_ghosts(s64)
    gmx.fill_ghosts(smx)
    n64 = g64.constraints(s64).cpu().numpy()
    nmx = g64.constraints(smx).cpu().numpy()
    print("c3 constraint norms (H, M1, M2, M3): fp64", n64, "mixed", nmx, flush=True)
    assert np.all(np.isfinite(n64)) and np.all(np.isfinite(nmx))


def test_batch_64_patches_fp64_and_mixed():
    specs = [{"n": p["n"], "h": p["h"], "origin": p["origin"]}
             for p in I.patch_list(I.SEED0 + 4, 64, 24, 96)]
    dt = 0.25 * min(sp["h"] for sp in specs)
    runs = {}
    for prec in (C.FP64, C.MIXED):
        grids, blocks, states, wss, y0s = _patches(specs, prec, seed=4)
        meta = torch.empty(C.batch_meta_bytes(len(grids)) // 8, dtype=torch.float64,
                           device="cuda")
        C.autotune(grids, states, wss, meta, None)
        C.batch_step(grids, states, wss, meta, 0.0, dt, 2)
        torch.cuda.synchronize()
        runs[prec] = (grids, blocks, states, wss, y0s, meta)
        print("c4 precision", prec, "2 steps done", flush=True)
    # FP64 and mixed against the oracle after 2 steps, patch by patch
    grids, blocks, states, wss, y0s, meta = runs[C.FP64]
    gmx, _, smx, _, _, _ = runs[C.MIXED]
    worst64 = worstmx = 0.0
    for q in range(len(grids)):
        yo = blocks[q].embed(y0s[q])
        oracle.rk4(blocks[q], oracle.BSSN, oracle.BC_GAUGEWAVE, yo, 0.0, dt, 2)
        yi = blocks[q].interior(yo)
        worst64 = max(worst64, parity(grids[q].download(states[q]), yi).max())
        worstmx = max(worstmx, parity(gmx[q].download(smx[q]), yi).max())
    print("c4 after 2 steps vs oracle: fp64", worst64, "mixed", worstmx, flush=True)
    assert worst64 <= 1e-12
    assert worstmx <= 1e-5
    # 18 more steps each, then mixed against FP64
    for prec in (C.FP64, C.MIXED):
        g, _, s, w, _, m = runs[prec]
        C.batch_step(g, s, w, m, 2 * dt, dt, 18)
    torch.cuda.synchronize()
    worst = 0.0
    for q in range(len(grids)):
        e = parity(gmx[q].download(smx[q]), grids[q].download(states[q]))
        worst = max(worst, e.max())
    print("c4 mixed vs fp64 after 20 steps:", worst, flush=True)
    assert worst <= 1e-5
    for prec in (C.FP64, C.MIXED):
        C.batch_release(runs[prec][5])
