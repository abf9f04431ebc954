"""GPU parity of Kreiss-Oliger dissipation and algebraic-constraint
enforcement (both off by default) against the oracle, through the C ABI:
right-hand side with dissipation, RK4 steps with dissipation and
enforcement (periodic and analytic ghosts, both gauges), the batched path,
FP64 (<= 1e-12 per grid function) and mixed (<= 1e-5)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1410_1764_amd import chemora as C
from paper_1410_1764_amd import inputs as I
from tests.helpers import pair, parity
from tests.test_oracle_bssn import _smooth_random

pytestmark = pytest.mark.gpu

GAUGES = {"1+log/Gamma-driver": dict(slicing=0, shift=1),
          "harmonic/frozen": dict(slicing=1, shift=0)}


@pytest.mark.parametrize("gauge", list(GAUGES))
@pytest.mark.parametrize("precision,tol", [(C.FP64, 1e-12), (C.MIXED, 1e-5)])
def test_rhs_with_dissipation(gauge, precision, tol):
    n = (37, 21, 19)
    h = tuple(1.0 / v for v in n)
    gr, b = pair(n, 3, h, C.BSSN, precision=precision, ko_sigma=0.3, **GAUGES[gauge])
    y0 = _smooth_random(n, 23)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    r = gr.rhs(st)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    e = parity(gr.download(r), b.interior(oracle.bssn_rhs(b, yo)))
    print("ko rhs", gauge, precision, e.max(), I.BSSN_NAMES[int(np.argmax(e))])
    assert e.max() <= tol


@pytest.mark.parametrize("bc", [C.BC_PERIODIC, C.BC_GAUGEWAVE])
@pytest.mark.parametrize("gauge", list(GAUGES))
@pytest.mark.parametrize("precision,tol", [(C.FP64, 1e-12), (C.MIXED, 1e-5)])
def test_rk4_with_dissipation_and_enforcement(bc, gauge, precision, tol):
    n = (26, 9, 7)
    h = (1 / 26, 1 / 26, 1 / 26)
    gr, b = pair(n, 3, h, C.BSSN, precision=precision, boundary=bc, gw_amp=0.1, gw_d=1.0,
                 gw_axis=0, ko_sigma=0.2, enforce=1, **GAUGES[gauge])
    y0 = I.gaugewave(n, h, axis=0) + (_smooth_random(n, 5) - I.minkowski(n))
    st = gr.upload(y0)
    ws = gr.new_workspace()
    dt = 0.25 / 26
    gr.rk4_step(st, ws, 0.0, dt, 3)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.rk4(b, oracle.BSSN, bc, yo, 0.0, dt, 3)
    got = gr.download(st)
    e = parity(got, b.interior(yo))
    print("ko+enforce rk4", bc, gauge, precision, e.max(), I.BSSN_NAMES[int(np.argmax(e))])
    assert e.max() <= tol
    # the returned state satisfies det gt = 1 (enforced in FP64 in both paths)
    g = np.empty(got.shape[1:] + (3, 3))
    for q, (i, j) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        g[..., i, j] = g[..., j, i] = got[1 + q]
    assert np.abs(np.linalg.det(g) - 1).max() <= 1e-13


@pytest.mark.parametrize("kind", ["0", "1"])
def test_batch_with_dissipation_and_enforcement(kind, monkeypatch):
    monkeypatch.setenv("CHEMORA_BATCH_KIND", kind)
    specs = [{"n": (24, 20, 17), "h": 1 / 64, "origin": (0.1, 0.2, 0.3)},
             {"n": (33, 24, 26), "h": 1 / 128, "origin": (0.5, 0.0, 0.7)}]
    rng = np.random.default_rng(8)
    grids, blocks, states, wss, y0s = [], [], [], [], []
    for sp in specs:
        kw = dict(slicing=C.SLICING_HARMONIC, shift=C.SHIFT_FROZEN, gw_amp=0.1,
                  gw_wavelength=1.0, gw_axis=0, ko_sigma=0.25, enforce=1)
        g = C.Grid(sp["n"], 3, sp["h"], origin=sp["origin"], system=C.BSSN, precision=C.FP64,
                   boundary=C.BC_GAUGEWAVE, **kw)
        b = oracle.Block(sp["n"], 3, sp["h"], sp["origin"], slicing=1, shift=0, gw_amp=0.1,
                         gw_d=1.0, gw_axis=0, ko_sigma=0.25, enforce=1)
        y0 = I.gaugewave(sp["n"], sp["h"], sp["origin"], 0.1, 1.0, 0, 0.0)
        y0 = y0 + (_smooth_random(sp["n"], int(rng.integers(1 << 30))) - I.minkowski(sp["n"]))
        grids.append(g)
        blocks.append(b)
        states.append(g.upload(y0))
        wss.append(g.new_workspace())
        y0s.append(y0)
    meta = torch.empty(C.batch_meta_bytes(len(grids)) // 8, dtype=torch.float64, device="cuda")
    dt = 0.25 / 128
    C.batch_step(grids, states, wss, meta, 0.0, dt, 2)
    torch.cuda.synchronize()
    C.batch_release(meta)
    for g, b, st, y0 in zip(grids, blocks, states, y0s):
        yo = b.embed(y0)
        oracle.rk4(b, oracle.BSSN, oracle.BC_GAUGEWAVE, yo, 0.0, dt, 2)
        e = parity(g.download(st), b.interior(yo))
        print("batch ko+enforce kind", kind, e.max(), I.BSSN_NAMES[int(np.argmax(e))])
        assert e.max() <= 1e-12
