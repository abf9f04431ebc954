"""Degenerate block sizes through the default BSSN paths: one interior point,
one-point-wide axes, a single plane.  Every tile of every kernel is then
ragged in x, y and z (a 32 x 8 x 2 block holding one point, a z-blocked
workgroup whose second plane is idle), so the clamped staging, the idle
lanes and the store masks are all exercised.  Analytic gauge-wave ghosts
(periodic images need n >= ghost).  Right-hand side, RK4 steps and the
constraints, FP64 and mixed, against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1410_1764_amd import chemora as C
from paper_1410_1764_amd import inputs as I
from tests.helpers import pair, parity
from tests.test_oracle_bssn import _smooth_random

pytestmark = pytest.mark.gpu

SIZES = [(1, 1, 1), (2, 3, 1), (33, 1, 2), (1, 9, 5), (5, 1, 17)]
TOL = {C.FP64: 1e-12, C.MIXED: 1e-5}
KW = dict(slicing=0, shift=1, boundary=C.BC_GAUGEWAVE, gw_amp=0.1, gw_d=1.0, gw_axis=0)


def _state(n, h, seed):
    origin = (0.1, 0.2, 0.3)
    y0 = I.gaugewave(n, h, origin, 0.1, 1.0, 0) + (_smooth_random(n, seed) - I.minkowski(n))
    return origin, y0


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("precision", [C.FP64, C.MIXED])
def test_tiny_rhs_and_rk4(n, precision):
    h = (1 / 32, 1 / 40, 1 / 48)
    origin, y0 = _state(n, h, 7)
    gr, b = pair(n, 3, h, C.BSSN, origin=origin, precision=precision, **KW)
    st = gr.upload(y0)
    gr.fill_ghosts(st, 0.0)
    r = gr.rhs(st)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.fill_gaugewave(b, yo, 0.0)
    e = parity(gr.download(r), b.interior(oracle.bssn_rhs(b, yo)))
    print("rhs", n, precision, e.max(), I.BSSN_NAMES[int(np.argmax(e))], flush=True)
    assert e.max() <= TOL[precision]
    dt = 0.25 / 48
    gr.rk4_step(st, gr.new_workspace(), 0.0, dt, 2)
    torch.cuda.synchronize()
    oracle.rk4(b, oracle.BSSN, oracle.BC_GAUGEWAVE, yo, 0.0, dt, 2)
    e = parity(gr.download(st), b.interior(yo))
    print("rk4", n, precision, e.max(), I.BSSN_NAMES[int(np.argmax(e))], flush=True)
    assert e.max() <= TOL[precision]


@pytest.mark.parametrize("n", SIZES)
def test_tiny_constraints(n):
    h = (1 / 32, 1 / 40, 1 / 48)
    origin, y0 = _state(n, h, 9)
    gr, b = pair(n, 3, h, C.BSSN, origin=origin, **KW)
    st = gr.upload(y0)
    gr.fill_ghosts(st, 0.0)
    hm = gr.new_state()[: 4 * gr.strides[3]].clone()
    norms = gr.constraints(st, hm=hm)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.fill_gaugewave(b, yo, 0.0)
    hmo, no = oracle.constraints(b, yo)
    e = parity(gr.download(hm, nvars=4), b.interior(hmo))
    print("constraints", n, e.max(), norms.cpu().numpy(), no, flush=True)
    assert e.max() <= 1e-12
    assert np.allclose(norms.cpu().numpy(), no, rtol=1e-12, atol=0)
