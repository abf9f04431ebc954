"""GPU parity of the 6th- and 8th-order finite differences (grid description
fd_order; LDS-staged high-order kernels) against the oracle through the C
ABI: right-hand side (ragged 32 x 8 and 16 x 16 tiles, the XCD column walk,
and the full 128^3 size), RK4 steps (periodic and analytic ghosts),
constraints, FP64 (<= 1e-12 per grid function) and mixed (<= 1e-5)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1410_1764_amd import chemora as C
from paper_1410_1764_amd import inputs as I
from tests.helpers import pair, parity
from tests.test_oracle_bssn import _smooth_random

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("order", [6, 8])
@pytest.mark.parametrize("gauge", [dict(slicing=0, shift=1), dict(slicing=1, shift=0)])
@pytest.mark.parametrize("precision,tol", [(C.FP64, 1e-12), (C.MIXED, 1e-5)])
@pytest.mark.parametrize("n,extra", [((37, 22, 19), 0), ((20, 18, 11), 1)])
def test_rhs_high_order(order, gauge, precision, tol, n, extra):
    """32 x 8 tiles (n_x >= 24) and 16 x 16 tiles, both ragged; the second
    shape with one ghost more than the order needs"""
    h = tuple(1.0 / v for v in n)
    gr, b = pair(n, order // 2 + 1 + extra, h, C.BSSN, precision=precision, fd_order=order,
                 **gauge)
    y0 = _smooth_random(n, 31)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    r = gr.rhs(st)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    e = parity(gr.download(r), b.interior(oracle.bssn_rhs(b, yo)))
    print("rhs order", order, n, gauge, precision, e.max(), I.BSSN_NAMES[int(np.argmax(e))],
          flush=True)
    assert e.max() <= tol


@pytest.mark.parametrize("order", [6, 8])
@pytest.mark.parametrize("bc", [C.BC_PERIODIC, C.BC_GAUGEWAVE])
def test_rk4_high_order(order, bc):
    n = (26, 10, 9)
    h = (1 / 26, 1 / 26, 1 / 26)
    gr, b = pair(n, order // 2 + 1, h, C.BSSN, boundary=bc, gw_amp=0.1, gw_d=1.0, gw_axis=0,
                 fd_order=order, slicing=1, shift=0)
    y0 = I.gaugewave(n, h, axis=0) + (_smooth_random(n, 6) - I.minkowski(n))
    st = gr.upload(y0)
    ws = gr.new_workspace()
    dt = 0.25 / 26
    gr.rk4_step(st, ws, 0.0, dt, 2)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.rk4(b, oracle.BSSN, bc, yo, 0.0, dt, 2)
    e = parity(gr.download(st), b.interior(yo))
    print("rk4 order", order, bc, e.max(), I.BSSN_NAMES[int(np.argmax(e))])
    assert e.max() <= 1e-12


@pytest.mark.parametrize("order", [6, 8])
@pytest.mark.parametrize("n", [(30, 17, 12), (20, 18, 11)])
def test_constraints_high_order(order, n):
    """staged 32 x 8 (n_x >= 24) and 16 x 16 tiles, both ragged"""
    h = tuple(1.0 / v for v in n)
    gr, b = pair(n, order // 2 + 1, h, C.BSSN, fd_order=order)
    y0 = _smooth_random(n, 12)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    hm = gr.new_state()[: 4 * gr.strides[3]].clone()
    norms = gr.constraints(st, hm=hm)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    hmo, no = oracle.constraints(b, yo)
    e = parity(gr.download(hm, nvars=4), b.interior(hmo))
    print("constraints order", order, n, e, norms.cpu().numpy(), no, flush=True)
    assert e.max() <= 1e-12
    assert np.allclose(norms.cpu().numpy(), no, rtol=1e-12, atol=0)


@pytest.mark.parametrize("order", [6, 8])
@pytest.mark.parametrize("precision,tol", [(C.FP64, 1e-12), (C.MIXED, 1e-5)])
def test_rhs_high_order_column_walk(order, precision, tol):
    """32 x 8 tiles in uneven XCD columns (some workgroups get no tile): the
    tile order the full-size launches take"""
    n = (70, 40, 9)
    h = tuple(1.0 / v for v in n)
    gr, b = pair(n, order // 2 + 1, h, C.BSSN, precision=precision, fd_order=order)
    y0 = _smooth_random(n, 41)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    r = gr.rhs(st)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    e = parity(gr.download(r), b.interior(oracle.bssn_rhs(b, yo)))
    print("rhs column walk order", order, precision, e.max(), flush=True)
    assert e.max() <= tol


@pytest.mark.parametrize("order", [6, 8])
def test_constraints_high_order_column_walk(order):
    n = (70, 40, 9)
    h = tuple(1.0 / v for v in n)
    gr, b = pair(n, order // 2 + 1, h, C.BSSN, fd_order=order)
    y0 = _smooth_random(n, 42)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    hm = gr.new_state()[: 4 * gr.strides[3]].clone()
    norms = gr.constraints(st, hm=hm)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    hmo, no = oracle.constraints(b, yo)
    e = parity(gr.download(hm, nvars=4), b.interior(hmo))
    assert e.max() <= 1e-12
    assert np.allclose(norms.cpu().numpy(), no, rtol=1e-12, atol=0)


@pytest.mark.parametrize("order", [6, 8])
def test_rhs_high_order_full_size_128(order):
    """128^3, the size bench.py times at orders 6 and 8 (1+log /
    Gamma-driver, gauge wave plus smooth perturbations), FP64 and mixed"""
    n = (128, 128, 128)
    h = (1 / 128,) * 3
    y0 = I.gaugewave(n, h, axis=0) + 0.2 * (_smooth_random(n, 43) - I.minkowski(n))
    b = oracle.Block(n, order // 2 + 1, h, slicing=0, shift=1, fd_order=order)
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    ro = b.interior(oracle.bssn_rhs(b, yo))
    del yo
    for precision, tol in ((C.FP64, 1e-12), (C.MIXED, 1e-5)):
        gr = C.Grid(n, order // 2 + 1, h, system=C.BSSN, precision=precision, fd_order=order)
        st = gr.upload(y0)
        gr.fill_ghosts(st)
        r = gr.rhs(st)
        torch.cuda.synchronize()
        e = parity(gr.download(r), ro)
        print("rhs 128^3 order", order, precision, e.max(), I.BSSN_NAMES[int(np.argmax(e))],
              flush=True)
        assert e.max() <= tol
        del gr, st, r
