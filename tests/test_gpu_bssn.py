"""GPU parity of the BSSN path against the oracle, element by element,
through the C ABI: right-hand side, ghost fills, RK4 steps and constraints,
FP64 (<= 1e-12 per grid function, max-normalised) and mixed (<= 1e-5)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1410_1764_amd import chemora as C
from paper_1410_1764_amd import inputs as I
from tests.helpers import pair, parity
from tests.test_oracle_bssn import _smooth_random

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12
TOL_MIXED = 1e-5

GAUGES = {"1+log/Gamma-driver": dict(slicing=0, shift=1),
          "harmonic/frozen": dict(slicing=1, shift=0)}


def _data(kind, n, h, axis=0):
    if kind == "minkowski":
        return I.minkowski(n)
    if kind == "noise":
        return I.minkowski(n, noise=1e-10, seed=I.SEED0 + 2)
    if kind == "smooth":
        return _smooth_random(n, 21)
    if kind == "gaugewave":
        return I.gaugewave(n, h, axis=axis)
    if kind == "oblique":
        return I.gaugewave_oblique(n, (1, -1, 1))
    raise ValueError(kind)


def _rhs_pair(n, kind, gauge, precision=C.FP64, axis=0):
    h = tuple(1.0 / v for v in n)
    gr, b = pair(n, 3, h, C.BSSN, precision=precision, **GAUGES[gauge])
    y0 = _data(kind, n, h, axis)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    r = gr.rhs(st)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    ro = b.interior(oracle.bssn_rhs(b, yo))
    return gr.download(r), ro


@pytest.mark.parametrize("gauge", list(GAUGES))
@pytest.mark.parametrize("kind", ["noise", "smooth", "gaugewave", "oblique"])
def test_bssn_rhs_parity_small(kind, gauge):
    n = (21, 17, 13) if kind not in ("gaugewave", "oblique") else (24, 24, 24)
    rg, ro = _rhs_pair(n, kind, gauge)
    e = parity(rg, ro)
    print(kind, gauge, e.max(), I.BSSN_NAMES[int(np.argmax(e))])
    assert e.max() <= TOL_FP64


@pytest.mark.parametrize("axis", [1, 2])
def test_bssn_rhs_parity_gaugewave_axes(axis):
    n = [6, 6, 6]
    n[axis] = 40
    h = tuple(1.0 / v for v in n)
    rg, ro = _rhs_pair(tuple(n), "gaugewave", "harmonic/frozen", axis=axis)
    e = parity(rg, ro)
    assert e.max() <= TOL_FP64


@pytest.mark.parametrize("precision", [C.FP64, C.MIXED])
def test_bssn_minkowski_rhs_exactly_zero(precision):
    rg, ro = _rhs_pair((19, 11, 9), "minkowski", "1+log/Gamma-driver", precision)
    assert np.count_nonzero(ro) == 0
    assert np.count_nonzero(rg) == 0


@pytest.mark.parametrize("kind", ["smooth", "gaugewave", "oblique"])
def test_bssn_rhs_mixed_error(kind):
    n = (24, 24, 24)
    rg, ro = _rhs_pair(n, kind, "1+log/Gamma-driver", C.MIXED)
    e = parity(rg, ro)
    print("mixed", kind, e.max(), I.BSSN_NAMES[int(np.argmax(e))])
    assert e.max() <= TOL_MIXED


@pytest.mark.parametrize("kind", ["noise", "gaugewave"])
def test_bssn_rhs_parity_full_size_128(kind):
    """128^3 + 3 ghosts, 1+log / Gamma-driver: the metric's workload"""
    n = (128, 128, 128)
    rg, ro = _rhs_pair(n, kind, "1+log/Gamma-driver")
    e = parity(rg, ro)
    print("128^3", kind, e.max(), I.BSSN_NAMES[int(np.argmax(e))])
    assert e.max() <= TOL_FP64


def test_gaugewave_ghost_fill_parity():
    n = (20, 9, 7)
    h = (1 / 20, 0.05, 0.07)
    gr, b = pair(n, 3, h, C.BSSN, origin=(0.3, -0.2, 0.1), boundary=C.BC_GAUGEWAVE,
                 gw_amp=0.1, gw_d=1.0, gw_axis=0, slicing=1, shift=0)
    st = gr.new_state()
    gr.fill_ghosts(st, 0.37)
    torch.cuda.synchronize()
    yo = b.zeros(24)
    oracle.fill_gaugewave(b, yo, 0.37)
    got = gr.download(st, ghosts=True)
    assert np.abs(got - yo).max() < 1e-14
    assert np.count_nonzero(b.interior(got)) == 0


@pytest.mark.parametrize("bc", [C.BC_PERIODIC, C.BC_GAUGEWAVE])
@pytest.mark.parametrize("gauge", list(GAUGES))
def test_bssn_rk4_parity(bc, gauge):
    n = (26, 7, 5)
    h = (1 / 26, 1 / 26, 1 / 26)
    kw = dict(GAUGES[gauge])
    gr, b = pair(n, 3, h, C.BSSN, boundary=bc, gw_amp=0.1, gw_d=1.0, gw_axis=0, **kw)
    # gauge wave plus a smooth 3-D perturbation of a few percent, so that
    # every component (off-diagonals included) is of the size of the terms
    # that feed it: a component that is zero but for ~1e-10 boundary
    # mismatches, or tiny against its own right-hand-side terms, measures
    # cancellation, not parity
    y0 = I.gaugewave(n, h, axis=0) + (_smooth_random(n, 5) - I.minkowski(n))
    st = gr.upload(y0)
    ws = gr.new_workspace()
    dt = 0.25 / 26
    gr.rk4_step(st, ws, 0.0, dt, 4)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.rk4(b, oracle.BSSN, bc, yo, 0.0, dt, 4)
    e = parity(gr.download(st), b.interior(yo))
    print("rk4", bc, gauge, e.max(), I.BSSN_NAMES[int(np.argmax(e))])
    assert e.max() <= TOL_FP64
    # ghosts on return are valid (periodic images / analytic at t + 4 dt)
    eg = np.abs(gr.download(st, ghosts=True) - yo).max() / np.abs(yo).max()
    assert eg <= TOL_FP64


@pytest.mark.parametrize("n", [(22, 18, 14), (37, 21, 13), (70, 40, 9)])
def test_constraints_parity(n):
    # 16 x 16 tiles; 32 x 8 tiles without a column split; 32 x 8 tiles in
    # uneven XCD columns (some workgroups get no tile)
    h = tuple(1.0 / v for v in n)
    gr, b = pair(n, 3, h, C.BSSN)
    y0 = _smooth_random(n, 9)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    hm = gr.new_state()[: 4 * gr.strides[3]].clone()
    norms = gr.constraints(st, hm=hm)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    hmo, no = oracle.constraints(b, yo)
    e = parity(gr.download(hm, nvars=4), b.interior(hmo))
    print("constraints", e, norms.cpu().numpy(), no)
    assert e.max() <= TOL_FP64
    assert np.allclose(norms.cpu().numpy(), no, rtol=1e-12, atol=0)
    # deterministic: a second evaluation is bitwise identical
    norms2 = gr.constraints(st)
    torch.cuda.synchronize()
    assert torch.equal(norms, norms2)
