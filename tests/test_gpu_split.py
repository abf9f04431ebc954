"""The z-blocked kernels of the BSSN right-hand side and RK4 substages (the
split curvature/rest pair, and in mixed precision the fused point code over
the same staging) against the oracle and against the single-plane fused
kernel, through the C ABI.

They run for 4th-order grids without dissipation and with 32 x 8 tiles
(x extent >= 24), two z-planes per workgroup; CHEMORA_BSSN_SPLIT=0|1|2
selects the single-plane kernel, the pair, or (mixed) the z-blocked fused
kernel.  Cases: ragged grids that leave partial tiles in x and y and an odd
number of planes (the last block's second plane idle), one wide enough for
the XCD column walk (some workgroups get no tile), both gauges, both
precisions, constraint enforcement, and RK4 steps, whose last substage keeps
the intermediates in a stage buffer instead of the output; the pair with
other tile heights (32 x 4 x 2 and 32 x 8 x 2 for either kernel)."""
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
TOL = {C.FP64: 1e-12, C.MIXED: 1e-5}


def _rhs(gr, st, split, monkeypatch):
    monkeypatch.setenv("CHEMORA_BSSN_SPLIT", str(int(split)))
    r = gr.rhs(st)
    torch.cuda.synchronize()
    return gr.download(r)


@pytest.mark.parametrize("n", [(37, 21, 13), (70, 40, 9)])
@pytest.mark.parametrize("gauge", list(GAUGES))
@pytest.mark.parametrize("precision,mode", [(C.FP64, 1), (C.MIXED, 1), (C.MIXED, 2)])
def test_split_rhs_matches_oracle_and_fused(n, gauge, precision, mode, monkeypatch):
    h = tuple(1.0 / v for v in n)
    gr, b = pair(n, 3, h, C.BSSN, precision=precision, **GAUGES[gauge])
    y0 = _smooth_random(n, 31)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    split = _rhs(gr, st, mode, monkeypatch)
    fused = _rhs(gr, st, 0, monkeypatch)
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    ro = b.interior(oracle.bssn_rhs(b, yo))
    e = parity(split, ro)
    ef = parity(split, fused)
    print("split", mode, n, gauge, precision, "vs oracle", e.max(), I.BSSN_NAMES[int(np.argmax(e))],
          "vs fused", ef.max(), flush=True)
    assert e.max() <= TOL[precision]
    # same arithmetic in the same order: equal up to contraction choices
    assert ef.max() <= (1e-13 if precision == C.FP64 else 1e-5)


@pytest.mark.parametrize("curv_ty,rest_ty", [("4", "8"), ("4", "4"), ("8", "4")])
@pytest.mark.parametrize("precision", [C.FP64, C.MIXED])
def test_split_tile_heights_bitwise(curv_ty, rest_ty, precision, monkeypatch):
    """The pair with other tile heights (CHEMORA_CURV_TY, CHEMORA_SPLIT_TY)
    evaluates every point with the same arithmetic: bitwise equal to the
    default tiles, and within the bar of the oracle."""
    n = (45, 27, 11)
    h = tuple(1.0 / v for v in n)
    gr, b = pair(n, 3, h, C.BSSN, precision=precision, **GAUGES["1+log/Gamma-driver"])
    y0 = _smooth_random(n, 37)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    monkeypatch.delenv("CHEMORA_CURV_TY", raising=False)
    monkeypatch.delenv("CHEMORA_SPLIT_TY", raising=False)
    default = _rhs(gr, st, 1, monkeypatch)
    monkeypatch.setenv("CHEMORA_CURV_TY", curv_ty)
    monkeypatch.setenv("CHEMORA_SPLIT_TY", rest_ty)
    other = _rhs(gr, st, 1, monkeypatch)
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    e = parity(other, b.interior(oracle.bssn_rhs(b, yo)))
    print("tile heights", curv_ty, rest_ty, precision, "vs oracle", e.max(), flush=True)
    assert np.array_equal(other, default)
    assert e.max() <= TOL[precision]


def test_split_rhs_minkowski_exactly_zero(monkeypatch):
    n = (40, 19, 7)
    gr, _ = pair(n, 3, tuple(1.0 / v for v in n), C.BSSN)
    st = gr.upload(I.minkowski(n))
    gr.fill_ghosts(st)
    assert np.count_nonzero(_rhs(gr, st, True, monkeypatch)) == 0


@pytest.mark.parametrize("bc", [C.BC_PERIODIC, C.BC_GAUGEWAVE])
@pytest.mark.parametrize("precision,mode", [(C.FP64, 1), (C.MIXED, 1), (C.MIXED, 2)])
def test_split_rk4_matches_oracle(bc, precision, mode, monkeypatch):
    """all four substages, including the last (output = state, the
    intermediates in the second stage buffer)"""
    monkeypatch.setenv("CHEMORA_BSSN_SPLIT", str(mode))
    n = (33, 10, 9)
    h = (1 / 33,) * 3
    kw = dict(slicing=0, shift=1)
    gr, b = pair(n, 3, h, C.BSSN, precision=precision, boundary=bc, gw_amp=0.1, gw_d=1.0,
                 gw_axis=0, **kw)
    y0 = I.gaugewave(n, h, axis=0) + (_smooth_random(n, 5) - I.minkowski(n))
    st = gr.upload(y0)
    gr.rk4_step(st, gr.new_workspace(), 0.0, 0.25 / 33, 3)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.rk4(b, oracle.BSSN, bc, yo, 0.0, 0.25 / 33, 3)
    e = parity(gr.download(st), b.interior(yo))
    print("split rk4", bc, precision, e.max(), I.BSSN_NAMES[int(np.argmax(e))], flush=True)
    assert e.max() <= TOL[precision]


def test_split_rk4_enforcement(monkeypatch):
    monkeypatch.setenv("CHEMORA_BSSN_SPLIT", "1")
    n = (29, 12, 7)
    h = (1 / 29,) * 3
    gr, b = pair(n, 3, h, C.BSSN, slicing=0, shift=1, enforce=1)
    y0 = _smooth_random(n, 13)
    st = gr.upload(y0)
    gr.rk4_step(st, gr.new_workspace(), 0.0, 0.25 / 29, 2)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.rk4(b, oracle.BSSN, oracle.BC_PERIODIC, yo, 0.0, 0.25 / 29, 2)
    e = parity(gr.download(st), b.interior(yo))
    print("split rk4 enforce", e.max(), I.BSSN_NAMES[int(np.argmax(e))], flush=True)
    assert e.max() <= 1e-12
