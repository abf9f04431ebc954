"""Pins behind the oracle references of the configured workloads.

The 192^3 gauge-wave workload depends on x alone.  Its oracle reference is
computed on a 192 x 4 x 4 periodic box with the same spacing on every axis
and repeated along y and z (tests/test_gpu_configs.py).  That is exact, not
an approximation: every point of the full box performs the same operations
on the same neighbour values as the matching point of the thin box, and the
differences across y and z are exactly zero.  Pinned here bit for bit on a
smaller cube, for both gauges and with dissipation.
"""
import numpy as np
import pytest

import oracle
from paper_1410_1764_amd import inputs as I


@pytest.mark.parametrize("slicing,shift,ko", [(0, 1, 0.0), (1, 0, 0.0), (0, 1, 0.3)])
def test_thin_box_evolution_equals_full_box(orc, slicing, shift, ko):
    n, steps = 20, 3
    h = (1.0 / n,) * 3
    outs = []
    for shape in ((n, n, n), (n, 4, 4)):
        b = oracle.Block(shape, 3, h, slicing=slicing, shift=shift, ko_sigma=ko)
        y = b.embed(I.gaugewave(shape, h, A=0.1, d=1.0, axis=0))
        oracle.rk4(b, oracle.BSSN, oracle.BC_PERIODIC, y, 0.0, 0.25 * h[0], steps)
        outs.append(b.interior(y))
    full, thin = outs
    assert np.array_equal(full, np.broadcast_to(thin[:, :1, :1, :], full.shape))
    # and the evolution did something in every non-frozen variable it drives
    y0 = I.gaugewave((n, 4, 4), h, A=0.1, d=1.0, axis=0)
    assert np.abs(thin[I.ALP] - y0[I.ALP]).max() > 1e-4
