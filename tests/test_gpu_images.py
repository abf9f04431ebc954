"""The write-through form of the periodic ghosts (CHEMORA_PERIODIC=images:
each substage kernel also stores every value at its periodic images in the
ghost zones, instead of a fill kernel after the substage) against the
default, through the C ABI.  Both copy the same interior values into the
same ghost points, so the states after RK4 steps, ghosts included, are
bitwise equal; the default itself is compared with the oracle elsewhere.
Ragged grids (partial tiles, odd plane counts), each system and precision."""
import numpy as np
import pytest
import torch

from paper_1410_1764_amd import chemora as C
from paper_1410_1764_amd import inputs as I
from tests.helpers import pair
from tests.test_oracle_bssn import _smooth_random

pytestmark = pytest.mark.gpu


def _steps(gr, y0, mode, monkeypatch, steps, dt):
    if mode:
        monkeypatch.setenv("CHEMORA_PERIODIC", mode)
    else:
        monkeypatch.delenv("CHEMORA_PERIODIC", raising=False)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    gr.rk4_step(st, gr.new_workspace(), 0.0, dt, steps)
    torch.cuda.synchronize()
    return gr.download(st, ghosts=True)


@pytest.mark.parametrize("system,nvar,n", [(C.WAVE, 2, (37, 21, 13)), (C.WAVE5, 5, (29, 18, 11))])
@pytest.mark.parametrize("precision", [C.FP64, C.MIXED])
def test_wave_images_bitwise(system, nvar, n, precision, monkeypatch):
    rng = np.random.default_rng(41)
    y0 = rng.standard_normal((nvar, n[2], n[1], n[0]))
    h = tuple(1.0 / v for v in n)
    gr, _ = pair(n, 2, h, system, precision=precision)
    dt = 0.25 * min(h)
    a = _steps(gr, y0, None, monkeypatch, 3, dt)
    b = _steps(gr, y0, "images", monkeypatch, 3, dt)
    print("images", system, precision, n, float(np.abs(a - b).max()), flush=True)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", [C.FP64, C.MIXED])
def test_bssn_images_bitwise(precision, monkeypatch):
    n = (37, 21, 13)
    h = tuple(1.0 / v for v in n)
    gr, _ = pair(n, 3, h, C.BSSN, precision=precision, slicing=0, shift=1)
    y0 = _smooth_random(n, 43)
    dt = 0.25 * min(h)
    a = _steps(gr, y0, None, monkeypatch, 2, dt)
    b = _steps(gr, y0, "images", monkeypatch, 2, dt)
    print("images bssn", precision, float(np.abs(a - b).max()), flush=True)
    assert np.array_equal(a, b)
