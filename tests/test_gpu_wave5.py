"""GPU parity of the first-order wave system (eq. (1) in the paper's own
five-variable form, Fig. 1 RHS) and of Fig. 1's Energy calculation against
the oracle, element by element, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_1410_1764_amd import chemora as C
from paper_1410_1764_amd import inputs as I
from tests.helpers import pair, parity
from tests.test_oracle_wave5 import fft_rk4_wave5

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [(24, 24, 24), (37, 29, 19), (70, 5, 3)])
def test_wave5_rhs_parity(n):
    rng = np.random.default_rng(31)
    y0 = rng.standard_normal((5, n[2], n[1], n[0]))
    h = tuple(1.0 / v for v in n)
    gr, b = pair(n, 2, h, C.WAVE5)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    r = gr.rhs(st)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    ro = b.interior(oracle.wave5_rhs(b, yo))
    e = parity(gr.download(r), ro)
    print(n, e)
    assert e.max() <= 1e-12


@pytest.mark.parametrize("precision,tol", [(C.FP64, 1e-12), (C.MIXED, 1e-5)])
def test_wave5_rk4_parity_and_closed_form(precision, tol):
    n, steps = 32, 10
    h = 1.0 / n
    dt = 0.25 * h
    y0 = I.wave5_fourier(n, 4, I.SEED0 + 5)
    gr, b = pair((n, n, n), 2, h, C.WAVE5, precision=precision)
    st = gr.upload(y0)
    gr.rk4_step(st, gr.new_workspace(), 0.0, dt, steps)
    torch.cuda.synchronize()
    yg = gr.download(st)
    yo = b.embed(y0)
    oracle.rk4(b, oracle.WAVE5, oracle.BC_PERIODIC, yo, 0.0, dt, steps)
    e = parity(yg, b.interior(yo))
    ef = parity(yg, fft_rk4_wave5(y0, h, dt, steps))
    print(precision, e.max(), ef.max())
    assert e.max() <= tol and ef.max() <= tol


def test_wave5_energy_parity_and_decay():
    """Fig. 1 Init (Gaussian rho) evolved on the GPU; the energy kernel
    matches the oracle's Energy calculation and decays monotonically"""
    n = 64
    h = 1.0 / n
    dt = 0.25 * h
    gr, b = pair((n, n, n), 2, h, C.WAVE5)
    y0 = I.gaussian_pulse(n, 1.0, 0.08)
    st = gr.upload(y0)
    ws = gr.new_workspace()
    eps = gr.new_state()[: gr.strides[3]].clone()
    es = []
    for _ in range(4):
        tot = gr.energy(st, eps=eps)
        torch.cuda.synchronize()
        es.append(float(tot.item()))
        yo = b.embed(gr.download(st))
        e_orc, eps_orc = oracle.wave5_energy(b, yo, want_field=True)
        assert abs(es[-1] - e_orc) <= 1e-12 * abs(e_orc)
        assert parity(gr.download(eps, nvars=1), b.interior(eps_orc)).max() <= 1e-15
        gr.rk4_step(st, ws, 0.0, dt, 5)
    assert all(es[i + 1] < es[i] for i in range(3)) and es[-1] > 0.999 * es[0], es
    # bitwise reproducible
    t1, t2 = gr.energy(st), gr.energy(st)
    torch.cuda.synchronize()
    assert torch.equal(t1, t2)
