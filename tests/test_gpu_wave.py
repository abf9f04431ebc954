"""GPU parity of the scalar-wave path (eq. (1), two-variable reading) against
the oracle, element by element, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_1410_1764_amd import chemora as C
from paper_1410_1764_amd import inputs as I
from tests.helpers import pair, parity
from tests.test_oracle_wave import fft_rk4, _laplacian_symbol

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12
TOL_MIXED = 1e-5


def _rhs_both(n, h, y0, precision):
    gr, b = pair(n, 2, h, C.WAVE, precision=precision)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    r = gr.rhs(st)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    ro = b.interior(oracle.wave_rhs(b, yo))
    return gr.download(r), ro, gr, st, b, yo


@pytest.mark.parametrize("n", [(32, 32, 32), (37, 29, 19), (70, 5, 3), (2, 2, 2)])
def test_wave_rhs_parity_fp64(n):
    rng = np.random.default_rng(11)
    y0 = rng.standard_normal((2, n[2], n[1], n[0]))
    h = tuple(1.0 / v for v in n)
    rg, ro, *_ = _rhs_both(n, h, y0, C.FP64)
    e = parity(rg, ro)
    print(n, e)
    assert e.max() <= TOL_FP64
    assert np.array_equal(rg[0], ro[0])  # du/dt = rho is a copy


def test_periodic_ghosts_bitwise():
    n = (37, 29, 19)
    rng = np.random.default_rng(12)
    y0 = rng.standard_normal((2, n[2], n[1], n[0]))
    _, _, gr, st, b, yo = _rhs_both(n, 1.0 / 37, y0, C.FP64)
    assert np.array_equal(gr.download(st, ghosts=True), yo)


def test_wave_rhs_mixed_error():
    n = 64
    y0 = I.fourier_modes(n, 16, I.SEED0 + 1)
    y0[1] = I.fourier_modes(n, 16, 5)[0]
    rg, ro, *_ = _rhs_both((n, n, n), 1.0 / n, y0, C.MIXED)
    e = parity(rg, ro)
    print("mixed rhs", e)
    assert e.max() <= TOL_MIXED


def _rk4_both(n, K, steps, precision, seed):
    h = 1.0 / n
    dt = 0.25 * h
    y0 = I.fourier_modes(n, K, seed)
    gr, b = pair((n, n, n), 2, h, C.WAVE, precision=precision)
    st = gr.upload(y0)
    ws = gr.new_workspace()
    gr.rk4_step(st, ws, 0.0, dt, steps)
    torch.cuda.synchronize()
    return y0, gr.download(st), gr, st, b, h, dt


def test_wave_rk4_parity_c0():
    """32^3 + 2 ghosts, |k| <= 4, dt = 0.25 h, 10 RK4 steps (FP64)"""
    y0, yg, gr, st, b, h, dt = _rk4_both(32, 4, 10, C.FP64, I.SEED0 + 0)
    yo = b.embed(y0)
    oracle.rk4(b, oracle.WAVE, oracle.BC_PERIODIC, yo, 0.0, dt, 10)
    e = parity(yg, b.interior(yo))
    print("rk4 c0 vs oracle", e)
    assert e.max() <= TOL_FP64
    # ghosts are periodic images on return
    assert np.array_equal(gr.download(st, ghosts=True)[:, :2], gr.download(st, ghosts=True)[:, 32:34])


def test_wave_rk4_mixed_c0():
    y0, yg, gr, st, b, h, dt = _rk4_both(32, 4, 10, C.MIXED, I.SEED0 + 0)
    yo = b.embed(y0)
    oracle.rk4(b, oracle.WAVE, oracle.BC_PERIODIC, yo, 0.0, dt, 10)
    e = parity(yg, b.interior(yo))
    print("rk4 c0 mixed vs oracle", e)
    assert e.max() <= TOL_MIXED


def _fft_power(y0, h, dt, steps):
    """closed-form RK4 over many steps: per-mode 2x2 amplification matrix to
    the power `steps` by repeated squaring"""
    n = y0.shape[1]
    lam = _laplacian_symbol(n, h)
    z = dt * dt * lam
    P = 1 + z / 2 + z * z / 24
    Q = 1 + z / 6
    A = [[P, Q * dt], [Q * dt * lam, P]]
    R = [[np.ones_like(P), np.zeros_like(P)], [np.zeros_like(P), np.ones_like(P)]]

    def mul(X, Y):
        return [[X[0][0] * Y[0][0] + X[0][1] * Y[1][0], X[0][0] * Y[0][1] + X[0][1] * Y[1][1]],
                [X[1][0] * Y[0][0] + X[1][1] * Y[1][0], X[1][0] * Y[0][1] + X[1][1] * Y[1][1]]]
    k = steps
    while k:
        if k & 1:
            R = mul(R, A)
        A = mul(A, A)
        k >>= 1
    U, Rh = np.fft.fftn(y0[0]), np.fft.fftn(y0[1])
    return (np.real(np.fft.ifftn(R[0][0] * U + R[0][1] * Rh)),
            np.real(np.fft.ifftn(R[1][0] * U + R[1][1] * Rh)))


@pytest.mark.parametrize("precision,tol", [(C.FP64, TOL_FP64), (C.MIXED, TOL_MIXED)])
def test_wave_c1_full_size(precision, tol):
    """256^3 + 2 ghosts, |k| <= 16, 100 RK4 steps, against the fully-discrete
    closed form (exact to rounding: the oracle reproduces it to ~1e-14 at
    32^3), plus one step against the oracle itself."""
    n, K, steps = 256, 16, 100
    y0, yg, gr, st, b, h, dt = _rk4_both(n, K, steps, precision, I.SEED0 + 1)
    ue, re = _fft_power(y0, h, dt, steps)
    e = parity(yg, np.stack([ue, re]))
    print("c1", precision, "vs closed form", e)
    assert e.max() <= tol
    if precision == C.FP64:
        st1 = gr.upload(y0)
        gr.rk4_step(st1, gr.new_workspace(), 0.0, dt, 1)
        torch.cuda.synchronize()
        yo = b.embed(y0)
        oracle.rk4(b, oracle.WAVE, oracle.BC_PERIODIC, yo, 0.0, dt, 1)
        e1 = parity(gr.download(st1), b.interior(yo))
        print("c1 one step vs oracle", e1)
        assert e1.max() <= TOL_FP64
