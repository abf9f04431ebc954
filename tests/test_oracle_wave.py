"""Pins for the oracle's scalar-wave path: eq. (1) in the two-variable reading
(du/dt = rho, drho/dt = Laplacian u), 4th-order centred differences,
periodic ghosts, classical RK4 (Sec. II time integrator).

  * fully-discrete closed form: per Fourier mode the semi-discrete system is
    d/dt (u, rho) = [[0, 1], [lam, 0]] (u, rho) with lam the (negative)
    symbol of the discrete Laplacian; one RK4 step multiplies by
    P I + Q dt M with z = dt^2 lam, P = 1 + z/2 + z^2/24, Q = 1 + z/6
    (M^2 = lam I).  An FFT evaluation of that is exact to rounding.
  * convergence to the exact continuum travelling wave at 4th order;
  * the discrete energy per mode decays each step by exactly
    P^2 - Q^2 z (monotone decay for 0 < -z < 8).
"""
import numpy as np
import pytest

import oracle
from paper_1410_1764_amd import inputs


def _laplacian_symbol(n, h):
    k = np.fft.fftfreq(n, d=1.0 / n)  # integer wavenumbers
    th = 2 * np.pi * k * h
    s = (30 - 32 * np.cos(th) + 2 * np.cos(2 * th)) / 12.0
    S = s[:, None, None] + s[None, :, None] + s[None, None, :]
    return -S / h ** 2


def fft_rk4(u0, rho0, h, dt, nsteps):
    n = u0.shape[0]
    lam = _laplacian_symbol(n, h)
    z = dt * dt * lam
    P = 1 + z / 2 + z * z / 24
    Q = 1 + z / 6
    U, R = np.fft.fftn(u0), np.fft.fftn(rho0)
    for _ in range(nsteps):
        U, R = P * U + Q * dt * R, Q * dt * lam * U + P * R
    return np.real(np.fft.ifftn(U)), np.real(np.fft.ifftn(R))


def test_wave_rk4_matches_fully_discrete_closed_form_c0(orc):
    """32^3 interior + 2 ghosts, |k| <= 4 Fourier data, dt = 0.25 h, 10 steps."""
    n, K, steps = 32, 4, 10
    h = 1.0 / n
    dt = 0.25 * h
    y0 = inputs.fourier_modes(n, K, inputs.SEED0 + 0)
    b = oracle.Block((n, n, n), 2, h)
    y = b.embed(y0)
    oracle.rk4(b, oracle.WAVE, oracle.BC_PERIODIC, y, 0.0, dt, steps)
    ue, re = fft_rk4(y0[0], y0[1], h, dt, steps)
    for got, exp in ((b.interior(y[0]), ue), (b.interior(y[1]), re)):
        err = np.abs(got - exp).max() / np.abs(exp).max()
        assert err < 1e-12, err


def test_wave_rhs_matches_symbol(orc):
    """drho/dt = FFT^-1(lam FFT(u)) exactly for periodic data"""
    n, h = 24, 1.0 / 24
    y0 = inputs.fourier_modes(n, 5, 99)
    y0[1] = np.random.default_rng(5).standard_normal((n, n, n))
    b = oracle.Block((n, n, n), 2, h)
    y = b.embed(y0)
    oracle.fill_periodic(b, y)
    r = oracle.wave_rhs(b, y)
    lap = np.real(np.fft.ifftn(_laplacian_symbol(n, h) * np.fft.fftn(y0[0])))
    assert np.array_equal(b.interior(r[0]), y0[1])
    assert np.abs(b.interior(r[1]) - lap).max() / np.abs(lap).max() < 1e-12


@pytest.mark.parametrize("kvec", [(1, 0, 0), (1, 2, 0)])
def test_wave_converges_at_fourth_order(orc, kvec):
    T = 0.25
    errs = []
    for n in (32, 64, 128):
        h = 1.0 / n
        dt = 0.25 * h
        steps = int(round(T / dt))
        nz = 4  # data independent of z: a thin periodic box is exact
        b = oracle.Block((n, n if kvec[1] else 4, nz), 2, h)
        nn = b.n
        y0 = inputs.travelling_mode((nn[0], nn[1], nn[2]), kvec, 0.0)
        # thin axes use h = 1/n too; the mode does not vary along them
        y = b.embed(y0)
        oracle.rk4(b, oracle.WAVE, oracle.BC_PERIODIC, y, 0.0, dt, steps)
        X = np.arange(nn[0]) * h
        Y = np.arange(nn[1]) * h
        ZZ, YY, XX = np.meshgrid(np.arange(nn[2]) * h, Y, X, indexing="ij")
        k = np.array(kvec, float)
        w = 2 * np.pi * np.sqrt((k ** 2).sum())
        ph = 2 * np.pi * (k[0] * XX + k[1] * YY) - w * T
        errs.append(np.abs(b.interior(y[0]) - np.sin(ph)).max())
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.8 <= o <= 4.2 for o in orders), (errs, orders)


def _energy(b, y):
    """E = 1/2 sum (rho^2 - u Lap_h u) h^3 with the oracle's own Laplacian"""
    oracle.fill_periodic(b, y)
    r = oracle.wave_rhs(b, y)
    u, rho, lap = b.interior(y[0]), b.interior(y[1]), b.interior(r[1])
    return 0.5 * np.sum(rho * rho - u * lap) * np.prod(b.h)


def test_wave_energy_decay_single_mode(orc):
    n, h = 16, 1.0 / 16
    dt = 0.25 * h
    k = (2, 1, 0)
    y0 = inputs.travelling_mode((n, n, n), k, 0.0)
    b = oracle.Block((n, n, n), 2, h)
    y = b.embed(y0)
    e0 = _energy(b, y)
    oracle.rk4(b, oracle.WAVE, oracle.BC_PERIODIC, y, 0.0, dt, 1)
    e1 = _energy(b, y)
    th = 2 * np.pi * np.array(k) * h
    lam = -np.sum((30 - 32 * np.cos(th) + 2 * np.cos(2 * th)) / 12.0) / h ** 2
    w = -dt * dt * lam
    factor = 1 - w ** 3 / 72 + w ** 4 / 576
    assert abs(e1 / e0 - factor) < 1e-12


def test_wave_energy_monotone_multimode(orc):
    n, h = 32, 1.0 / 32
    dt = 0.25 * h
    b = oracle.Block((n, n, n), 2, h)
    y = b.embed(inputs.fourier_modes(n, 4, inputs.SEED0))
    es = [_energy(b, y)]
    for _ in range(5):
        oracle.rk4(b, oracle.WAVE, oracle.BC_PERIODIC, y, 0.0, dt, 1)
        es.append(_energy(b, y))
    assert all(es[i + 1] < es[i] for i in range(5)), es
    assert es[-1] > 0.99 * es[0]
