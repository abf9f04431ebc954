"""Pins for the oracle's BSSN path (the Einstein equations that Sec. III.D
evolves; chi-form BSSN with 1+log or harmonic slicing, Gamma-driver or
frozen shift, 4th-order centred stencils plus lopsided advection).

The paper prints no equations, so every pin is an exact solution or a
mathematical property:
  * Minkowski data -> right-hand side exactly zero;
  * the gauge wave (exact vacuum solution under harmonic slicing, zero
    shift) along each axis: RHS at t = 0 equals the exact dt of every
    variable, converging at 4th order;
  * flat space in sheared, moving coordinates (nonzero shift, non-diagonal
    metric, lapse 1, K_ij = 0): RHS of chi, gt_ij, Gamt^i equal the exact
    dt; RHS of trK and At_ij vanish; 4th-order convergence;
  * covariance under a permutation of the axes (catches index mistakes);
  * Hamiltonian / momentum constraints vanish at 4th order on exact data;
  * harmonic gauge-wave evolution converges to the exact solution at 4th
    order; under 1+log / Gamma-driver the Hamiltonian constraint converges.
The 1+log / Gamma-driver gauge right-hand sides are pinned separately on
closed-form data in test_oracle_gauge.py.
"""
import numpy as np
import pytest

import oracle
from paper_1410_1764_amd import inputs as I

HARMONIC, ONEPLUSLOG = 1, 0
FROZEN, GAMMADRIVER = 0, 1


def gw_block(n, axis, g=3, thin=4, slicing=HARMONIC, shift=FROZEN, A=0.1):
    nn = [thin, thin, thin]
    nn[axis] = n
    return oracle.Block(tuple(nn), g, 1.0 / n, slicing=slicing, shift=shift,
                        gw_amp=A, gw_d=1.0, gw_axis=axis)


def gw_exact_dt(b, t=0.0):
    """exact dt of all 24 variables via a complex step in theta = 2 pi (x_a - t)"""
    a = b.gw_axis
    X = np.meshgrid(*[b.origin[d] + b.h[d] * np.arange(b.n[d]) for d in (2, 1, 0)],
                    indexing="ij")[::-1]
    th = 2 * np.pi * (X[a] - t) / b.gw_d
    dth = 1e-30
    f = I.gaugewave_fields(th + 1j * dth, b.gw_amp, b.gw_d, a)
    return -(2 * np.pi / b.gw_d) * np.imag(f) / dth


def rhs_errors(b, y0, exact):
    y = b.embed(y0)
    oracle.fill_periodic(b, y)
    r = b.interior(oracle.bssn_rhs(b, y))
    return np.abs(r - exact).reshape(24, -1).max(axis=1), r


def test_minkowski_rhs_exactly_zero(orc):
    for slicing, shift in ((ONEPLUSLOG, GAMMADRIVER), (HARMONIC, FROZEN)):
        b = oracle.Block((10, 8, 6), 3, (0.1, 0.12, 0.09), slicing=slicing, shift=shift)
        y = b.embed(I.minkowski(b.n))
        oracle.fill_periodic(b, y)
        r = oracle.bssn_rhs(b, y)
        assert np.count_nonzero(r) == 0


def test_gaugewave_ghost_fill_matches_closed_form(orc):
    b = oracle.Block((12, 5, 4), 3, (1 / 12, 0.2, 0.25), origin=(0.1, -0.3, 0.7),
                     gw_amp=0.1, gw_d=1.0, gw_axis=0)
    y = b.zeros(24)
    oracle.fill_gaugewave(b, y, 0.37)
    nn = tuple(v + 2 * b.g for v in b.n)
    want = I.gaugewave(nn, b.h, tuple(b.origin[d] - b.g * b.h[d] for d in range(3)),
                       b.gw_amp, b.gw_d, 0, 0.37)
    mask = np.ones(b.ext, bool)
    b.interior(mask)[...] = False
    assert np.abs(y[:, mask] - want[:, mask]).max() < 1e-14
    assert np.count_nonzero(b.interior(y)) == 0


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_gaugewave_rhs_converges_to_exact_dt(orc, axis):
    errs = []
    for n in (16, 32):
        b = gw_block(n, axis)
        y0 = I.gaugewave(b.n, b.h, axis=axis)
        e, _ = rhs_errors(b, y0, gw_exact_dt(b))
        errs.append(e)
    scale = np.abs(gw_exact_dt(gw_block(32, axis))).reshape(24, -1).max(axis=1)
    for v in range(24):
        if scale[v] == 0:
            assert errs[1][v] < 1e-13, (I.BSSN_NAMES[v], errs[1][v])
        elif errs[1][v] > 1e-12 * scale[v]:  # else no stencil error at all
            ratio = errs[0][v] / errs[1][v]
            assert ratio > 13.0, (I.BSSN_NAMES[v], errs[0][v], errs[1][v])
            assert errs[1][v] < 2e-3 * scale[v]


def test_gaugewave_1pluslog_lapse_rhs(orc):
    """with 1+log slicing and zero shift, dt alpha = -2 alpha K exactly (no stencil)"""
    b = gw_block(16, 0, slicing=ONEPLUSLOG, shift=GAMMADRIVER)
    y0 = I.gaugewave(b.n, b.h, axis=0)
    y = b.embed(y0)
    oracle.fill_periodic(b, y)
    r = b.interior(oracle.bssn_rhs(b, y))
    assert np.abs(r[I.ALP] - (-2 * y0[I.ALP] * y0[I.TRK])).max() < 1e-15


def oblique_exact_dt(n, m, A=0.1):
    """exact dt via a complex step: theta = 2 pi (m.x - |m| t)"""
    X = np.meshgrid(*[np.arange(n[d]) / n[d] for d in (2, 1, 0)], indexing="ij")[::-1]
    th = 2 * np.pi * (m[0] * X[0] + m[1] * X[1] + m[2] * X[2])
    dth = 1e-30
    f = I.gaugewave_oblique_fields(th + 1j * dth, A, m)
    return -2 * np.pi * np.sqrt(float(np.dot(m, m))) * np.imag(f) / dth


@pytest.mark.parametrize("m", [(1, 1, 0), (1, -1, 1), (0, 2, -1)])
def test_oblique_gaugewave_rhs_converges_to_exact_dt(orc, m):
    """every tensor component nonzero: pins the off-diagonal terms of all
    24 right-hand sides (harmonic slicing, frozen shift)"""
    errs, scale = [], None
    for n in (24, 48):
        nn = tuple(n if m[d] else 4 for d in range(3))
        b = oracle.Block(nn, 3, tuple(1.0 / v for v in nn), slicing=HARMONIC, shift=FROZEN)
        ex = oblique_exact_dt(nn, m)
        e, _ = rhs_errors(b, I.gaugewave_oblique(nn, m), ex)
        errs.append(e)
        scale = np.abs(ex).reshape(24, -1).max(axis=1)
    for v in range(24):
        if scale[v] == 0:
            assert errs[1][v] < 1e-13, (I.BSSN_NAMES[v], errs[1][v])
        elif errs[1][v] > 1e-12 * scale[v]:
            assert errs[0][v] / errs[1][v] > 13.0, (I.BSSN_NAMES[v], errs[0][v], errs[1][v])
            assert errs[1][v] < 2e-3 * scale[v], (I.BSSN_NAMES[v], errs[1][v], scale[v])


SH_M, SH_EPS, SH_OMEGA = (1, -1, 1), (0.03, -0.02, 0.025), 2.5


def sheared_exact_dt(b):
    """exact dt: every field is F(theta), theta = k.x - omega t, so
    dt F = -omega F'(theta); chi and gt by a complex step, Gamt by an
    8th-order central difference of its (complex-step) closed form."""
    X = np.meshgrid(*[b.h[d] * np.arange(b.n[d]) for d in (2, 1, 0)], indexing="ij")[::-1]
    k = 2 * np.pi * np.array(SH_M, float)
    th = k[0] * X[0] + k[1] * X[1] + k[2] * X[2]
    dth = 1e-30
    f = I.sheared_metric(th + 1j * dth, SH_M, SH_EPS, SH_OMEGA)
    dt = -SH_OMEGA * np.imag(f) / dth
    dt[I.GAM:I.GAM + 3] = 0.0
    c = [1 / 280, -4 / 105, 1 / 5, -4 / 5, 0, 4 / 5, -1 / 5, 4 / 105, -1 / 280]
    dd = 1e-2
    acc = np.zeros((3, *th.shape))
    for m, cm in zip(range(-4, 5), c):
        if cm:
            acc += cm * I.sheared_flat_fields(th + m * dd, SH_M, SH_EPS, SH_OMEGA)[I.GAM:I.GAM + 3]
    dt[I.GAM:I.GAM + 3] = -SH_OMEGA * acc / dd
    # exact: trK, At stay zero; gauge variables are not compared
    return dt


SH_CHECK = [I.CHI, *range(I.GT, I.GT + 6), I.TRK, *range(I.AT, I.AT + 6),
            *range(I.GAM, I.GAM + 3)]


def test_sheared_flat_rhs_converges_to_exact_dt(orc):
    errs, scales = [], []
    for n in (32, 64):
        b = oracle.Block((n, n, n), 3, 1.0 / n, slicing=ONEPLUSLOG, shift=GAMMADRIVER)
        y0 = I.sheared_flat(b.n, b.h, SH_M, SH_EPS, SH_OMEGA)
        ex = sheared_exact_dt(b)
        e, r = rhs_errors(b, y0, ex)
        errs.append(e)
        scales.append(np.abs(ex).reshape(24, -1).max(axis=1))
    norm = max(scales[1][v] for v in SH_CHECK)
    for v in SH_CHECK:
        assert errs[1][v] < 2e-3 * norm, (I.BSSN_NAMES[v], errs[1][v], norm)
        if errs[1][v] > 1e-12 * norm:  # else exact (e.g. trK: every term vanishes)
            ratio = errs[0][v] / errs[1][v]
            assert ratio > 12.0, (I.BSSN_NAMES[v], errs[0][v], errs[1][v])


def _smooth_random(n, seed, amp=0.02):
    """Minkowski plus a few random smooth periodic modes on every variable,
    with shift components of both signs (exercises every term and both
    lopsided stencils)"""
    rng = np.random.default_rng(seed)
    y = I.minkowski(n)
    nx, ny, nz = n
    Z, Y, X = np.meshgrid(np.arange(nz) / nz, np.arange(ny) / ny, np.arange(nx) / nx,
                          indexing="ij")
    for v in range(24):
        for _ in range(3):
            m = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            y[v] += amp * rng.standard_normal() * np.sin(
                2 * np.pi * (m[0] * X + m[1] * Y + m[2] * Z) + ph)
    return y


def _permute(y, sigma):
    """new axis a is old axis sigma[a]; tensor components follow"""
    ax = [2 - sigma[2], 2 - sigma[1], 2 - sigma[0]]
    out = np.empty_like(np.transpose(y, (0, *[a + 1 for a in ax])))
    for v in range(24):
        out[v] = np.transpose(y[v], ax)
    res = out.copy()
    for i in range(3):
        for j in range(i, 3):
            si, sj = sigma[i], sigma[j]
            res[I.GT + I.SYM[i][j]] = out[I.GT + I.SYM[si][sj]]
            res[I.AT + I.SYM[i][j]] = out[I.AT + I.SYM[si][sj]]
        for base in (I.GAM, I.BETA, I.BB):
            res[base + i] = out[base + sigma[i]]
    return res


@pytest.mark.parametrize("sigma", [(1, 2, 0), (2, 0, 1), (1, 0, 2), (0, 2, 1)])
def test_axis_permutation_covariance(orc, sigma):
    n = (14, 12, 10)
    h = (1 / 14, 1 / 12, 1 / 10)
    y0 = _smooth_random(n, 7)
    b = oracle.Block(n, 3, h, slicing=ONEPLUSLOG, shift=GAMMADRIVER)
    y = b.embed(y0)
    oracle.fill_periodic(b, y)
    r = b.interior(oracle.bssn_rhs(b, y))
    n2 = tuple(n[sigma[a]] for a in range(3))
    h2 = tuple(h[sigma[a]] for a in range(3))
    b2 = oracle.Block(n2, 3, h2, slicing=ONEPLUSLOG, shift=GAMMADRIVER)
    y2 = b2.embed(_permute(y0, sigma))
    oracle.fill_periodic(b2, y2)
    r2 = b2.interior(oracle.bssn_rhs(b2, y2))
    want = _permute(r, sigma)
    for v in range(24):
        s = np.abs(want[v]).max()
        assert np.abs(r2[v] - want[v]).max() <= 1e-12 * max(s, 1e-300), I.BSSN_NAMES[v]


def test_constraints_vanish_at_fourth_order_on_exact_data(orc):
    # gauge wave, each axis
    for axis in range(3):
        hs = []
        for n in (16, 32):
            b = gw_block(n, axis)
            y = b.embed(I.gaugewave(b.n, b.h, axis=axis))
            oracle.fill_periodic(b, y)
            _, norms = oracle.constraints(b, y)
            hs.append(norms)
        assert hs[0][0] / hs[1][0] > 13.0, hs
        assert hs[1][0] < 1e-3
        for c in range(1, 4):
            assert hs[1][c] < 1e-3
            if hs[0][c] > 1e-12:
                assert hs[0][c] / hs[1][c] > 13.0, hs
    # oblique gauge wave: momentum constraint with every component nonzero
    hs = []
    for n in (24, 48):
        m = (1, -1, 1)
        b = oracle.Block((n, n, n), 3, 1.0 / n)
        y = b.embed(I.gaugewave_oblique(b.n, m))
        oracle.fill_periodic(b, y)
        _, norms = oracle.constraints(b, y)
        hs.append(norms)
    for c in range(4):
        assert hs[0][c] / hs[1][c] > 13.0, hs
        assert hs[1][c] < 1e-3
    # sheared flat coordinates (K_ij = 0, so M^i vanishes identically)
    hs = []
    for n in (24, 48):
        b = oracle.Block((n, n, n), 3, 1.0 / n)
        y = b.embed(I.sheared_flat(b.n, b.h, SH_M, SH_EPS, SH_OMEGA))
        oracle.fill_periodic(b, y)
        hm, norms = oracle.constraints(b, y)
        hs.append(norms)
        rms = np.sqrt((b.interior(hm) ** 2).reshape(4, -1).mean(axis=1))
        assert np.allclose(rms, norms, rtol=1e-12, atol=0)
    assert hs[0][0] / hs[1][0] > 12.0, hs
    assert hs[0][1:].max() == 0 and hs[1][1:].max() == 0


def _gw_evolve_error(n, axis, T, bc):
    b = gw_block(n, axis)
    dt = 0.25 * b.h[axis]
    steps = int(round(T / dt))
    y = b.embed(I.gaugewave(b.n, b.h, axis=axis))
    oracle.rk4(b, oracle.BSSN, bc, y, 0.0, dt, steps)
    ex = I.gaugewave(b.n, b.h, axis=axis, t=steps * dt)
    return np.abs(b.interior(y) - ex).max()


def test_harmonic_gaugewave_evolution_converges(orc):
    errs = [_gw_evolve_error(n, 0, 0.25, oracle.BC_PERIODIC) for n in (32, 64, 128)]
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.7 <= o <= 4.3 for o in orders), (errs, orders)


def test_harmonic_gaugewave_evolution_analytic_ghosts(orc):
    """Analytic ghosts at the stage time t_n + c_s dt do not match the RK
    stage values (those are only low-order approximations of the solution at
    that time), so the boundary injects an error of size A (dt/h)^2-ish that
    does not shrink with h: the classic order reduction of time-dependent
    boundary data in RK methods.  Pin: the error stays at that small,
    resolution-independent level (and is zero-order in h, not growing)."""
    errs = [_gw_evolve_error(n, 0, 0.25, oracle.BC_GAUGEWAVE) for n in (32, 64, 128)]
    assert max(errs) < 1e-4, errs
    assert errs[2] <= 1.05 * errs[1], errs


def test_gaugewave_evolution_each_axis_agrees(orc):
    """the same 1-D problem along x, y and z gives the same numbers up to rounding"""
    outs = []
    for axis in range(3):
        b = gw_block(24, axis)
        y = b.embed(I.gaugewave(b.n, b.h, axis=axis))
        oracle.rk4(b, oracle.BSSN, oracle.BC_PERIODIC, y, 0.0, 0.25 / 24, 6)
        line = b.interior(y)
        idx = [slice(None)] * 4
        for d in range(3):
            if d != axis:
                idx[3 - d] = 0
        outs.append(_permute_components_to_x(line[tuple(idx)], axis))
    for o in outs[1:]:
        assert np.abs(o - outs[0]).max() < 1e-13


def _permute_components_to_x(line, axis):
    """components of a 1-D line along `axis` relabelled as if along x"""
    sigma = {0: (0, 1, 2), 1: (1, 0, 2), 2: (2, 1, 0)}[axis]
    res = line.copy()
    for i in range(3):
        for j in range(i, 3):
            res[I.GT + I.SYM[i][j]] = line[I.GT + I.SYM[sigma[i]][sigma[j]]]
            res[I.AT + I.SYM[i][j]] = line[I.AT + I.SYM[sigma[i]][sigma[j]]]
        for base in (I.GAM, I.BETA, I.BB):
            res[base + i] = line[base + sigma[i]]
    return res


def test_onepluslog_gaugewave_hamiltonian_converges(orc):
    """1+log / Gamma-driver: not an exact solution, but H must converge at 4th order"""
    hs = []
    for n in (32, 64):
        b = gw_block(n, 0, slicing=ONEPLUSLOG, shift=GAMMADRIVER)
        dt = 0.25 / n
        y = b.embed(I.gaugewave(b.n, b.h, axis=0))
        oracle.rk4(b, oracle.BSSN, oracle.BC_PERIODIC, y, 0.0, dt, n // 4)
        _, norms = oracle.constraints(b, y)
        hs.append(norms[0])
    assert hs[0] / hs[1] > 12.0, hs
