"""Pins for the oracle's finite-difference operators (Sec. III.B.2,
discretisation description: standard centred operators of a chosen order,
4th order here; lopsided 4th-order operators for advection).

Pinned to what the mathematics fixes, not to a retyped formula:
  * exactness on polynomials up to the operator's order (brute force on a
    small non-periodic block whose ghosts hold the polynomial itself), and
    failure one degree higher (so the order is exactly 4);
  * the Fourier symbol of each operator on periodic grids.
"""
import numpy as np
import pytest

import oracle


def _block(n=(7, 6, 5), g=3, h=(0.11, 0.07, 0.13), origin=(-0.3, 0.2, -0.1)):
    return oracle.Block(n, g, h, origin)


def _mesh(b):
    x, y, z = b.coords()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def _rel(a, e):
    return np.abs(a - e).max() / max(np.abs(e).max(), 1e-300)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_first_centred_exact_to_degree4(orc, axis):
    b = _block()
    C = _mesh(b)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(6)
    x = C[axis]
    f = sum(c[m] * x ** m for m in range(5))[None].copy()
    df = sum(m * c[m] * x ** (m - 1) for m in range(1, 5))
    out = oracle.stencil(b, f, 1, axis)
    assert _rel(b.interior(out[0]), b.interior(df)) < 1e-12
    # degree 5 is not reproduced: the operator is exactly 4th order
    f5 = (x ** 5)[None].copy()
    out5 = oracle.stencil(b, f5, 1, axis)
    assert _rel(b.interior(out5[0]), b.interior(5 * x ** 4)) > 1e-6


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_second_centred_exact_to_degree5(orc, axis):
    b = _block()
    C = _mesh(b)
    rng = np.random.default_rng(2)
    c = rng.standard_normal(6)
    x = C[axis]
    f = sum(c[m] * x ** m for m in range(6))[None].copy()
    d2f = sum(m * (m - 1) * c[m] * x ** (m - 2) for m in range(2, 6))
    out = oracle.stencil(b, f, 2, axis, axis)
    assert _rel(b.interior(out[0]), b.interior(d2f)) < 1e-11
    f6 = (x ** 6)[None].copy()
    out6 = oracle.stencil(b, f6, 2, axis, axis)
    assert _rel(b.interior(out6[0]), b.interior(30 * x ** 4)) > 1e-6


@pytest.mark.parametrize("a,bb", [(0, 1), (0, 2), (1, 2), (2, 0)])
def test_mixed_exact_on_tensor_polynomials(orc, a, bb):
    b = _block()
    C = _mesh(b)
    xa, xb = C[a], C[bb]
    for p in range(5):
        for q in range(5):
            f = (xa ** p * xb ** q)[None].copy()
            exact = (p * q) * (xa ** max(p - 1, 0)) * (xb ** max(q - 1, 0))
            out = oracle.stencil(b, f, 2, a, bb)
            err = np.abs(b.interior(out[0]) - b.interior(exact)).max()
            assert err < 1e-10 * max(1.0, np.abs(exact).max()), (p, q, err)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_lopsided_exact_to_degree4(orc, axis, sign):
    b = _block()
    C = _mesh(b)
    rng = np.random.default_rng(3)
    c = rng.standard_normal(5)
    x = C[axis]
    f = sum(c[m] * x ** m for m in range(5))[None].copy()
    df = sum(m * c[m] * x ** (m - 1) for m in range(1, 5))
    sgn = np.full_like(f, sign)
    out = oracle.stencil(b, f, 3, axis, sgn=sgn)
    assert _rel(b.interior(out[0]), b.interior(df)) < 1e-12
    f5 = (x ** 5)[None].copy()
    out5 = oracle.stencil(b, f5, 3, axis, sgn=sgn)
    assert _rel(b.interior(out5[0]), b.interior(5 * x ** 4)) > 1e-6


def _periodic_mode(n, m, axis):
    """sin and cos of 2 pi m x_axis on the periodic unit cube, with ghosts"""
    b = oracle.Block((n, n, n), 3, 1.0 / n)
    C = _mesh(b)
    ph = 2 * np.pi * m * C[axis]
    return b, np.sin(ph)[None].copy(), ph


@pytest.mark.parametrize("m", [1, 3, 7])
def test_fourier_symbols(orc, m):
    """Symbols with theta = 2 pi m h: centred d1 -> i (8 sin t - sin 2t)/(6h);
    centred d2 -> -(30 - 32 cos t + 2 cos 2t)/(12 h^2); lopsided (+) ->
    (-3 e^{-it} - 10 + 18 e^{it} - 6 e^{2it} + e^{3it})/(12h)."""
    n, axis = 16, 1
    b, f, ph = _periodic_mode(n, m, axis)
    oracle.fill_periodic(b, f)
    h = 1.0 / n
    t = 2 * np.pi * m * h
    e = np.exp(1j * ph)  # f = Im(e)
    s1 = 1j * (8 * np.sin(t) - np.sin(2 * t)) / (6 * h)
    s2 = -(30 - 32 * np.cos(t) + 2 * np.cos(2 * t)) / (12 * h * h)
    sl = (-3 * np.exp(-1j * t) - 10 + 18 * np.exp(1j * t) - 6 * np.exp(2j * t)
          + np.exp(3j * t)) / (12 * h)
    sr = (3 * np.exp(1j * t) + 10 - 18 * np.exp(-1j * t) + 6 * np.exp(-2j * t)
          - np.exp(-3j * t)) / (12 * h)
    got1 = oracle.stencil(b, f, 1, axis)[0]
    got2 = oracle.stencil(b, f, 2, axis, axis)[0]
    gotl = oracle.stencil(b, f, 3, axis, sgn=np.ones_like(f))[0]
    gotr = oracle.stencil(b, f, 3, axis, sgn=-np.ones_like(f))[0]
    for got, sym in ((got1, s1), (got2, s2), (gotl, sl), (gotr, sr)):
        exp = np.imag(sym * e)
        assert _rel(b.interior(got), b.interior(exp)) < 1e-12


def test_periodic_fill_matches_wrap(orc):
    rng = np.random.default_rng(4)
    b = oracle.Block((9, 5, 4), 3, 0.1)
    y = b.embed(rng.standard_normal((2, 4, 5, 9)))
    oracle.fill_periodic(b, y)
    for v in range(2):
        want = np.pad(b.interior(y[v]), 3, mode="wrap")
        assert np.array_equal(y[v], want)


@pytest.mark.parametrize("kind,a,bb", [(1, 0, 0), (2, 1, 1), (2, 0, 2), (3, 2, 0)])
def test_operators_blind_to_a_constant_offset(orc, kind, a, bb):
    """Every operator annihilates constants, so D(x) = D(x - 1) for x = 1 + n
    with noise n of size 1e-10 (x - 1 is exact in floating point).  Written
    on neighbour differences the oracle keeps this to the rounding of the
    small result; a weighted sum of the values themselves would round at the
    size of the constant and lose about six digits."""
    rng = np.random.default_rng(6)
    b = oracle.Block((8, 7, 6), 3, (0.1, 0.11, 0.09))
    x = 1.0 + rng.uniform(-1e-10, 1e-10, size=(1, *b.ext))
    sgn = rng.choice([-1.0, 1.0], size=x.shape)
    d_x = oracle.stencil(b, x, kind, a, bb, sgn=sgn)
    d_n = oracle.stencil(b, x - 1.0, kind, a, bb, sgn=sgn)
    scale = np.abs(b.interior(d_n)).max()
    assert np.abs(b.interior(d_x - d_n)).max() < 1e-13 * scale
