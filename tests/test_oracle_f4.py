"""Pins for the oracle's 6th- and 8th-order finite-difference operators (the
paper's generator takes the order as a parameter, Sec. III.B.2).

Pinned to what the mathematics fixes:
  * exactness on polynomials up to the operator's order and failure one
    degree higher (brute force on non-periodic blocks whose ghosts hold the
    polynomial itself), for the centred first, pure second and mixed second
    derivatives and both sides of the lopsided derivative;
  * the right-hand side of the oblique gauge wave (every tensor component
    nonzero) converges to the exact time derivative at the chosen order, and
    order 4 is bitwise the 4th-order code path.
"""
import numpy as np
import pytest

import oracle
from paper_1410_1764_amd import inputs as I
from tests.test_oracle_bssn import oblique_exact_dt, rhs_errors


def _block(order, n=(11, 10, 9), h=(0.11, 0.07, 0.13), origin=(-0.3, 0.2, -0.1)):
    return oracle.Block(n, order // 2 + 1, h, origin, fd_order=order)


def _mesh(b):
    x, y, z = b.coords()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def _rel(a, e):
    return np.abs(a - e).max() / max(np.abs(e).max(), 1e-300)


@pytest.mark.parametrize("order", [6, 8])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_first_centred_exact_to_order(orc, order, axis):
    b = _block(order)
    x = _mesh(b)[axis]
    c = np.random.default_rng(order + axis).standard_normal(order + 2)
    f = sum(c[m] * x ** m for m in range(order + 1))[None].copy()
    df = sum(m * c[m] * x ** (m - 1) for m in range(1, order + 1))
    assert _rel(b.interior(oracle.stencil(b, f, 1, axis)[0]), b.interior(df)) < 1e-11
    fh = (x ** (order + 1))[None].copy()
    out = oracle.stencil(b, fh, 1, axis)
    assert _rel(b.interior(out[0]), b.interior((order + 1) * x ** order)) > 1e-9


@pytest.mark.parametrize("order", [6, 8])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_second_centred_exact_to_order(orc, order, axis):
    b = _block(order)
    x = _mesh(b)[axis]
    c = np.random.default_rng(10 + order + axis).standard_normal(order + 3)
    f = sum(c[m] * x ** m for m in range(order + 2))[None].copy()
    d2f = sum(m * (m - 1) * c[m] * x ** (m - 2) for m in range(2, order + 2))
    assert _rel(b.interior(oracle.stencil(b, f, 2, axis, axis)[0]), b.interior(d2f)) < 1e-10
    p = order + 2
    fh = (x ** p)[None].copy()
    out = oracle.stencil(b, fh, 2, axis, axis)
    assert _rel(b.interior(out[0]), b.interior(p * (p - 1) * x ** (p - 2))) > 1e-9


@pytest.mark.parametrize("order", [6, 8])
@pytest.mark.parametrize("a,bdir", [(0, 1), (0, 2), (1, 2)])
def test_mixed_exact_to_order(orc, order, a, bdir):
    b = _block(order)
    C = _mesh(b)
    x, y = C[a], C[bdir]
    rng = np.random.default_rng(20 + order + a + bdir)
    terms = [(i, j, rng.standard_normal()) for i in range(order + 1) for j in range(order + 1)
             if i + j <= order + 1]
    f = sum(c * x ** i * y ** j for i, j, c in terms)[None].copy()
    dxy = sum(c * i * j * x ** max(i - 1, 0) * y ** max(j - 1, 0) for i, j, c in terms if i and j)
    out = oracle.stencil(b, f, 2, a, bdir)
    assert _rel(b.interior(out[0]), b.interior(dxy)) < 1e-10
    # x^(order+1) y is not reproduced
    fh = (x ** (order + 1) * y)[None].copy()
    outh = oracle.stencil(b, fh, 2, a, bdir)
    assert _rel(b.interior(outh[0]), b.interior((order + 1) * x ** order)) > 1e-9


@pytest.mark.parametrize("order", [6, 8])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("side", [1.0, -1.0])
def test_lopsided_exact_to_order(orc, order, axis, side):
    b = _block(order)
    x = _mesh(b)[axis]
    c = np.random.default_rng(30 + order + axis).standard_normal(order + 2)
    f = sum(c[m] * x ** m for m in range(order + 1))[None].copy()
    df = sum(m * c[m] * x ** (m - 1) for m in range(1, order + 1))
    sgn = np.full_like(f[0], side)
    assert _rel(b.interior(oracle.stencil(b, f, 3, axis, 0, sgn)[0]), b.interior(df)) < 1e-10
    fh = (x ** (order + 1))[None].copy()
    out = oracle.stencil(b, fh, 3, axis, 0, sgn)
    assert _rel(b.interior(out[0]), b.interior((order + 1) * x ** order)) > 1e-9


def test_order4_is_the_fourth_order_path(orc):
    n = (12, 10, 8)
    y = I.gaugewave_oblique(n, (1, -1, 1))
    r = []
    for order in (0, 4):
        b = oracle.Block(n, 3, tuple(1.0 / v for v in n), slicing=1, shift=0, fd_order=order)
        yo = b.embed(y)
        oracle.fill_periodic(b, yo)
        r.append(oracle.bssn_rhs(b, yo))
    assert np.array_equal(r[0], r[1])


@pytest.mark.parametrize("order,rate", [(6, 45.0), (8, 170.0)])
def test_oblique_gaugewave_rhs_converges_at_order(orc, order, rate):
    """2^order = 64 / 256: the error ratio between n = 24 and 48 approaches it
    (measured 53-61 and 201-225; order 4 gives 15.5-15.9)"""
    m = (1, -1, 1)
    errs, scale = [], None
    for n in (24, 48):
        nn = (n, n, n)
        b = oracle.Block(nn, order // 2 + 1, tuple(1.0 / v for v in nn), slicing=1, shift=0,
                         fd_order=order)
        ex = oblique_exact_dt(nn, m)
        e, _ = rhs_errors(b, I.gaugewave_oblique(nn, m), ex)
        errs.append(e)
        scale = np.abs(ex).reshape(24, -1).max(axis=1)
    checked = 0
    for v in range(24):
        if scale[v] > 0 and errs[1][v] > 1e-12 * scale[v]:
            assert errs[0][v] / errs[1][v] > rate, (I.BSSN_NAMES[v], errs[0][v], errs[1][v])
            checked += 1
    assert checked >= 10
