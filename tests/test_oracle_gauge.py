"""Pins for the oracle's gauge right-hand sides: 1+log or harmonic slicing
and the Gamma-driver shift (the gauge of the Einstein system evolved in
Sec. III.D; the paper prints no equations, so the forms are the readings
listed in the design notes):

  dt alpha  = beta^k d_k alpha - 2 alpha K          (1+log)
            = beta^k d_k alpha - alpha^2 K          (harmonic)
  dt beta^i = beta^k d_k beta^i + F B^i
  dt B^i    = beta^k d_k B^i + (dt Gt^i - beta^k d_k Gt^i) - eta B^i

Data: flat space in sheared, moving coordinates (lapse 1, K_ij = 0,
non-diagonal metric, a shift of both signs, every field a function of
theta = k.x - omega t), with the lapse, B^i and (for the slicing pin) trK
replaced by seeded smooth periodic fields.  With At_ij = 0 and K = 0 the
non-advective part of dt Gt^i depends on neither the lapse nor B^i, so it is
the exact dt Gt^i of the sheared coordinates minus its advection:
-(omega + beta.k) dGt^i/dtheta.  Every expected value is built from closed
forms and their exact derivatives (complex step or analytic), never from a
stencil; the oracle's stencils (centred for d beta in the Gamma terms,
lopsided on the upwind side for every advection) must converge to them at
4th order.  A second test shows that the plausible mistakes (a sign or
coefficient on F, eta or K, a dropped advection term, the Gt advection left
inside the B^i driver) each miss the oracle by far more than its stencil
error, and a third that F and eta are taken from the parameters.
"""
import numpy as np
import pytest

import oracle
from paper_1410_1764_amd import inputs as I

SH_M, SH_EPS, SH_OMEGA = (1, -1, 1), (0.03, -0.02, 0.025), 2.5
ONEPLUSLOG, HARMONIC = 0, 1
GAMMADRIVER = 1

# seeded smooth periodic fields: (amplitude, integer mode, phase)
ALPHA_MODES = [(0.05, (1, 0, -1), 0.3), (0.02, (0, 2, 1), 1.1)]
K_MODES = [(0.04, (1, 1, 0), 0.7), (0.015, (-1, 0, 2), 2.0)]
B_MODES = [[(0.06, (0, 1, 1), 0.2)], [(0.05, (1, -1, 0), 1.3)], [(0.07, (2, 0, -1), 2.4)]]


def _coords(n):
    h = 1.0 / n
    x = h * np.arange(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return (X, Y, Z), h


def _smooth(X, modes):
    """value and exact gradient of sum_a amp_a sin(2 pi m_a.x + ph_a)"""
    f = np.zeros_like(X[0])
    g = [np.zeros_like(X[0]) for _ in range(3)]
    for amp, m, ph in modes:
        arg = 2 * np.pi * (m[0] * X[0] + m[1] * X[1] + m[2] * X[2]) + ph
        f += amp * np.sin(arg)
        for d in range(3):
            g[d] += amp * 2 * np.pi * m[d] * np.cos(arg)
    return f, g


def _theta(X):
    k = 2 * np.pi * np.asarray(SH_M, float)
    return k, k[0] * X[0] + k[1] * X[1] + k[2] * X[2]


def _beta_and_dbeta(th):
    """shift of the sheared coordinates and d beta^i / d theta (complex step)"""
    dth = 1e-30
    f = I.sheared_metric(th + 1j * dth, SH_M, SH_EPS, SH_OMEGA)
    beta = np.real(f[I.BETA:I.BETA + 3])
    dbeta = np.imag(f[I.BETA:I.BETA + 3]) / dth
    return beta, dbeta


def _dgam_dtheta(th):
    """d Gt^i / d theta: 8th-order central difference of the closed form
    (Gt^i itself is a complex-step derivative, so it cannot take another)"""
    c = [1 / 280, -4 / 105, 1 / 5, -4 / 5, 0, 4 / 5, -1 / 5, 4 / 105, -1 / 280]
    dd = 1e-2
    acc = np.zeros((3, *th.shape))
    for m, cm in zip(range(-4, 5), c):
        if cm:
            acc += cm * I.sheared_flat_fields(th + m * dd, SH_M, SH_EPS, SH_OMEGA)[I.GAM:I.GAM + 3]
    return acc / dd


def gauge_case(n, with_K):
    """(interior data, exact gauge right-hand sides) on an n^3 periodic block.
    exact = dict of named terms so that the tests can assemble the correct
    right-hand side and its plausible mistakes from the same pieces."""
    X, h = _coords(n)
    k, th = _theta(X)
    y = I.sheared_flat((n, n, n), h, SH_M, SH_EPS, SH_OMEGA)
    alpha_p, dalpha = _smooth(X, ALPHA_MODES)
    y[I.ALP] = 1.0 + alpha_p
    K = np.zeros_like(th)
    if with_K:
        K, _ = _smooth(X, K_MODES)
        y[I.TRK] = K
    B, dB = [], []
    for i in range(3):
        f, g = _smooth(X, B_MODES[i])
        y[I.BB + i] = f
        B.append(f)
        dB.append(g)
    beta, dbeta_th = _beta_and_dbeta(th)
    assert np.abs(beta - y[I.BETA:I.BETA + 3]).max() == 0.0
    assert (beta > 0).any() and (beta < 0).any()
    bk = beta[0] * k[0] + beta[1] * k[1] + beta[2] * k[2]  # beta^k k_k
    dG = _dgam_dtheta(th)
    terms = {
        "alpha": y[I.ALP], "K": K, "B": np.array(B),
        "adv_alpha": sum(beta[d] * dalpha[d] for d in range(3)),
        "adv_beta": bk[None] * dbeta_th,
        "adv_B": np.array([sum(beta[d] * dB[i][d] for d in range(3)) for i in range(3)]),
        # dt Gt^i = -omega dGt/dtheta; minus its advection beta^k k_k dGt/dtheta
        "dtG": -SH_OMEGA * dG,
        "advG": bk[None] * dG,
    }
    return y, terms


BETA_CONST = (0.3, -0.2, 0.15)


def const_shift_case(n, with_K):
    """flat metric in uniformly moving coordinates (a constant shift of both
    signs), with a smooth lapse, B^i and optionally K: Gt^i = 0 and, with
    At_ij = 0 and K = 0, the non-advective part of dt Gt^i vanishes exactly,
    so the B^i driver reduces to its advection and damping"""
    X, h = _coords(n)
    y = I.minkowski((n, n, n))
    for i in range(3):
        y[I.BETA + i] = BETA_CONST[i]
    alpha_p, dalpha = _smooth(X, ALPHA_MODES)
    y[I.ALP] = 1.0 + alpha_p
    K = np.zeros_like(X[0])
    if with_K:
        K, _ = _smooth(X, K_MODES)
        y[I.TRK] = K
    B, dB = [], []
    for i in range(3):
        f, g = _smooth(X, B_MODES[i])
        y[I.BB + i] = f
        B.append(f)
        dB.append(g)
    zero = np.zeros((3, *X[0].shape))
    terms = {
        "alpha": y[I.ALP], "K": K, "B": np.array(B),
        "adv_alpha": sum(BETA_CONST[d] * dalpha[d] for d in range(3)),
        "adv_beta": zero,
        "adv_B": np.array([sum(BETA_CONST[d] * dB[i][d] for d in range(3)) for i in range(3)]),
        "dtG": zero, "advG": zero,
    }
    return y, terms


def expected(terms, slicing=ONEPLUSLOG, F=0.75, eta=2.0):
    a, K = terms["alpha"], terms["K"]
    lapse = -2.0 * a * K if slicing == ONEPLUSLOG else -a * a * K
    return {
        "alpha": terms["adv_alpha"] + lapse,
        "beta": terms["adv_beta"] + F * terms["B"],
        "B": terms["adv_B"] + (terms["dtG"] - terms["advG"]) - eta * terms["B"],
    }


def oracle_gauge_rhs(y, n, slicing=ONEPLUSLOG, F=0.75, eta=2.0):
    b = oracle.Block((n, n, n), 3, 1.0 / n, slicing=slicing, shift=GAMMADRIVER,
                     shift_F=F, eta=eta)
    yy = b.embed(y)
    oracle.fill_periodic(b, yy)
    r = b.interior(oracle.bssn_rhs(b, yy))
    return {"alpha": r[I.ALP], "beta": r[I.BETA:I.BETA + 3], "B": r[I.BB:I.BB + 3]}


def _err(got, want):
    return float(np.abs(got - want).max())


CASES = {"sheared": gauge_case, "const_shift": const_shift_case}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("with_K,slicing", [(False, ONEPLUSLOG), (True, ONEPLUSLOG),
                                            (True, HARMONIC)])
def test_gauge_rhs_converges_to_closed_form(orc, case, with_K, slicing):
    """alpha, beta^i, B^i right-hand sides -> exact values at 4th order.
    Without K, the B^i driver is pinned against the exact dt Gt^i; with a
    smooth K the lapse pin includes its -2 alpha K (or -alpha^2 K) term
    with a nonzero shift (dt Gt^i then has a K term the closed form lacks,
    so B^i is compared only in the K-free case)."""
    errs, scale = [], {}
    for n in (32, 64):
        y, terms = CASES[case](n, with_K)
        want = expected(terms, slicing)
        got = oracle_gauge_rhs(y, n, slicing)
        names = ["alpha", "beta"] + ([] if with_K else ["B"])
        errs.append({q: _err(got[q], want[q]) for q in names})
        scale = {q: float(np.abs(want[q]).max()) for q in names}
    for q in errs[1]:
        assert scale[q] > 1e-2, (q, scale[q])
        if case == "const_shift" and q == "beta":
            # constant shift: every difference of beta is exactly zero
            assert errs[1][q] == 0.0 and errs[0][q] == 0.0
            continue
        assert errs[1][q] < 1e-3 * scale[q], (q, errs[1][q], scale[q])
        ratio = errs[0][q] / errs[1][q]
        assert 13.0 < ratio < 19.0, (q, errs[0][q], errs[1][q], ratio)


def _caught(got, good, wrong, margin=30.0):
    """the oracle sits on the correct closed form and far from the wrong one"""
    return _err(got, wrong) > margin * _err(got, good)


def test_gauge_rhs_plausible_mistakes_are_caught(orc):
    """each mistake that a reading of the gauge could plausibly introduce
    moves a right-hand side by far more than the stencil error that the
    convergence pin leaves (n = 64)"""
    n = 64
    # constant shift: F, eta, the advection of B^i and alpha, the lapse term
    for with_K in (False, True):
        y, terms = const_shift_case(n, with_K)
        got = oracle_gauge_rhs(y, n)
        good = expected(terms)
        wrong_alpha = {
            "alpha not advected": good["alpha"] - terms["adv_alpha"],
            "advection sign": good["alpha"] - 2 * terms["adv_alpha"],
        }
        if with_K:
            wrong_alpha.update({
                "K coefficient 1": terms["adv_alpha"] - terms["alpha"] * terms["K"],
                "K term sign": terms["adv_alpha"] + 2 * terms["alpha"] * terms["K"],
                "harmonic instead of 1+log": expected(terms, slicing=HARMONIC)["alpha"],
            })
        for name, wrong in wrong_alpha.items():
            assert _caught(got["alpha"], good["alpha"], wrong), name
        if with_K:
            continue
        for name, (q, wrong) in {
            "F sign": ("beta", expected(terms, F=-0.75)["beta"]),
            "F = 1": ("beta", expected(terms, F=1.0)["beta"]),
            "eta sign": ("B", expected(terms, eta=-2.0)["B"]),
            "eta = 1": ("B", expected(terms, eta=1.0)["B"]),
            "B not advected": ("B", good["B"] - terms["adv_B"]),
            "B advection sign": ("B", good["B"] - 2 * terms["adv_B"]),
        }.items():
            assert np.abs(got[q] - wrong).max() > 0.01, name
            if _err(got[q], good[q]) > 0:
                assert _caught(got[q], good[q], wrong), name
    # sheared coordinates: the shift's own advection and the Gamma terms
    y, terms = gauge_case(n, with_K=False)
    got = oracle_gauge_rhs(y, n)
    good = expected(terms)
    for name, (q, wrong) in {
        "beta not advected": ("beta", good["beta"] - terms["adv_beta"]),
        "Gt advection kept in the driver": ("B", good["B"] + terms["advG"]),
        "driver without the Gt term": ("B", good["B"] - (terms["dtG"] - terms["advG"])),
        "Gt term sign": ("B", good["B"] - 2 * (terms["dtG"] - terms["advG"])),
    }.items():
        assert _caught(got[q], good[q], wrong), name


def test_gauge_parameters_are_used(orc):
    """F and eta come from the block's parameters, not constants (constant
    shift: the closed form there is known to within a tiny stencil error)"""
    n = 32
    for case in (const_shift_case,):
        y, terms = case(n, False)
        for F, eta in ((0.5, 1.0), (1.25, 3.5)):
            got = oracle_gauge_rhs(y, n, F=F, eta=eta)
            want = expected(terms, F=F, eta=eta)
            for q in ("beta", "B"):
                s = float(np.abs(want[q]).max())
                assert _err(got[q], want[q]) < 2e-2 * s, (F, eta, q)
                other = expected(terms, F=0.75, eta=2.0)[q]
                assert _caught(got[q], want[q], other, margin=5.0), (F, eta, q)
