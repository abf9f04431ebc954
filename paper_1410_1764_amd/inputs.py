"""Seeded synthetic inputs for the tests, the oracle runs and the benchmark.

This module draws random numbers and writes down closed-form initial data
(the "Init" calculation of a physics system, Fig. 1).  It holds none of the
right-hand-side arithmetic and imports neither the oracle nor the HIP
library; both sides receive the same arrays from here.

Every generator returns interior values only, shape (nvar, n_z, n_y, n_x),
x fastest; point (i, j, k) sits at origin + (i, j, k) * h.  Ghost zones are
the method's business.

Variable order -- wave: u, rho.  BSSN (24): chi, gt11, gt12, gt13, gt22,
gt23, gt33, trK, At11, At12, At13, At22, At23, At33, Gamt1, Gamt2, Gamt3,
alpha, beta1, beta2, beta3, B1, B2, B3.
"""
from __future__ import annotations

import numpy as np

SEED0 = 17640  # workload i uses SEED0 + i

CHI, GT, TRK, AT, GAM, ALP, BETA, BB = 0, 1, 7, 8, 14, 17, 18, 21
SYM = ((0, 1, 2), (1, 3, 4), (2, 4, 5))
BSSN_NAMES = ["chi", "gt11", "gt12", "gt13", "gt22", "gt23", "gt33", "trK",
              "At11", "At12", "At13", "At22", "At23", "At33", "Gamt1", "Gamt2",
              "Gamt3", "alpha", "beta1", "beta2", "beta3", "B1", "B2", "B3"]
WAVE_NAMES = ["u", "rho"]
WAVE5_NAMES = ["u", "rho", "v1", "v2", "v3"]


def _ntuple(n):
    return tuple(int(v) for v in (n if np.ndim(n) else (n, n, n)))


def _grid(n, h, origin):
    n = _ntuple(n)
    h = tuple(float(v) for v in (h if np.ndim(h) else (h, h, h)))
    x = [origin[d] + h[d] * np.arange(n[d]) for d in range(3)]
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    return X, Y, Z


# ----------------------------------------------------------------------------
# scalar wave data


def fourier_modes(n: int, K: int, seed: int) -> np.ndarray:
    """u = sum over integer k with 0 < |k| <= K of a_k cos(2 pi k.x) + b_k sin(2 pi k.x),
    a_k, b_k ~ N(0, 1)/|k|^2 (all a drawn in lexicographic (kx, ky, kz)
    order, then all b); rho = 0.  Domain [0,1)^3, x_i = i/n.  Evaluated
    exactly by an inverse FFT of the coefficients placed at k mod n."""
    ks = [(kx, ky, kz) for kx in range(-K, K + 1) for ky in range(-K, K + 1)
          for kz in range(-K, K + 1) if 0 < kx * kx + ky * ky + kz * kz <= K * K]
    kk = np.array(ks)
    k2 = (kk ** 2).sum(axis=1).astype(float)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(len(ks)) / k2
    b = rng.standard_normal(len(ks)) / k2
    assert 2 * K < n
    c = np.zeros((n, n, n), dtype=complex)  # indexed [kz, ky, kx] to match (z, y, x)
    np.add.at(c, (kk[:, 2] % n, kk[:, 1] % n, kk[:, 0] % n), a - 1j * b)
    u = np.real(np.fft.ifftn(c)) * n ** 3
    out = np.zeros((2, n, n, n))
    out[0] = u
    return out


def travelling_mode(n, kvec, t: float = 0.0) -> np.ndarray:
    """u = sin(2 pi k.x - w t), rho = du/dt, w = 2 pi |k| (exact continuum
    solution of the wave equation on the periodic unit cube)."""
    n = _ntuple(n)
    X, Y, Z = _grid(n, tuple(1.0 / v for v in n), (0.0, 0.0, 0.0))
    k = np.asarray(kvec, dtype=float)
    w = 2 * np.pi * np.sqrt((k ** 2).sum())
    ph = 2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) - w * t
    return np.stack([np.sin(ph), -w * np.cos(ph)])


def gaussian_pulse(n, A: float = 1.0, W: float = 0.08, centre=(0.5, 0.5, 0.5)) -> np.ndarray:
    """Fig. 1's Init calculation for the first-order wave system:
    u = 0, rho = A exp(-(r/W)^2 / 2) with r the distance to `centre`, v_i = 0,
    on the unit cube with x_i = i/n."""
    nn = _ntuple(n)
    X = _grid(nn, tuple(1.0 / v for v in nn), (0.0, 0.0, 0.0))
    r2 = sum((X[d] - centre[d]) ** 2 for d in range(3))
    y = np.zeros((5, nn[2], nn[1], nn[0]))
    y[1] = A * np.exp(-0.5 * r2 / W ** 2)
    return y


def wave5_plane(n, kvec, t: float = 0.0) -> np.ndarray:
    """Exact plane wave of the first-order system: u = sin(theta),
    theta = 2 pi k.x - w t, w = 2 pi |k|; rho = du/dt, v_i = d_i u."""
    nn = _ntuple(n)
    X = _grid(nn, tuple(1.0 / v for v in nn), (0.0, 0.0, 0.0))
    k = np.asarray(kvec, dtype=float)
    w = 2 * np.pi * np.sqrt((k ** 2).sum())
    th = 2 * np.pi * (k[0] * X[0] + k[1] * X[1] + k[2] * X[2]) - w * t
    y = np.zeros((5, nn[2], nn[1], nn[0]))
    y[0] = np.sin(th)
    y[1] = -w * np.cos(th)
    for d in range(3):
        y[2 + d] = 2 * np.pi * k[d] * np.cos(th)
    return y


def wave5_fourier(n: int, K: int, seed: int) -> np.ndarray:
    """five independent seeded Fourier-mode fields (|k| <= K), one per variable"""
    y = np.zeros((5, n, n, n))
    for v in range(5):
        y[v] = fourier_modes(n, K, seed + 97 * v)[0]
    return y


# ----------------------------------------------------------------------------
# BSSN data


def minkowski(n, noise: float = 0.0, seed: int | None = None) -> np.ndarray:
    """Flat space (chi = alpha = 1, gt = identity, all else 0) plus independent
    uniform(-noise, noise) on every grid function at every point (GF-major)."""
    nx, ny, nz = _ntuple(n)
    y = np.zeros((24, nz, ny, nx))
    y[CHI] = 1.0
    y[ALP] = 1.0
    for i in range(3):
        y[GT + SYM[i][i]] = 1.0
    if noise:
        rng = np.random.default_rng(seed)
        y += rng.uniform(-noise, noise, size=y.shape)
    return y


def gaugewave_fields(theta, A: float, d: float, axis: int) -> np.ndarray:
    """BSSN variables of the gauge wave ds^2 = -H dt^2 + H dx_a^2 + dx_b^2 + dx_c^2,
    H = 1 - A sin(theta), theta = 2 pi (x_a - t)/d, zero shift.  theta may be
    complex (for complex-step derivatives)."""
    theta = np.asarray(theta)
    H = 1 - A * np.sin(theta)
    c = np.cos(theta)
    y = np.zeros((24, *theta.shape), dtype=np.result_type(theta, float))
    y[CHI] = H ** (-1 / 3)
    for b in range(3):
        if b == axis:
            y[GT + SYM[b][b]] = H ** (2 / 3)
            y[AT + SYM[b][b]] = -(2 * np.pi * A / (3 * d)) * c * H ** (-5 / 6)
        else:
            y[GT + SYM[b][b]] = H ** (-1 / 3)
            y[AT + SYM[b][b]] = (np.pi * A / (3 * d)) * c * H ** (-11 / 6)
    y[TRK] = -(np.pi * A / d) * c * H ** (-1.5)
    y[GAM + axis] = -(4 * np.pi * A / (3 * d)) * c * H ** (-5 / 3)
    y[ALP] = np.sqrt(H)
    return y


def gaugewave(n, h, origin=(0.0, 0.0, 0.0), A: float = 0.1, d: float = 1.0,
              axis: int = 0, t: float = 0.0) -> np.ndarray:
    X = _grid(n, h, origin)
    return gaugewave_fields(2 * np.pi * (X[axis] - t) / d, A, d, axis)


def gaugewave_oblique_fields(theta, A: float, m) -> np.ndarray:
    """Gauge wave travelling along the integer direction m on the periodic
    unit cube: H = 1 - A sin(theta), theta = 2 pi (m.x - |m| t),
    3-metric gamma_ij = delta_ij + (H - 1) n_i n_j with n = m/|m|, lapse
    sqrt(H), zero shift (a rotated copy of the axis-aligned gauge wave, so
    every tensor component is nonzero).  theta may be complex."""
    theta = np.asarray(theta)
    m = np.asarray(m, dtype=float)
    mm = np.sqrt((m ** 2).sum())
    nv = m / mm
    H = 1 - A * np.sin(theta)
    dtH = 2 * np.pi * mm * A * np.cos(theta)
    chi = H ** (-1 / 3)
    trK = -dtH / (2 * H ** 1.5)
    y = np.zeros((24, *theta.shape), dtype=np.result_type(theta, float))
    y[CHI] = chi
    y[TRK] = trK
    for i in range(3):
        for j in range(i, 3):
            gam = (1.0 if i == j else 0.0) + (H - 1) * nv[i] * nv[j]
            Kij = -dtH * nv[i] * nv[j] / (2 * np.sqrt(H))
            y[GT + SYM[i][j]] = chi * gam
            y[AT + SYM[i][j]] = chi * (Kij - gam * trK / 3)
        y[GAM + i] = -(4 * np.pi * mm * A / 3) * nv[i] * np.cos(theta) * H ** (-5 / 3)
    y[ALP] = np.sqrt(H)
    return y


def gaugewave_oblique(n, m, A: float = 0.1, t: float = 0.0) -> np.ndarray:
    nn = _ntuple(n)
    X = _grid(nn, tuple(1.0 / v for v in nn), (0.0, 0.0, 0.0))
    mm = np.sqrt(float(np.dot(m, m)))
    theta = 2 * np.pi * (m[0] * X[0] + m[1] * X[1] + m[2] * X[2] - mm * t)
    return gaugewave_oblique_fields(theta, A, m)


def sheared_flat_fields(theta, m, eps, omega: float) -> np.ndarray:
    """Flat space in the moving coordinates x = x' + eps sin(theta),
    theta = 2 pi m.x' - omega t: Jacobian J = I + eps k^T cos(theta) with
    k = 2 pi m, 3-metric J^T J, lapse 1, shift J^{-1} dx/dt, K_ij = 0.
    Every field is a function of theta alone.  Gamt^i = -d_j gt^{ij} is
    evaluated with a complex step in theta (so theta must be real here).
    B = 0."""
    theta = np.asarray(theta, dtype=float)
    f = sheared_metric(theta.astype(complex), m, eps, omega)
    y = np.zeros((24, *theta.shape))
    for q in range(24):
        y[q] = np.real(f[q])
    # Gamt^i = -sum_j k_j d/dtheta gt^{ij}
    dth = 1e-30
    gu_c = sheared_gtinv(theta + 1j * dth, m, eps)
    k = 2 * np.pi * np.asarray(m, dtype=float)
    for i in range(3):
        y[GAM + i] = -sum(k[j] * np.imag(gu_c[i][j]) / dth for j in range(3))
    return y


def _sheared_jac(theta, m, eps):
    k = 2 * np.pi * np.asarray(m, dtype=float)
    e = np.asarray(eps, dtype=float)
    c = np.cos(theta)
    J = np.zeros((*np.shape(theta), 3, 3), dtype=np.result_type(theta, float))
    for i in range(3):
        for j in range(3):
            J[..., i, j] = (1.0 if i == j else 0.0) + e[i] * k[j] * c
    return J


def sheared_gtinv(theta, m, eps):
    J = _sheared_jac(theta, m, eps)
    gam = np.swapaxes(J, -1, -2) @ J
    det = np.linalg.det(gam)
    chi = det ** (-1 / 3)
    gtu = np.linalg.inv(gam) / chi[..., None, None]
    return [[gtu[..., i, j] for j in range(3)] for i in range(3)]


def sheared_metric(theta, m, eps, omega):
    J = _sheared_jac(theta, m, eps)
    gam = np.swapaxes(J, -1, -2) @ J
    det = np.linalg.det(gam)
    chi = det ** (-1 / 3)
    e = np.asarray(eps, dtype=float)
    xdot = np.zeros((*np.shape(theta), 3), dtype=J.dtype)
    for i in range(3):
        xdot[..., i] = -e[i] * omega * np.cos(theta)
    beta = np.linalg.solve(J, xdot[..., None])[..., 0]
    y = np.zeros((24, *np.shape(theta)), dtype=J.dtype)
    y[CHI] = chi
    for i in range(3):
        for j in range(i, 3):
            y[GT + SYM[i][j]] = chi * gam[..., i, j]
    y[ALP] = 1.0
    for i in range(3):
        y[BETA + i] = beta[..., i]
    return y


def sheared_flat(n, h, m=(1, -1, 1), eps=(0.03, -0.02, 0.025), omega: float = 2.5,
                 t: float = 0.0, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    X = _grid(n, h, origin)
    k = 2 * np.pi * np.asarray(m, dtype=float)
    theta = k[0] * X[0] + k[1] * X[1] + k[2] * X[2] - omega * t
    return sheared_flat_fields(theta, m, eps, omega)


# ----------------------------------------------------------------------------
# batch of uneven patches


def patch_list(seed: int, npatch: int = 64, lo: int = 24, hi: int = 96):
    """Seeded uneven patches: per-axis sizes uniform in [lo, hi], origins
    uniform in [0,1)^3, refinement level l in {0,1,2} with h = 2^-l / 64."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(npatch):
        n = tuple(int(v) for v in rng.integers(lo, hi + 1, size=3))
        origin = tuple(float(v) for v in rng.uniform(0.0, 1.0, size=3))
        level = int(rng.integers(0, 3))
        out.append({"n": n, "origin": origin, "level": level, "h": 2.0 ** -level / 64})
    return out
