"""Shared test helpers: parity metric and grid builders for both sides."""
import numpy as np

import oracle


def parity(gpu: np.ndarray, orc: np.ndarray) -> np.ndarray:
    """Per grid function: max |gpu - orc| / max |orc| over the points given.
    A grid function that is identically zero in the oracle must be exactly
    zero on the GPU (returns inf otherwise, 0 if so)."""
    a = gpu.reshape(gpu.shape[0], -1)
    b = orc.reshape(orc.shape[0], -1)
    out = np.zeros(a.shape[0])
    for v in range(a.shape[0]):
        s = np.abs(b[v]).max()
        if s == 0:
            out[v] = 0.0 if np.abs(a[v]).max() == 0 else np.inf
        else:
            out[v] = np.abs(a[v] - b[v]).max() / s
    return out


def pair(n, g, h, system, origin=(0.0, 0.0, 0.0), precision=0, boundary=0, **kw):
    """(library grid, oracle block) describing the same block"""
    from paper_1410_1764_amd import chemora as C
    gr = C.Grid(n, g, h, origin=origin, system=system, precision=precision, boundary=boundary,
                **{k: v for k, v in kw.items() if k != "gw_d"},
                **({"gw_wavelength": kw["gw_d"]} if "gw_d" in kw else {}))
    okw = {k: v for k, v in kw.items() if k in ("slicing", "shift", "shift_F", "eta", "gw_amp",
                                                  "gw_d", "gw_axis", "ko_sigma", "enforce",
                                                  "fd_order")}
    if "gw_wavelength" in kw:
        okw["gw_d"] = kw["gw_wavelength"]
    return gr, oracle.Block(n, g, h, origin, **okw)


# BSSN tensors (grid-function index ranges): chi, gt_ij, trK, At_ij, Gamt^i,
# alpha, beta^i, B^i
BSSN_TENSORS = ((0, 1), (1, 7), (7, 8), (8, 14), (14, 17), (17, 18), (18, 21), (21, 24))


def parity_tensor(gpu: np.ndarray, orc: np.ndarray) -> np.ndarray:
    """Per grid function: max |gpu - orc| over the points given, divided by
    the largest |orc| of any component of the same BSSN tensor.  A component
    that is tiny next to the other components of its tensor (an off-diagonal
    metric term that is zero but for ~1e-10 boundary mismatches) is measured
    against the tensor's size, not its own.  A tensor that is identically
    zero in the oracle must be exactly zero on the GPU (inf otherwise)."""
    a = gpu.reshape(gpu.shape[0], -1)
    b = orc.reshape(orc.shape[0], -1)
    out = np.zeros(a.shape[0])
    for lo, hi in BSSN_TENSORS:
        s = max(np.abs(b[v]).max() for v in range(lo, hi))
        for v in range(lo, hi):
            if s == 0:
                out[v] = 0.0 if np.abs(a[v]).max() == 0 else np.inf
            else:
                out[v] = np.abs(a[v] - b[v]).max() / s
    return out


def increment_error(gpu: np.ndarray, orc: np.ndarray, y0: np.ndarray) -> np.ndarray:
    """Per grid function: max |(gpu - y0) - (orc - y0)| / max |orc - y0|, the
    error of the change over the run relative to that change (absolute where
    the oracle's change is exactly zero)."""
    out = np.zeros(gpu.shape[0])
    for v in range(gpu.shape[0]):
        d_orc = orc[v] - y0[v]
        e = np.abs((gpu[v] - y0[v]) - d_orc).max()
        s = np.abs(d_orc).max()
        out[v] = e / s if s else e
    return out


def increment_error_tensor(gpu: np.ndarray, orc: np.ndarray, y0: np.ndarray) -> np.ndarray:
    """Per grid function: max |(gpu - y0) - (orc - y0)| divided by the
    largest change max |orc - y0| of any component of the same BSSN tensor
    (absolute where the whole tensor is unchanged)."""
    out = np.zeros(gpu.shape[0])
    for lo, hi in BSSN_TENSORS:
        s = max(np.abs(orc[v] - y0[v]).max() for v in range(lo, hi))
        for v in range(lo, hi):
            e = np.abs(gpu[v] - orc[v]).max()
            out[v] = e / s if s else e
    return out
