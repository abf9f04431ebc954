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
