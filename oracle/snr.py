"""Matched-filter and effective SNR from the time-domain inner product (Sec. II.B item 7).

rho_mf = <d, h> / sqrt(<h, h>);  rho_eff^2 = <d, d> - <r, r>, r = d - h.
Inner products are <a, b> = a^T C^-1 b over the retained samples of each
segment, evaluated with the whitened vectors of ``tdlik``: <a, b> =
(L^-1 a)^T (L^-1 b) (test infrastructure).
"""
from __future__ import annotations

import numpy as np

from .tdlik import Factor, whiten


def inner_products(f: Factor, d: np.ndarray, H: np.ndarray):
    """Return (<d, h_b>, <h_b, h_b>) per template row of H for one detector."""
    wd = whiten(f, d)
    wh = whiten(f, np.atleast_2d(H))
    return wh @ wd, np.sum(wh * wh, axis=-1)


def snrs(f: Factor, d: np.ndarray, H: np.ndarray):
    """Return (rho_mf, rho_eff_sq) per template row of H for one detector."""
    wd = whiten(f, d)
    wh = whiten(f, np.atleast_2d(H))
    dh = wh @ wd
    hh = np.sum(wh * wh, axis=-1)
    dd = float(wd @ wd)
    wr = wd[None, :] - wh
    rr = np.sum(wr * wr, axis=-1)
    return dh / np.sqrt(hh), dd - rr
