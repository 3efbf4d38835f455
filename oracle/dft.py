"""Direct Fourier inversion of the measurement equation (the oracle's O-DFT part).

Test infrastructure only: the imaging library never imports, links or calls this.

Eq. 1 of the paper gives V(u,v,w) as a sum over the sky of
I(l,m)/n * exp(-2 pi i (u l + v m + w (n - 1))).  Its adjoint, evaluated at a
pixel, is the plain definition of the dirty image with the exact w-term:

    S(i,j) = sum_m W_m V_m exp(+2 pi i (u_m l_j + v_m m_i + w_m (n_ij - 1)))
    D(i,j) = Re S(i,j) / sum_m W_m

(u, v, w in wavelengths; l_j = (j - N/2) dl, m_i = (i - N/2) dl).  Every input
row is used; the caller passes the rows it wants imaged.
"""

from __future__ import annotations

from typing import Optional, Sequence, Tuple

import numpy as np

from ._native import lib as _lib, ptr as _ptr
from .wstack import C_LIGHT, direction_cosines


def dft_image(uvw_m, vis, weights, freq_hz: float, n: int, pixel_rad: float,
              pixels: Optional[Tuple[Sequence[int], Sequence[int]]] = None,
              complex_out: bool = False) -> np.ndarray:
    """D (or S / sum W if complex_out) at the product set pixels = (rows, cols), default all."""
    uvw_m = np.ascontiguousarray(uvw_m, dtype=np.float64)
    wt = np.asarray(weights).astype(np.float64)
    wv = wt * np.asarray(vis).astype(np.complex128)
    u = np.ascontiguousarray(uvw_m[:, 0] * freq_hz / C_LIGHT)
    v = np.ascontiguousarray(uvw_m[:, 1] * freq_hz / C_LIGHT)
    w = np.ascontiguousarray(uvw_m[:, 2] * freq_hz / C_LIGHT)
    if pixels is None:
        rows = cols = np.arange(n)
    else:
        rows, cols = np.asarray(pixels[0]), np.asarray(pixels[1])
    lj, mi, nm1 = direction_cosines(n, pixel_rad, rows, cols)
    L = np.ascontiguousarray(np.broadcast_to(lj[None, :], nm1.shape).ravel())
    Mm = np.ascontiguousarray(np.broadcast_to(mi[:, None], nm1.shape).ravel())
    N1 = np.ascontiguousarray(nm1.ravel())
    out = np.zeros((N1.size, 2))
    wr = np.ascontiguousarray(wv.real)
    wi = np.ascontiguousarray(wv.imag)
    _lib().oracle_dft(u.size, _ptr(u), _ptr(v), _ptr(w), _ptr(wr), _ptr(wi),
                      N1.size, _ptr(L), _ptr(Mm), _ptr(N1), _ptr(out))
    S = (out[:, 0] + 1j * out[:, 1]).reshape(nm1.shape)
    sw = float(wt.sum())
    D = S / sw
    return D if complex_out else D.real
