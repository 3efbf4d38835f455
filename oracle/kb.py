"""Kaiser-Bessel gridding kernel and its Fourier transform (the grid-correction taper).

Test infrastructure only: nothing in the imaging library imports this.

The paper names a Kaiser-Bessel convolution function G (Sec. 2, the gridding
component, citing Jackson et al. 1991) without giving its form.  The reading
used here is the standard one from that reference:

    G(t) = I0(beta * sqrt(1 - (2 t / W)^2)) / I0(beta)   for |t| <= W/2, else 0,

with t in grid cells, W the (odd) support and beta the shape; G(0) = 1.
Its continuous Fourier transform, which the image is divided by, is

    C(xi) = integral G(t) exp(2 pi i t xi) dt
          = (W / I0(beta)) * sinh(sqrt(beta^2 - (pi W xi)^2)) / sqrt(beta^2 - (pi W xi)^2)

(the sin form applies when pi W |xi| > beta).  xi is in cycles per grid cell.
"""

from __future__ import annotations

import math

import numpy as np


def i0(z):
    """Modified Bessel function of the first kind, order 0, by its power series.

    I0(z) = sum_k ((z/2)^(2k)) / (k!)^2, summed until a term drops below
    1e-17 of the running sum.  Float64, elementwise on arrays.
    """
    z = np.asarray(z, dtype=np.float64)
    q = 0.25 * z * z
    term = np.ones_like(z)
    total = np.ones_like(z)
    k = 0
    while True:
        k += 1
        term = term * q / (k * k)
        total = total + term
        if np.all(term <= 1e-17 * total):
            break
        if k > 500:
            raise RuntimeError("I0 series did not converge")
    return total


def kb_numpy(t, support: int, beta: float):
    """G(t) with numpy's array arithmetic and the series of i0 above."""
    t = np.asarray(t, dtype=np.float64)
    s = 2.0 * t / support
    inside = np.abs(t) <= 0.5 * support
    arg = np.sqrt(np.clip(1.0 - s * s, 0.0, None))
    g = i0(beta * arg) / i0(np.float64(beta))
    return np.where(inside, g, 0.0)


def kb(t, support: int, beta: float):
    """G(t): the Kaiser-Bessel kernel in grid cells, normalised to G(0) = 1.

    The same formula and I0 series as kb_numpy, one offset at a time in the oracle's plain C
    helper (the series stops per offset instead of at the slowest element of the array)."""
    from ._native import lib, ptr
    t = np.asarray(t, dtype=np.float64)
    tc = np.ascontiguousarray(t.ravel())
    out = np.empty_like(tc)
    lib().oracle_kb_eval(tc.size, ptr(tc), int(support), float(beta), ptr(out))
    return out.reshape(t.shape)


def kb_taper(xi, support: int, beta: float):
    """C(xi): the continuous Fourier transform of G at xi cycles per cell."""
    xi = np.asarray(xi, dtype=np.float64)
    a2 = beta * beta - (math.pi * support * xi) ** 2
    out = np.empty_like(xi)
    pos = a2 > 0
    r = np.sqrt(np.abs(a2))
    with np.errstate(invalid="ignore", divide="ignore"):
        out[pos] = np.sinh(r[pos]) / r[pos]
        neg = a2 < 0
        out[neg] = np.sin(r[neg]) / r[neg]
    out[a2 == 0] = 1.0
    return out * (support / i0(np.float64(beta)))
