"""Reference w-stacking imager in float64 (the oracle's O-WS part).

Test infrastructure only: the imaging library never imports, links or calls this.

It follows the method of Sec. 2 of the paper in its own order:
  1. baselines in wavelengths, (u, v, w) = uvw * nu / c  (Eq. 1 defines u, v, w in wavelengths);
     grid positions x = u / du + N/2, y = v / du + N/2 with du = 1 / (N * dl);
  2. the W taps start at floor(x + 1/2) - (W-1)/2; a visibility whose taps leave
     the grid, or whose uvw or weight is not finite, is dropped;
  3. Nw uniform w-planes over [w_lo, w_hi] (Eq. 2's integration range), each
     visibility going to the plane that holds it (Sec. 2: the nearest w-plane):
     k = clamp(floor((w - w_lo) / dw), 0, Nw-1), plane centre w_k = w_lo + (k + 1/2) dw;
  4. the separable Kaiser-Bessel kernel G (oracle.kb);
  5. convolutional gridding, Eq. 3: grid_k[p0+b][q0+a] += W_m V_m G(q0+a-x) G(p0+b-y);
  6. each plane's 2D transform with the + sign of Eq. 2 and the phase centre at N/2:
     P_k(i,j) = sum_{p,q} grid_k[p][q] exp(+2 pi i [(q-N/2)(j-N/2) + (p-N/2)(i-N/2)] / N);
  7. the w-correction and reduction of the planes (Sec. 2: each plane is phase-shifted, then
     the planes are summed; the w-term sign of Eq. 2):
     S(i,j) = sum_k P_k(i,j) exp(+2 pi i w_k (n_ij - 1));
  8. division by the kernel's Fourier transform on both axes and by the sum of
     weights (natural weighting, Sec. 4.2.1): D = Re S / (sum W * C(xi_j) C(xi_i)),
     xi_j = (j - N/2) / N.

Pixel (i, j): row i carries m_i = (i - N/2) dl, column j carries l_j = (j - N/2) dl.

The w-kernel variant (w_support = Ww >= 3, odd) reads Eq. 3's kernel G(u - u_m, v - v_m,
w - w_m) with its third argument too: a separable Kaiser-Bessel factor along w, so that each
visibility is convolved onto its Ww nearest planes instead of going to one.  Steps 3, 5, 7 and 8
then read:
  3'. Nw planes with centres w_k = w_c0 + k dw, spaced so that every kept visibility's Ww taps
      exist: dw = (w_hi - w_lo) / (Nw - Ww), w_c0 = w_lo - h dw (h = (Ww - 1)/2); a visibility
      sits at plane coordinate z = (w - w_lo) / dw + h (z = h when dw = 0; clamped to
      [h, Nw - 1 - h] for rows outside a fixed range), its first w-tap is k0 = floor(z + 1/2) - h;
  5'. it adds W_m V_m G_w(k - z) G(q0+a-x) G(p0+b-y) to plane k for k = k0 .. k0 + Ww - 1, with
      G_w the Kaiser-Bessel kernel of support Ww and shape beta_w (2.34 Ww);
  7'. the planes are stacked with their phase exp(+2 pi i w_k (n - 1)) as before;
  8'. the image is also divided by C_w(dw (n_ij - 1)), the w-kernel's Fourier transform: the
      stacked phase of a visibility is exp(2 pi i w (n - 1)) sum_j G_w(t_j) exp(2 pi i t_j dw (n-1))
      with t_j the integer-spaced w-tap offsets, and by Poisson's summation formula that sum is
      C_w(dw (n - 1)) plus aliases C_w(dw (n - 1) + m), m != 0.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np

from . import kb as _kb
from ._native import lib as _lib, ptr as _ptr

C_LIGHT = 299_792_458.0


@dataclasses.dataclass
class Params:
    n: int
    pixel_rad: float
    n_wplanes: int
    support: int
    beta: float
    w_lo: Optional[float] = None    # both None: the range comes from the data
    w_hi: Optional[float] = None
    fold: bool = False              # w-folding: a row with w < 0 is imaged as its conjugate partner
    pad: int = 1                    # grid side = pad * n; the image is the grid image's central n x n
    w_support: int = 0              # 0: nearest plane; odd >= 3: Kaiser-Bessel kernel across planes
    beta_w: Optional[float] = None  # the w-kernel's shape (None: 2.34 * w_support)

    @property
    def wbeta(self) -> float:
        return 2.34 * self.w_support if self.beta_w is None else float(self.beta_w)

    @property
    def n_grid(self) -> int:
        return self.pad * self.n

    @property
    def crop(self) -> int:
        """Offset of the image inside the transformed grid, (n_grid - n) / 2."""
        return (self.n_grid - self.n) // 2


@dataclasses.dataclass
class Prepared:
    """Steps 1-3 for every input row (arrays are full length M)."""
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    x: np.ndarray
    y: np.ndarray
    q0: np.ndarray      # int64, first tap column (meaningful where keep)
    p0: np.ndarray      # int64, first tap row
    keep: np.ndarray    # bool
    k: np.ndarray       # int64 plane index (meaningful where keep)
    w_lo: float
    w_hi: float
    dw: float
    sum_w: float
    flip: Optional[np.ndarray] = None   # rows replaced by their conjugate partner (fold)
    z: Optional[np.ndarray] = None      # w-kernel: plane coordinate of each row (k = first w-tap)
    w_c0: Optional[float] = None        # centre of plane 0 (w_lo + dw / 2 for the nearest plane)

    def centre(self, k: int) -> float:
        """Plane k's centre w_k."""
        if self.z is None:
            return self.w_lo + (k + 0.5) * self.dw
        return self.w_c0 + k * self.dw

    @property
    def n_kept(self) -> int:
        return int(self.keep.sum())


def prepare(uvw_m: np.ndarray, weights: np.ndarray, freq_hz: float, prm: Params) -> Prepared:
    """Steps 1-3: wavelength coordinates, tap origins, the keep mask and plane indices."""
    uvw_m = np.asarray(uvw_m, dtype=np.float64)
    wt = np.asarray(weights).astype(np.float64)
    n, W = prm.n_grid, prm.support
    u = uvw_m[:, 0] * freq_hz / C_LIGHT
    v = uvw_m[:, 1] * freq_hz / C_LIGHT
    w = uvw_m[:, 2] * freq_hz / C_LIGHT
    flip = np.zeros(u.shape[0], dtype=bool)
    if prm.fold:
        # w-folding: V(-u, -v, -w) = conj V(u, v, w) for a real sky, so a row with w < 0 is
        # replaced by (-u, -v, -w, conj V); the planes then span |w| only
        with np.errstate(invalid="ignore"):
            flip = uvw_m[:, 2] < 0
        u, v, w = np.where(flip, -u, u), np.where(flip, -v, v), np.where(flip, -w, w)
    du = 1.0 / (n * prm.pixel_rad)
    x = u / du + n / 2
    y = v / du + n / 2
    half = (W - 1) // 2
    with np.errstate(invalid="ignore"):
        fq = np.floor(x + 0.5) - half
        fp = np.floor(y + 0.5) - half
        finite = np.isfinite(uvw_m).all(axis=1) & np.isfinite(wt)
        keep = finite & (fq >= 0) & (fq + W - 1 <= n - 1) & (fp >= 0) & (fp + W - 1 <= n - 1)
    q0 = np.where(keep, fq, 0).astype(np.int64)
    p0 = np.where(keep, fp, 0).astype(np.int64)

    if prm.w_lo is not None and prm.w_hi is not None:
        w_lo, w_hi = float(prm.w_lo), float(prm.w_hi)
    else:
        sel = keep & (wt > 0)
        if sel.any():
            w_lo, w_hi = float(w[sel].min()), float(w[sel].max())
        else:
            w_lo = w_hi = 0.0
    sum_w = float(wt[keep].sum())
    if prm.w_support:
        # step 3': planes spaced so that the Ww w-taps of every kept row exist
        ww = int(prm.w_support)
        if ww < 3 or ww % 2 == 0 or prm.n_wplanes <= ww:
            raise ValueError("w_support must be odd, >= 3 and below n_wplanes")
        hw = (ww - 1) // 2
        dw = (w_hi - w_lo) / (prm.n_wplanes - ww)
        w_c0 = w_lo - hw * dw
        if dw == 0.0:
            z = np.full(u.shape[0], float(hw))
        else:
            with np.errstate(invalid="ignore"):
                z = (w - w_lo) / dw + hw
        # rows outside a fixed range are taken at the nearest end of the plane coordinates
        # (as the nearest-plane method clamps them to the edge planes)
        z = np.where(keep, np.clip(z, float(hw), float(prm.n_wplanes - 1 - hw)), float(hw))
        k0 = np.clip(np.floor(z + 0.5) - hw, 0, prm.n_wplanes - ww).astype(np.int64)
        return Prepared(u, v, w, x, y, q0, p0, keep, k0, w_lo, w_hi, dw, sum_w, flip, z, w_c0)
    dw = (w_hi - w_lo) / prm.n_wplanes
    if dw == 0.0:
        k = np.zeros(u.shape[0], dtype=np.int64)
    else:
        with np.errstate(invalid="ignore"):
            kf = np.floor((w - w_lo) / dw)
        kf = np.where(keep, kf, 0)
        k = np.clip(kf, 0, prm.n_wplanes - 1).astype(np.int64)
    return Prepared(u, v, w, x, y, q0, p0, keep, k, w_lo, w_hi, dw, sum_w, flip)


def plane_rows(pr: Prepared, prm: Params, plane: int):
    """The kept rows that add to a plane and the factor of each (1, or G_w(plane - z) with the
    w-kernel: rows whose first w-tap k0 satisfies k0 <= plane < k0 + Ww)."""
    if pr.z is None:
        rows = np.nonzero(pr.keep & (pr.k == plane))[0]
        return rows, np.ones(rows.size)
    ww = int(prm.w_support)
    rows = np.nonzero(pr.keep & (pr.k <= plane) & (pr.k + ww > plane))[0]
    return rows, _kb.kb(plane - pr.z[rows], ww, prm.wbeta)


def tap_weights(pr: Prepared, prm: Params, rows: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Step 4 at the taps of the given rows: gx[r, a] = G(q0+a-x), gy[r, b] = G(p0+b-y)."""
    a = np.arange(prm.support)
    gx = _kb.kb((pr.q0[rows, None] + a[None, :]) - pr.x[rows, None], prm.support, prm.beta)
    gy = _kb.kb((pr.p0[rows, None] + a[None, :]) - pr.y[rows, None], prm.support, prm.beta)
    return np.ascontiguousarray(gx), np.ascontiguousarray(gy)


def grid_plane(pr: Prepared, vis: np.ndarray, weights: np.ndarray, prm: Params, plane: int,
               chunk: int = 1 << 20) -> np.ndarray:
    """Step 5 for one w-plane: the complex float64 grid [N, N] of Eq. 3."""
    n = prm.n_grid
    grid = np.zeros((n, n, 2), dtype=np.float64)
    rows, fac = plane_rows(pr, prm, plane)
    vis = np.asarray(vis)
    wt = np.asarray(weights).astype(np.float64)
    L = _lib()
    for c0 in range(0, rows.size, chunk):
        r = rows[c0:c0 + chunk]
        vr = vis[r].astype(np.complex128)
        if pr.flip is not None:
            vr = np.where(pr.flip[r], np.conj(vr), vr)
        wv = wt[r] * vr * fac[c0:c0 + chunk]
        wv_re = np.ascontiguousarray(wv.real)
        wv_im = np.ascontiguousarray(wv.imag)
        gx, gy = tap_weights(pr, prm, r)
        idx = np.arange(r.size, dtype=np.int64)
        p0 = np.ascontiguousarray(pr.p0[r])
        q0 = np.ascontiguousarray(pr.q0[r])
        L.oracle_grid_accumulate(n, prm.support, r.size, _ptr(idx), _ptr(p0), _ptr(q0),
                                 _ptr(wv_re), _ptr(wv_im), _ptr(gx), _ptr(gy), _ptr(grid))
    return grid[..., 0] + 1j * grid[..., 1]


def _centred_phase(idx_a: np.ndarray, idx_b: np.ndarray, n: int) -> np.ndarray:
    """exp(+2 pi i (a - N/2)(b - N/2) / N) for all pairs, with the product reduced mod N exactly."""
    a = (np.asarray(idx_a, dtype=np.int64) - n // 2)[:, None]
    b = (np.asarray(idx_b, dtype=np.int64) - n // 2)[None, :]
    r = np.mod(a * b, n)
    return np.exp(2j * math.pi * (r / n))


def plane_transform(grid: np.ndarray, pixels: Optional[Tuple[Sequence[int], Sequence[int]]] = None,
                    grid_rows: Optional[np.ndarray] = None) -> np.ndarray:
    """Step 6.  Full plane: N^2 * fftshift(ifft2(ifftshift(grid))) (numpy's ifft has the + sign).

    With pixels = (rows I, cols J) the same sum is taken directly at the product set I x J
    as two matrix products over the grid rows that can be non-zero (``grid_rows``, by
    default every row holding a non-zero cell).
    """
    n = grid.shape[0]
    if pixels is None:
        return (n * n) * np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(grid)))
    rows_i, cols_j = (np.asarray(pixels[0]), np.asarray(pixels[1]))
    nz = np.nonzero(np.any(grid != 0, axis=1))[0] if grid_rows is None else np.asarray(grid_rows)
    if nz.size == 0:
        return np.zeros((rows_i.size, cols_j.size), dtype=np.complex128)
    ecol = _centred_phase(np.arange(n), cols_j, n)          # [q, j]
    erow = _centred_phase(nz, rows_i, n)                     # [p, i]
    t = grid[nz] @ ecol                                      # [p, j]
    return erow.T @ t                                        # [i, j]


def direction_cosines(n: int, pixel_rad: float, rows, cols):
    """l_j, m_i and n_ij - 1 for the product set rows x cols (float64).

    n - 1 is evaluated as -(l^2 + m^2) / (1 + sqrt(1 - l^2 - m^2)), which equals
    sqrt(1 - l^2 - m^2) - 1 without its cancellation.
    """
    lj = (np.asarray(cols, dtype=np.float64) - n // 2) * pixel_rad
    mi = (np.asarray(rows, dtype=np.float64) - n // 2) * pixel_rad
    r2 = mi[:, None] ** 2 + lj[None, :] ** 2
    if np.any(r2 >= 1.0):
        raise ValueError("pixel beyond the horizon (l^2 + m^2 >= 1)")
    nm1 = -r2 / (1.0 + np.sqrt(1.0 - r2))
    return lj, mi, nm1


def wstack_image(uvw_m, vis, weights, freq_hz: float, prm: Params,
                 pixels: Optional[Tuple[Sequence[int], Sequence[int]]] = None,
                 planes: Optional[Sequence[int]] = None, complex_out: bool = False,
                 prepared: Optional[Prepared] = None, normalize: bool = True,
                 threads: int = 1) -> np.ndarray:
    """Steps 1-8: the dirty image [N, N] (or [|I|, |J|] at pixels = (I, J)).

    ``planes`` restricts steps 5-7 to a subset of w-planes (the rest contribute
    nothing); the normalisation keeps the full sum of weights.  normalize=False leaves
    out the division by the sum of weights (the imaging operator itself).

    ``threads`` > 1 runs steps 5-7 for groups of planes in that many threads (plane k in
    group k mod threads) and adds the groups' sums in group order: the same per-plane
    arithmetic, only the order in which the planes' terms are added differs.
    """
    n = prm.n
    pr = prepared if prepared is not None else prepare(uvw_m, weights, freq_hz, prm)
    if pixels is None:
        rows = cols = np.arange(n)
    else:
        rows, cols = np.asarray(pixels[0]), np.asarray(pixels[1])
    shape = (rows.size, cols.size)
    if pr.sum_w == 0.0 and normalize:
        return np.zeros(shape, dtype=np.complex128 if complex_out else np.float64)
    _, _, nm1 = direction_cosines(n, prm.pixel_rad, rows, cols)
    plist = list(range(prm.n_wplanes) if planes is None else planes)

    def stack(group):
        """Steps 5-7 over the planes of one group: sum_k P_k exp(+2 pi i w_k (n - 1))."""
        S = np.zeros(shape, dtype=np.complex128)
        for k in group:
            prow, _ = plane_rows(pr, prm, k)
            if prow.size == 0:
                continue
            g = grid_plane(pr, vis, weights, prm, k)
            o = prm.crop
            if pixels is None:
                P = plane_transform(g)[o:o + n, o:o + n]
            else:
                lo, hi = int(pr.p0[prow].min()), int(pr.p0[prow].max()) + prm.support - 1
                P = plane_transform(g, (rows + o, cols + o), grid_rows=np.arange(lo, hi + 1))
            del g
            wk = pr.centre(k)
            cyc = wk * nm1
            cyc = cyc - np.round(cyc)
            S += P * np.exp(2j * math.pi * cyc)
        return S

    if threads <= 1 or len(plist) <= 1:
        S = stack(plist)
    else:
        from concurrent.futures import ThreadPoolExecutor
        t = min(int(threads), len(plist))
        groups = [plist[g::t] for g in range(t)]
        with ThreadPoolExecutor(t) as ex:
            parts = list(ex.map(stack, groups))
        S = parts[0]
        for q in parts[1:]:
            S += q
    xi_j = (cols - n // 2) / prm.n_grid
    xi_i = (rows - n // 2) / prm.n_grid
    corr = np.outer(_kb.kb_taper(xi_i, prm.support, prm.beta), _kb.kb_taper(xi_j, prm.support, prm.beta))
    if pr.z is not None:
        # step 8': the w-kernel's transform at dw (n - 1) (a visibility's w-tap weights sum to
        # about C_w(0), as its uv taps to C(0): dividing by C_w keeps the scale of a unit weight)
        corr = corr * _kb.kb_taper(pr.dw * nm1, prm.w_support, prm.wbeta)
    D = S / ((pr.sum_w if normalize else 1.0) * corr)
    return D if complex_out else D.real


def grid_stack(uvw_m, vis, weights, freq_hz: float, prm: Params,
               prepared: Optional[Prepared] = None) -> np.ndarray:
    """Step 5 for every plane: the complex float64 grid [Nw, pad N, pad N]."""
    pr = prepared if prepared is not None else prepare(uvw_m, weights, freq_hz, prm)
    return np.stack([grid_plane(pr, vis, weights, prm, k) for k in range(prm.n_wplanes)])


def wstack_predict(uvw_m, weights, freq_hz: float, prm: Params, image: np.ndarray,
                   prepared: Optional[Prepared] = None) -> np.ndarray:
    """Prediction (degridding): the transpose of the unnormalised imaging operator.

    With A the map z -> Re S(z) / (C(xi_i) C(xi_j)) of steps 5-8 (gridding z_m = W_m V_m,
    normalize=False), this returns y = A^T X, so that for every complex z and real X
        sum_ij A(z)_ij X_ij = Re sum_m z_m conj(y_m).
    The steps of Sec. 2 run backwards:
      8'. divide the image by the kernel's transform on both axes:  Y = X / (C(xi_i) C(xi_j));
      7'. per plane, the conjugate w-phase:  Y_k = Y exp(-2 pi i w_k (n_ij - 1));
      6'. the transform with the - sign, phase centre at N/2:
          g_k[p][q] = sum_{i,j} Y_k(i,j) exp(-2 pi i [(q-N/2)(j-N/2) + (p-N/2)(i-N/2)] / N)
                    = fftshift(fft2(ifftshift(Y_k)))   (numpy's fft has the - sign);
      5'. each kept row reads its taps:  y_m = sum_{a,b} G(q0+a-x_m) G(p0+b-y_m) g_k[p0+b][q0+a].
    Dropped rows predict 0.  ``weights`` only decide which rows are kept and the plane range
    (as in steps 2-3); they do not scale the prediction.
    """
    if prm.w_support:
        raise NotImplementedError("the prediction is the transpose of nearest-plane imaging only")
    n, ng, o = prm.n, prm.n_grid, prm.crop
    pr = prepared if prepared is not None else prepare(uvw_m, weights, freq_hz, prm)
    rows = cols = np.arange(n)
    _, _, nm1 = direction_cosines(n, prm.pixel_rad, rows, cols)
    xi = (rows - n // 2) / ng
    ck = _kb.kb_taper(xi, prm.support, prm.beta)
    Y = np.asarray(image, dtype=np.float64) / np.outer(ck, ck)
    out = np.zeros(pr.u.shape[0], dtype=np.complex128)
    L = _lib()
    for k in range(prm.n_wplanes):
        sel = np.nonzero(pr.keep & (pr.k == k))[0]
        if sel.size == 0:
            continue
        wk = pr.w_lo + (k + 0.5) * pr.dw
        cyc = wk * nm1
        cyc = cyc - np.round(cyc)
        Yk = np.zeros((ng, ng), dtype=np.complex128)
        Yk[o:o + n, o:o + n] = Y * np.exp(-2j * math.pi * cyc)     # the image inside the grid image
        g = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(Yk)))
        gri = np.ascontiguousarray(np.stack([g.real, g.imag], axis=-1))
        gx, gy = tap_weights(pr, prm, sel)
        p0 = np.ascontiguousarray(pr.p0[sel])
        q0 = np.ascontiguousarray(pr.q0[sel])
        res = np.zeros((sel.size, 2), dtype=np.float64)
        L.oracle_degrid(ng, prm.support, sel.size, _ptr(p0), _ptr(q0), _ptr(gx), _ptr(gy), _ptr(gri),
                        _ptr(res))
        out[sel] = res[:, 0] + 1j * res[:, 1]
    if pr.flip is not None:
        out = np.where(pr.flip, np.conj(out), out)     # the transpose of gridding conj(z)
    return out
