"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine, a closed form, a brute-force sum written out differently, an exact
identity of the measurement equation, or a bound derived from the kernel's
Fourier transform.  Each is chosen so that a plausible slip in the oracle
(wrong sign, swapped axes, tap origin off by one, missing normalisation,
wrong plane centre) fails at least one of them.
"""

import math
import os

import numpy as np
import pytest

C = 299_792_458.0
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _prm(oracle, n, dl, nw, W=7, beta=None, w_lo=None, w_hi=None):
    return oracle.Params(n=n, pixel_rad=dl, n_wplanes=nw, support=W,
                         beta=2.34 * W if beta is None else beta, w_lo=w_lo, w_hi=w_hi)


def _alias_ratio(oracle, xi, W, beta):
    """sum_{k != 0} |C(xi + k)| / |C(xi)|: the aliasing of a grid with no padding."""
    xi = np.asarray(xi, dtype=np.float64)
    ks = np.concatenate([np.arange(-40, 0), np.arange(1, 41)])
    al = np.abs(oracle.kb.kb_taper(xi[..., None] + ks, W, beta)).sum(-1)
    return al / np.abs(oracle.kb.kb_taper(xi, W, beta))


def _random_uv(rng, m, n, dl, freq, W, wscale=0.0, frac=0.35):
    """uvw in metres whose taps stay on an N grid: |u|, |v| < frac * N cells."""
    du = 1.0 / (n * dl)
    lam = C / freq
    uv = rng.uniform(-frac * n, frac * n, size=(m, 2)) * du * lam
    w = rng.normal(0.0, 1.0, size=m) * wscale * lam
    return np.column_stack([uv, w])


# ---------------------------------------------------------------------------
# the kernel and its transform

def test_i0_matches_library(oracle_mod):
    from scipy.special import i0 as sp_i0
    z = np.linspace(0.0, 30.0, 301)
    got = oracle_mod.kb.i0(z)
    assert np.max(np.abs(got / sp_i0(z) - 1.0)) < 1e-14


def test_kb_native_matches_numpy_series(oracle_mod):
    """The kernel evaluated in the C helper equals the numpy series of the same formula."""
    rng = np.random.default_rng(3)
    for W in (3, 7, 9, 15):
        t = rng.uniform(-W / 2 - 0.5, W / 2 + 0.5, 20000)
        t[:3] = (-W / 2, 0.0, W / 2)
        got = oracle_mod.kb.kb(t, W, 2.34 * W)
        ref = oracle_mod.kb.kb_numpy(t, W, 2.34 * W)
        assert np.max(np.abs(got - ref)) <= 1e-15


def test_kb_shape(oracle_mod):
    kbm = oracle_mod.kb
    for W in (7, 9):
        beta = 2.34 * W
        assert kbm.kb(0.0, W, beta) == pytest.approx(1.0, abs=1e-15)
        t = np.linspace(-W / 2, W / 2, 101)
        g = kbm.kb(t, W, beta)
        assert np.allclose(g, g[::-1], rtol=1e-13, atol=0)
        # edge value 1/I0(beta): 7.7e-7 for W=7, 8.2e-9 for W=9
        from scipy.special import i0 as sp_i0
        assert kbm.kb(W / 2, W, beta) == pytest.approx(1.0 / sp_i0(beta), rel=1e-13)
        assert kbm.kb(W / 2 + 1e-9, W, beta) == 0.0
        assert np.all(np.diff(g[50:]) < 0)


@pytest.mark.parametrize("W", [7, 9])
def test_taper_closed_form_against_quadrature(oracle_mod, W):
    """P9: C(xi) against 64-point Gauss-Legendre quadrature of the kernel's transform."""
    kbm = oracle_mod.kb
    beta = 2.34 * W
    x, wq = np.polynomial.legendre.leggauss(64)
    t = 0.5 * W * x
    g = kbm.kb(t, W, beta)
    c0 = kbm.kb_taper(0.0, W, beta)
    # includes the sin branch (pi W xi > beta) at xi = 0.8 and 1.3
    for xi in (0.0, 0.1, 0.25, 0.4, 0.5, 0.8, 1.3, -0.37):
        quad = 0.5 * W * np.sum(wq * g * np.cos(2 * math.pi * t * xi))
        assert abs(kbm.kb_taper(xi, W, beta) - quad) < 1e-12 * c0, xi


# ---------------------------------------------------------------------------
# steps 1-3: taps and planes, against independent formulations

def test_tap_origin_is_the_support_window(oracle_mod):
    """Step 2: the W taps are exactly the cells c with |c - x| < W/2 (brute force)."""
    rng = np.random.default_rng(1)
    n, dl, f, W = 64, 1e-3, 1e9, 7
    uvw = _random_uv(rng, 500, n, dl, f, W)
    prm = _prm(oracle_mod, n, dl, 1, W)
    pr = oracle_mod.prepare(uvw, np.ones(500), f, prm)
    for r in range(500):
        cells = [c for c in range(n) if abs(c - pr.x[r]) < W / 2]
        assert cells == list(range(pr.q0[r], pr.q0[r] + W))
        rows = [c for c in range(n) if abs(c - pr.y[r]) < W / 2]
        assert rows == list(range(pr.p0[r], pr.p0[r] + W))


def test_plane_is_the_nearest_centre(oracle_mod):
    """Step 3: k is the plane whose centre w_k is nearest to w (brute-force argmin)."""
    rng = np.random.default_rng(2)
    n, dl, f = 64, 1e-3, 1e9
    uvw = _random_uv(rng, 2000, n, dl, f, 7, wscale=300.0)
    for nw in (1, 3, 8, 32):
        prm = _prm(oracle_mod, n, dl, nw)
        pr = oracle_mod.prepare(uvw, np.ones(2000), f, prm)
        centres = pr.w_lo + (np.arange(nw) + 0.5) * pr.dw
        nearest = np.argmin(np.abs(pr.w[:, None] - centres[None, :]), axis=1)
        assert np.array_equal(nearest, pr.k)
        assert pr.k[np.argmax(pr.w)] == nw - 1 and pr.k[np.argmin(pr.w)] == 0


def test_drops_and_degenerate_range(oracle_mod):
    n, dl, f, W = 32, 1e-3, 1e9, 7
    du = 1.0 / (n * dl)
    lam = C / f
    uvw = np.zeros((6, 3))
    uvw[1, 0] = (n / 2 - 4.0) * du * lam       # x = N-4: last tap at N-1, kept
    uvw[2, 0] = (n / 2 - 3.4) * du * lam       # x = N-3.4: a tap at N, dropped
    uvw[3, 1] = -(n / 2 - 3.0) * du * lam      # y = 3: first tap row 0, kept
    uvw[4, 2] = np.nan                          # non-finite: dropped
    wts = np.array([1.0, 1.0, 1.0, 1.0, 1.0, np.inf])
    prm = _prm(oracle_mod, n, dl, 4, W)
    pr = oracle_mod.prepare(uvw, wts, f, prm)
    assert pr.keep.tolist() == [True, True, False, True, False, False]
    assert pr.q0[1] + W - 1 == n - 1 and pr.p0[3] == 0
    assert pr.sum_w == 3.0
    assert pr.dw == 0.0 and np.all(pr.k == 0)          # every kept w is 0
    # nothing kept: the image is zero
    img = oracle_mod.wstack_image(uvw[[2, 4]], wts[[2, 4]], wts[[2, 4]], f, prm)
    assert not np.any(img)


# ---------------------------------------------------------------------------
# steps 4-6: the tap-sum invariant and the plane transform

@pytest.mark.parametrize("W,bound", [(7, 1.0e-6), (9, 5.0e-9)])
def test_tap_sum_invariant(oracle_mod, W, bound):
    """P10: by Poisson summation, sum_a G(q0+a-x) = C(0) (1 + e), |e| <= 2 sum_{k>=1}|C(k)|/C(0)."""
    kbm = oracle_mod.kb
    beta = 2.34 * W
    rng = np.random.default_rng(3)
    n, dl, f = 128, 1e-3, 1e9
    uvw = _random_uv(rng, 4000, n, dl, f, W)
    prm = _prm(oracle_mod, n, dl, 1, W)
    pr = oracle_mod.prepare(uvw, np.ones(4000), f, prm)
    gx, gy = oracle_mod.wstack.tap_weights(pr, prm, np.arange(4000))
    c0 = kbm.kb_taper(0.0, W, beta)
    poisson = 2 * np.sum(np.abs(kbm.kb_taper(np.arange(1, 20000), W, beta))) / c0
    assert poisson < bound
    for g in (gx, gy):
        e = g.sum(axis=1) / c0 - 1.0
        assert np.max(np.abs(e)) <= poisson * (1 + 1e-9) + 1e-14


def test_plane_transform_against_brute_force(oracle_mod):
    """P8: step 6 against the double sum over cells written out, and the sampled form."""
    rng = np.random.default_rng(4)
    for n in (8, 16, 32):
        g = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        P = oracle_mod.plane_transform(g)
        ref = np.zeros((n, n), complex)
        for i in range(n):
            for j in range(n):
                acc = 0j
                for p in range(n):
                    for q in range(n):
                        acc += g[p, q] * np.exp(2j * math.pi * ((q - n / 2) * (j - n / 2)
                                                                 + (p - n / 2) * (i - n / 2)) / n)
                ref[i, j] = acc
        assert np.max(np.abs(P - ref)) < 1e-12 * np.max(np.abs(ref))
        I, J = np.array([0, 3, n - 1]), np.array([1, n // 2, n - 2, 5])
        S = oracle_mod.plane_transform(g, (I, J))
        assert np.max(np.abs(S - P[np.ix_(I, J)])) < 1e-12 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# whole-method pins

def test_unit_visibility_at_origin_gives_flat_image(oracle_mod):
    """P1: one unit visibility at uvw = 0.  The DFT image is exactly 1; the w-stacking
    image is the ratio of the sampled kernel's Fourier series to its transform, which is
    1 within 3.3e-6 per axis for |xi| <= 1/4 (W = 7)."""
    kbm = oracle_mod.kb
    n, dl, f, W = 64, 2e-3, 1e9, 7
    beta = 2.34 * W
    uvw = np.zeros((1, 3))
    prm = _prm(oracle_mod, n, dl, 4, W)
    D = oracle_mod.wstack_image(uvw, np.ones(1), np.ones(1), f, prm, complex_out=True)
    Dd = oracle_mod.dft_image(uvw, np.ones(1), np.ones(1), f, n, dl, complex_out=True)
    assert np.max(np.abs(Dd - 1.0)) < 1e-15
    # the 7 taps sit at integer offsets t = -3..3; their Fourier series, axis by axis
    t = np.arange(W) - (W - 1) // 2
    xi = (np.arange(n) - n // 2) / n
    series = (kbm.kb(t, W, beta)[None, :] * np.cos(2 * math.pi * np.outer(xi, t))).sum(1)
    ratio = series / kbm.kb_taper(xi, W, beta)
    assert np.max(np.abs(D - np.outer(ratio, ratio))) < 1e-13 * np.max(np.abs(D))
    inner = slice(n // 4, 3 * n // 4 + 1)
    assert np.max(np.abs(D[inner, inner] - 1.0)) < 7e-6
    assert np.max(np.abs(D.imag)) < 1e-13


def test_point_source_at_phase_centre(oracle_mod, c1):
    """P2: V = 1 everywhere images to exactly 1 at the centre (DFT) and to 1 within the
    tap-sum deviation for w-stacking; random positive weights exercise the normalisation."""
    rng = np.random.default_rng(5)
    ds = c1.subset(slice(0, 4000))
    wts = rng.uniform(0.5, 2.0, ds.m)
    vis = np.ones(ds.m, complex)
    n = ds.n
    prm = _prm(oracle_mod, n, ds.pixel_rad, ds.n_wplanes, ds.support)
    px = (np.array([n // 2]), np.array([n // 2]))
    Dd = oracle_mod.dft_image(ds.uvw_m, vis, wts, ds.freq_hz, n, ds.pixel_rad, pixels=px)
    Dw = oracle_mod.wstack_image(ds.uvw_m, vis, wts, ds.freq_hz, prm, pixels=px)
    assert abs(Dd[0, 0] - 1.0) < 1e-13
    assert abs(Dw[0, 0] - 1.0) < 2e-6


def _point_source_vis(uvw_m, freq, l0, m0, flux):
    u, v, w = (uvw_m * freq / C).T
    n0 = math.sqrt(1 - l0 * l0 - m0 * m0)
    return (flux / n0) * np.exp(-2j * math.pi * (u * l0 + v * m0 + w * (n0 - 1))), n0


def test_point_source_off_centre(oracle_mod, c1):
    """P3: a source at the centre of pixel (i0, j0) images to F/n0 there (DFT exactly;
    w-stacking within pi*dw*|n0-1| plus the aliasing bound), the peak sits on that pixel,
    and the w-correction shrinks the error as planes are added."""
    ds = c1
    n, dl = ds.n, ds.pixel_rad
    i0, j0 = n // 2 - 37, n // 2 + 20          # distinct offsets: catches swapped axes and signs
    l0, m0 = (j0 - n // 2) * dl, (i0 - n // 2) * dl
    F = 0.7
    vis, n0 = _point_source_vis(ds.uvw_m, ds.freq_hz, l0, m0, F)
    wts = np.ones(ds.m)
    rows = np.arange(i0 - 3, i0 + 4)
    cols = np.arange(j0 - 3, j0 + 4)
    Dd = oracle_mod.dft_image(ds.uvw_m, vis, wts, ds.freq_hz, n, dl, pixels=(rows, cols))
    assert abs(Dd[3, 3] - F / n0) < 1e-12
    assert np.unravel_index(np.argmax(Dd), Dd.shape) == (3, 3)
    errs = {}
    xi = np.array([(j0 - n // 2) / n, (i0 - n // 2) / n])
    alias = _alias_ratio(oracle_mod, xi, ds.support, ds.beta).sum()
    for nw in (1, 4, 16):
        prm = _prm(oracle_mod, n, dl, nw, ds.support)
        Dw = oracle_mod.wstack_image(ds.uvw_m, vis, wts, ds.freq_hz, prm, pixels=(rows, cols))
        assert np.unravel_index(np.argmax(Dw), Dw.shape) == (3, 3)
        pr = oracle_mod.prepare(ds.uvw_m, wts, ds.freq_hz, prm)
        bound = math.pi * pr.dw * abs(n0 - 1) + alias + 1e-9
        errs[nw] = abs(Dw[3, 3] * n0 / F - 1.0)
        assert errs[nw] <= bound, (nw, errs[nw], bound)
    assert errs[16] < errs[4] < errs[1]


def test_linearity(oracle_mod, c1):
    """P4."""
    rng = np.random.default_rng(6)
    ds = c1.subset(slice(0, 8000))
    v2 = rng.normal(size=ds.m) + 1j * rng.normal(size=ds.m)
    prm = _prm(oracle_mod, ds.n, ds.pixel_rad, ds.n_wplanes, ds.support)
    a, b = 0.3 - 1.1j, 2.5
    # complex coefficients act on the complex image; the real image is its real part
    S1 = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, prm, complex_out=True)
    S2 = oracle_mod.wstack_image(ds.uvw_m, v2, ds.weights, ds.freq_hz, prm, complex_out=True)
    S12 = oracle_mod.wstack_image(ds.uvw_m, a * ds.vis + b * v2, ds.weights, ds.freq_hz, prm,
                                  complex_out=True)
    assert np.max(np.abs(S12 - (a * S1 + b * S2))) < 1e-12 * np.max(np.abs(S12))


def test_shift_theorem_coplanar(oracle_mod, c1):
    """P5: with w = 0, multiplying V by exp(-2 pi i (u l0 + v m0)) for whole-pixel (l0, m0)
    shifts the DFT image exactly, and the w-stacking image within the aliasing bound."""
    ds = c1.subset(slice(0, 6000))
    uvw = ds.uvw_m.copy()
    uvw[:, 2] = 0.0
    n, dl = ds.n, ds.pixel_rad
    di, dj = 9, -14
    u, v, _ = (uvw * ds.freq_hz / C).T
    vs = ds.vis * np.exp(-2j * math.pi * (u * dj * dl + v * di * dl))
    rows = np.arange(n // 2 - 30, n // 2 + 30, 3)
    cols = np.arange(n // 2 - 30, n // 2 + 30, 4)
    D0 = oracle_mod.dft_image(uvw, ds.vis, ds.weights, ds.freq_hz, n, dl, pixels=(rows, cols))
    D1 = oracle_mod.dft_image(uvw, vs, ds.weights, ds.freq_hz, n, dl, pixels=(rows + di, cols + dj))
    assert np.max(np.abs(D1 - D0)) < 1e-11 * np.max(np.abs(D0))
    prm = _prm(oracle_mod, n, dl, 1, ds.support)
    W0 = oracle_mod.wstack_image(uvw, ds.vis, ds.weights, ds.freq_hz, prm, pixels=(rows, cols))
    W1 = oracle_mod.wstack_image(uvw, vs, ds.weights, ds.freq_hz, prm, pixels=(rows + di, cols + dj))
    tol = 4 * _alias_ratio(oracle_mod, 0.2, ds.support, ds.beta) * np.max(np.abs(D0))
    assert np.max(np.abs(W1 - W0)) < tol


def test_hermitian_completion_is_real(oracle_mod, c1):
    """P6: adding (-uvw, conj V) for every row makes S real for both oracles."""
    ds = c1.subset(slice(0, 3000))
    uvw = np.concatenate([ds.uvw_m, -ds.uvw_m])
    vis = np.concatenate([ds.vis, np.conj(ds.vis)])
    wts = np.concatenate([ds.weights, ds.weights])
    n = ds.n
    prm = _prm(oracle_mod, n, ds.pixel_rad, ds.n_wplanes, ds.support)
    S = oracle_mod.wstack_image(uvw, vis, wts, ds.freq_hz, prm, complex_out=True)
    assert np.max(np.abs(S.imag)) < 1e-10 * np.max(np.abs(S.real))
    rows = np.arange(0, n, 17)
    Sd = oracle_mod.dft_image(uvw, vis, wts, ds.freq_hz, n, ds.pixel_rad, pixels=(rows, rows),
                              complex_out=True)
    assert np.max(np.abs(Sd.imag)) < 1e-12 * np.max(np.abs(Sd.real))


def test_coplanar_reduction_matches_brute_force(oracle_mod):
    """P7: with w = 0 and one plane, w-stacking is 2D KB gridding plus the centred 2D
    Fourier sum; checked here against a hand-written double sum at N = 16."""
    kbm = oracle_mod.kb
    rng = np.random.default_rng(7)
    n, dl, f, W = 16, 4e-3, 1e9, 7
    beta = 2.34 * W
    uvw = _random_uv(rng, 40, n, dl, f, W, frac=0.2)
    uvw[:, 2] = 0.0
    vis = rng.normal(size=40) + 1j * rng.normal(size=40)
    wts = rng.uniform(0.1, 1.0, 40)
    prm = _prm(oracle_mod, n, dl, 1, W)
    D = oracle_mod.wstack_image(uvw, vis, wts, f, prm, complex_out=True)
    du = 1.0 / (n * dl)
    x = uvw[:, 0] * f / C / du + n / 2
    y = uvw[:, 1] * f / C / du + n / 2
    ref = np.zeros((n, n), complex)
    for r in range(40):
        for p in range(n):
            for q in range(n):
                g = kbm.kb(q - x[r], W, beta) * kbm.kb(p - y[r], W, beta)
                if g == 0.0:
                    continue
                ph = np.exp(2j * math.pi * ((q - n / 2) * (np.arange(n)[None, :] - n / 2)
                                            + (p - n / 2) * (np.arange(n)[:, None] - n / 2)) / n)
                ref += wts[r] * vis[r] * g * ph
    xi = (np.arange(n) - n / 2) / n
    ref /= wts.sum() * np.outer(kbm.kb_taper(xi, W, beta), kbm.kb_taper(xi, W, beta))
    assert np.max(np.abs(D - ref)) < 1e-12 * np.max(np.abs(ref))


def test_nw_convergence_and_alias_floor(oracle_mod, c1):
    """P11/P12: against the DFT on the inner half, the error falls as planes are added
    and ends near the aliasing-plus-quantisation floor."""
    ds = c1
    n = ds.n
    rows = np.arange(n // 4, 3 * n // 4, 4)
    cols = np.arange(n // 4 + 1, 3 * n // 4, 4)
    Dd = oracle_mod.dft_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, n, ds.pixel_rad,
                              pixels=(rows, cols))
    # doubling from two planes halves the largest w-quantisation error at every step
    # (one plane centred near w = 0 is a special case that is not part of the sequence)
    errs = []
    for nw in (2, 4, 8, 16, 32, 64, 128):
        prm = _prm(oracle_mod, n, ds.pixel_rad, nw, ds.support)
        Dw = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, prm, pixels=(rows, cols))
        errs.append(np.linalg.norm(Dw - Dd) / np.linalg.norm(Dd))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-5, errs


def test_permutation_and_weight_scale_invariance(oracle_mod, c1):
    """P13."""
    rng = np.random.default_rng(8)
    ds = c1.subset(slice(0, 10000))
    prm = _prm(oracle_mod, ds.n, ds.pixel_rad, ds.n_wplanes, ds.support)
    D = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, prm)
    perm = rng.permutation(ds.m)
    Dp = oracle_mod.wstack_image(ds.uvw_m[perm], ds.vis[perm], ds.weights[perm], ds.freq_hz, prm)
    Ds = oracle_mod.wstack_image(ds.uvw_m, ds.vis, 3.7 * ds.weights, ds.freq_hz, prm)
    scale = np.max(np.abs(D))
    assert np.max(np.abs(Dp - D)) < 1e-14 * ds.m ** 0.5 * scale
    assert np.max(np.abs(Ds - D)) < 1e-13 * scale


def test_grid_memory_matches_paper(oracle_mod):
    """P14: the paper's 8192^2 x 32-plane grid takes 32 GB (Sec. 4.2.1), i.e. 16 B per
    cell: a complex float64 grid, which is what the oracle's grid holds."""
    with open(os.path.join(GOLDEN, "paper_grid_bytes.txt")) as fh:
        vals = dict(line.split("=") for line in fh.read().split("\n") if "=" in line and not line.startswith("#"))
    n, nw, nbytes = int(vals["n"]), int(vals["n_wplanes"]), int(vals["bytes"])
    g = oracle_mod.grid_plane(oracle_mod.prepare(np.zeros((1, 3)), np.ones(1), 1e9,
                                                 _prm(oracle_mod, 16, 1e-3, 1)),
                              np.ones(1), np.ones(1), _prm(oracle_mod, 16, 1e-3, 1), 0)
    assert nw * n * n * g.itemsize == nbytes


def test_wide_field_point_source_dft(oracle_mod):
    """P3 at a wide field, where n - 1 is far from its small-angle form: the DFT image of a
    source at a pixel centre is F/n0 there, for visibilities with a large w-term."""
    rng = np.random.default_rng(9)
    n, dl, f = 32, 0.02, 1e9
    uvw = _random_uv(rng, 3000, n, dl, f, 7, wscale=2000.0)
    i0, j0 = n // 2 - 7, n // 2 + 5
    l0, m0 = (j0 - n // 2) * dl, (i0 - n // 2) * dl
    vis, n0 = _point_source_vis(uvw, f, l0, m0, 1.3)
    assert abs(n0 - 1.0) > 0.01
    D = oracle_mod.dft_image(uvw, vis, np.ones(3000), f, n, dl)
    assert abs(D[i0, j0] - 1.3 / n0) < 1e-12
    assert np.unravel_index(np.argmax(D), D.shape) == (i0, j0)


# ---------------------------------------------------------------------------------------
# the prediction (degridding) operator: the transpose of the unnormalised imager

def test_predict_is_the_transpose_of_imaging(oracle_mod, c1):
    """P15: <A z, X> = Re <z, P X> for random complex z and real X, with A the unnormalised
    oracle imager (steps 5-8) and P the oracle prediction.  A sign error in any phase, a
    transposed axis or a missing taper factor in P breaks the identity."""
    rng = np.random.default_rng(31)
    ds = c1.subset(slice(0, 20000))
    prm = _prm(oracle_mod, ds.n, ds.pixel_rad, ds.n_wplanes, ds.support)
    ones = np.ones(ds.m)
    z = rng.normal(size=ds.m) + 1j * rng.normal(size=ds.m)
    X = rng.normal(size=(ds.n, ds.n))
    A = oracle_mod.wstack_image(ds.uvw_m, z, ones, ds.freq_hz, prm, normalize=False)
    y = oracle_mod.wstack_predict(ds.uvw_m, ones, ds.freq_hz, prm, X)
    lhs = float(np.sum(A * X))
    rhs = float(np.real(np.sum(z * np.conj(y))))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    # the normalised image is the unnormalised one over the sum of weights
    D = oracle_mod.wstack_image(ds.uvw_m, z, ones, ds.freq_hz, prm)
    assert np.max(np.abs(D * ds.m - A)) <= 1e-12 * np.max(np.abs(A))


def test_predict_point_sources(oracle_mod, c1):
    """P16: a unit point at the phase centre predicts 1 on every kept row and 0 on dropped
    ones; a unit point at pixel (i0, j0) predicts exp(-2 pi i (u l + v m + w_k (n - 1))) with
    w_k the row's plane centre (the method's w approximation), both within the kernel's
    aliasing error (Poisson summation of the tap sums: below 1e-5 here)."""
    ds = c1
    prm = _prm(oracle_mod, ds.n, ds.pixel_rad, ds.n_wplanes, ds.support)
    ones = np.ones(ds.m)
    pr = oracle_mod.prepare(ds.uvw_m, ones, ds.freq_hz, prm)
    n = ds.n
    X0 = np.zeros((n, n))
    X0[n // 2, n // 2] = 1.0
    y0 = oracle_mod.wstack_predict(ds.uvw_m, ones, ds.freq_hz, prm, X0, prepared=pr)
    assert np.max(np.abs(y0[pr.keep] - 1.0)) < 1e-5
    assert np.all(y0[~pr.keep] == 0)
    i0, j0 = n // 2 + 17, n // 2 - 40
    X1 = np.zeros((n, n))
    X1[i0, j0] = 1.0
    y1 = oracle_mod.wstack_predict(ds.uvw_m, ones, ds.freq_hz, prm, X1, prepared=pr)
    l0, m0 = (j0 - n // 2) * ds.pixel_rad, (i0 - n // 2) * ds.pixel_rad
    nm1 = -(l0 * l0 + m0 * m0) / (1.0 + math.sqrt(1.0 - l0 * l0 - m0 * m0))
    wk = pr.w_lo + (pr.k + 0.5) * pr.dw
    expect = np.exp(-2j * math.pi * (pr.u * l0 + pr.v * m0 + wk * nm1))
    assert np.max(np.abs(y1[pr.keep] - expect[pr.keep])) < 1e-5
    # and the same point with the row's own w is off by the plane quantisation only
    exact = np.exp(-2j * math.pi * (pr.u * l0 + pr.v * m0 + pr.w * nm1))
    dphi = 2 * math.pi * np.abs(pr.w - wk) * abs(nm1)
    assert np.all(np.abs(y1[pr.keep] - exact[pr.keep]) <= dphi[pr.keep] + 1e-5)


# ---------------------------------------------------------------------------------------
# w-folding (an accuracy variant): rows with w < 0 taken as their conjugate partners

def test_fold_is_the_conjugate_partner(oracle_mod, c1):
    """P17: folding equals flipping the rows by hand, (u, v, w, V) -> (-u, -v, -w, conj V)
    for w < 0, and imaging without folding; every kept w is then >= 0; the prediction with
    folding stays the transpose of the folded imager."""
    ds = c1.subset(slice(0, 30000))
    prm_f = _prm(oracle_mod, ds.n, ds.pixel_rad, ds.n_wplanes, ds.support)
    prm_f.fold = True
    prm = _prm(oracle_mod, ds.n, ds.pixel_rad, ds.n_wplanes, ds.support)
    neg = ds.uvw_m[:, 2] < 0
    assert 0 < neg.sum() < ds.m
    uvw2 = np.where(neg[:, None], -ds.uvw_m, ds.uvw_m)
    vis2 = np.where(neg, np.conj(ds.vis), ds.vis)
    Df = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, prm_f)
    Dh = oracle_mod.wstack_image(uvw2, vis2, ds.weights, ds.freq_hz, prm)
    assert np.max(np.abs(Df - Dh)) <= 1e-13 * np.max(np.abs(Dh))
    pr = oracle_mod.prepare(ds.uvw_m, ds.weights, ds.freq_hz, prm_f)
    assert pr.w_lo >= 0 and np.all(pr.w[pr.keep] >= 0)
    rng = np.random.default_rng(51)
    z = rng.normal(size=ds.m) + 1j * rng.normal(size=ds.m)
    X = rng.normal(size=(ds.n, ds.n))
    ones = np.ones(ds.m)
    A = oracle_mod.wstack_image(ds.uvw_m, z, ones, ds.freq_hz, prm_f, normalize=False)
    y = oracle_mod.wstack_predict(ds.uvw_m, ones, ds.freq_hz, prm_f, X)
    lhs, rhs = float(np.sum(A * X)), float(np.real(np.sum(z * np.conj(y))))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_fold_reduces_the_w_error(oracle_mod, c1):
    """P18: at the same number of planes, folding halves the w range per plane, so the
    w-stacked image moves closer to the direct DFT of Eq. 1 (inner half of the image)."""
    ds = c1
    Dd = oracle_mod.dft_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, ds.n, ds.pixel_rad)
    c = slice(ds.n // 4, 3 * ds.n // 4)
    errs = []
    for fold in (False, True):
        prm = _prm(oracle_mod, ds.n, ds.pixel_rad, ds.n_wplanes, ds.support)
        prm.fold = fold
        D = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, prm)
        errs.append(np.linalg.norm((D - Dd)[c, c]) / np.linalg.norm(Dd[c, c]))
    assert errs[1] < 0.7 * errs[0], errs


# ---------------------------------------------------------------------------------------
# grid padding x2 (an accuracy variant): the image is the central crop of a 2n grid

def test_padded_unit_visibility_is_flat_everywhere(oracle_mod):
    """P19: with a 2n grid the taper is only evaluated for |xi| <= 1/4, so the image of one
    unit visibility at uvw = 0 is the closed-form ratio (kernel Fourier series over its
    transform, at xi = (j - n/2) / 2n) on every pixel, and within 7e-6 of 1 everywhere."""
    kbm = oracle_mod.kb
    n, dl, f, W = 64, 2e-3, 1e9, 7
    beta = 2.34 * W
    prm = _prm(oracle_mod, n, dl, 4, W)
    prm.pad = 2
    D = oracle_mod.wstack_image(np.zeros((1, 3)), np.ones(1), np.ones(1), f, prm, complex_out=True)
    t = np.arange(W) - (W - 1) // 2
    xi = (np.arange(n) - n // 2) / (2 * n)
    series = (kbm.kb(t, W, beta)[None, :] * np.cos(2 * math.pi * np.outer(xi, t))).sum(1)
    ratio = series / kbm.kb_taper(xi, W, beta)
    assert np.max(np.abs(D - np.outer(ratio, ratio))) < 1e-13
    assert np.max(np.abs(D - 1.0)) < 7e-6


def test_padding_removes_the_edge_aliasing(oracle_mod, c1):
    """P20: against the direct DFT of Eq. 1, padding leaves the inner-half error (set by the
    w planes) unchanged and cuts the full-image error (the edge aliasing of an unpadded
    grid) by more than 20x; the padded prediction stays the transpose of the padded imager."""
    ds = c1
    Dd = oracle_mod.dft_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, ds.n, ds.pixel_rad)
    c = slice(ds.n // 4, 3 * ds.n // 4)
    inner, full = [], []
    for pad in (1, 2):
        prm = _prm(oracle_mod, ds.n, ds.pixel_rad, ds.n_wplanes, ds.support)
        prm.pad = pad
        D = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, prm)
        inner.append(np.linalg.norm((D - Dd)[c, c]) / np.linalg.norm(Dd[c, c]))
        full.append(np.linalg.norm(D - Dd) / np.linalg.norm(Dd))
    assert abs(inner[1] - inner[0]) < 0.1 * inner[0]
    assert full[1] < full[0] / 20, full
    sub = ds.subset(slice(0, 20000))
    prm = _prm(oracle_mod, sub.n, sub.pixel_rad, sub.n_wplanes, sub.support)
    prm.pad = 2
    prm.fold = True
    rng = np.random.default_rng(61)
    z = rng.normal(size=sub.m) + 1j * rng.normal(size=sub.m)
    X = rng.normal(size=(sub.n, sub.n))
    ones = np.ones(sub.m)
    A = oracle_mod.wstack_image(sub.uvw_m, z, ones, sub.freq_hz, prm, normalize=False)
    y = oracle_mod.wstack_predict(sub.uvw_m, ones, sub.freq_hz, prm, X)
    lhs, rhs = float(np.sum(A * X)), float(np.real(np.sum(z * np.conj(y))))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


# ---------------------------------------------------------------------------------------
# the w-kernel across planes (an accuracy variant): Eq. 3's kernel with its w argument

def _w_alias(oracle, y, Ww, beta_w):
    """sum_{m != 0} |C_w(y + m)| / |C_w(y)|: the Poisson-sum aliasing of Ww integer-spaced taps."""
    y = np.asarray(y, dtype=np.float64)
    ms = np.concatenate([np.arange(-40, 0), np.arange(1, 41)])
    al = np.abs(oracle.kb.kb_taper(y[..., None] + ms, Ww, beta_w)).sum(-1)
    return al / np.abs(oracle.kb.kb_taper(y, Ww, beta_w))


@pytest.mark.parametrize("Ww", [3, 5, 7])
def test_wkernel_unit_visibility_carries_the_exact_w_term(oracle_mod, Ww):
    """P21: one unit visibility at u = v = 0 and w = w0 between plane centres.  Its uv taps give
    P1's closed-form flat image F(i, j); the w-taps, stacked with the planes' phases and divided
    by C_w(dw (n - 1)), must give the exact w-term exp(2 pi i w0 (n_ij - 1)) of Eq. 1 up to the
    Poisson aliasing of the w-taps, sum_{m != 0} |C_w(y + m)| / |C_w(y)| at y = dw (n_ij - 1).
    A wrong plane centre, w-tap origin, tap sign or correction fails the bound by orders of
    magnitude."""
    kbm = oracle_mod.kb
    n, dl, f, W = 64, 5e-3, 1e9, 7
    beta, bw = 2.34 * W, 2.34 * Ww
    nw = Ww + 4
    w_lo, w_hi = -16.0, 16.0 + 0.37
    lam = C / f
    w0 = 5.3
    uvw = np.array([[0.0, 0.0, w0 * lam]])
    prm = _prm(oracle_mod, n, dl, nw, W, w_lo=w_lo, w_hi=w_hi)
    prm.w_support = Ww
    D = oracle_mod.wstack_image(uvw, np.ones(1), np.ones(1), f, prm, complex_out=True)
    pr = oracle_mod.prepare(uvw, np.ones(1), f, prm)
    assert pr.dw == (w_hi - w_lo) / (nw - Ww)
    t = np.arange(W) - (W - 1) // 2
    xi = (np.arange(n) - n // 2) / n
    series = (kbm.kb(t, W, beta)[None, :] * np.cos(2 * math.pi * np.outer(xi, t))).sum(1)
    flat = np.outer(series / kbm.kb_taper(xi, W, beta), series / kbm.kb_taper(xi, W, beta))
    _, _, nm1 = oracle_mod.direction_cosines(n, dl, np.arange(n), np.arange(n))
    exact = np.exp(2j * math.pi * w0 * nm1)
    y = pr.dw * nm1
    assert np.max(np.abs(y)) < 0.25
    dev = np.abs(D / flat - exact)
    bound = _w_alias(oracle_mod, y, Ww, bw)
    assert np.all(dev <= 1.05 * bound + 1e-13), float(np.max(dev / (bound + 1e-300)))
    # and the w-term is really there: without the w-kernel's taps the phase is far off
    assert np.max(np.abs(exact - 1.0)) > 0.5


def test_wkernel_error_falls_at_fixed_nw(oracle_mod, c1):
    """P22: on the 256^2 plain-method workload at its 8 planes, the w-kernel image is far
    closer to the direct DFT of Eq. 1 than the nearest-plane image (inner half, where P12's uv
    aliasing bound is 3.2e-6), the error falls as the w-support grows, and each stays within
    the w-taps' Poisson aliasing at y = 0 plus that uv bound (support 3 aliases more than the
    nearest-plane quantisation costs here: its kernel's sidelobes decay slowly)."""
    ds = c1
    n = ds.n
    rows = np.arange(n // 4, 3 * n // 4, 4)
    cols = np.arange(n // 4 + 1, 3 * n // 4, 4)
    Dd = oracle_mod.dft_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, n, ds.pixel_rad, pixels=(rows, cols))
    errs = {}
    for Ww in (0, 3, 5, 7):
        prm = _prm(oracle_mod, n, ds.pixel_rad, ds.n_wplanes, ds.support)
        prm.w_support = Ww
        Dw = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, prm, pixels=(rows, cols))
        errs[Ww] = np.linalg.norm(Dw - Dd) / np.linalg.norm(Dd)
    assert errs[7] < errs[5] < errs[3], errs
    assert errs[5] < 0.1 * errs[0] and errs[7] < 0.01 * errs[0], errs
    for Ww in (3, 5, 7):
        assert errs[Ww] < _w_alias(oracle_mod, 0.0, Ww, 2.34 * Ww) + 3.2e-6, (Ww, errs)


def test_wkernel_planes_and_taps(oracle_mod):
    """P23: the plane layout of the w-kernel: every kept row's Ww taps lie on the planes, the
    data's w range maps to plane coordinates [h, Nw - 1 - h], a row's factors on its planes are
    the kernel at integer-spaced offsets (they sum to about C_w(0), P10 along w), and a plane
    receives exactly the rows whose taps reach it."""
    rng = np.random.default_rng(17)
    n, dl, f, W, Ww, nw = 64, 2e-3, 1e9, 5, 5, 9
    uvw = _random_uv(rng, 400, n, dl, f, W, wscale=50.0)
    prm = _prm(oracle_mod, n, dl, nw, W)
    prm.w_support = Ww
    pr = oracle_mod.prepare(uvw, np.ones(400), f, prm)
    h = (Ww - 1) // 2
    kept = pr.keep
    assert np.all(pr.k[kept] >= 0) and np.all(pr.k[kept] + Ww - 1 <= nw - 1)
    assert abs(pr.z[kept].min() - h) < 1e-9 and abs(pr.z[kept].max() - (nw - 1 - h)) < 1e-9
    assert np.all(np.abs(pr.k[kept] + h - pr.z[kept]) <= 0.5 + 1e-12)   # nearest plane is the middle tap
    tot = np.zeros(pr.u.shape[0])
    for k in range(nw):
        r, fac = oracle_mod.wstack.plane_rows(pr, prm, k)
        assert np.array_equal(r, np.nonzero(kept & (pr.k <= k) & (k < pr.k + Ww))[0])
        tot[r] += fac
    c0 = oracle_mod.kb.kb_taper(0.0, Ww, 2.34 * Ww)
    assert np.max(np.abs(tot[kept] / c0 - 1.0)) < 2e-4
    with pytest.raises(ValueError):
        bad = _prm(oracle_mod, n, dl, Ww, W)
        bad.w_support = Ww
        oracle_mod.prepare(uvw, np.ones(400), f, bad)
