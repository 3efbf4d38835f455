"""The w-kernel across planes (w_support > 0: Eq. 3's kernel with its w argument) on the GPU,
through the C ABI, against the float64 oracle's w-kernel images and grids.

Tolerances as for every image: float64 1e-12, float32 1e-5 in relative L2 and peak error,
untapered everywhere and on the inner half, and over every pixel for the support-7 workload."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from helpers import TOL, _check, _dev, _errs, _prm, _random_ds, _torch  # noqa: E402


def _wprm(oracle, ds, Ww, nw=None, w_range=None):
    prm = _prm(oracle, ds, nw=nw, w_range=w_range)
    prm.w_support = Ww
    return prm


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("Ww", [5, 7])
def test_wkernel_image_c1(oracle_mod, c1, prec, Ww):
    """The 256^2 plain-method workload with its 8 planes and the w-kernel, whole image."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = c1.as_precision(prec)
    img, st = ws.image(*_dev(ds, torch), ds.freq_hz, n=ds.n, pixel_rad=ds.pixel_rad, n_wplanes=ds.n_wplanes,
                       support=ds.support, beta=ds.beta, w_support=Ww, stats=True)
    img = img.cpu().numpy()
    prm = _wprm(oracle_mod, ds, Ww)
    pr = oracle_mod.prepare(ds.uvw_m, ds.weights, ds.freq_hz, prm)
    assert st["w_lo"] == pr.w_lo and st["w_hi"] == pr.w_hi and st["n_gridded"] == pr.n_kept
    ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, prm, prepared=pr)
    _check(oracle_mod, img, ref, ds.n, ds.support, ds.beta, TOL[prec], full=True, tag=f"wkernel {Ww} c1 {prec}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,nw,W,Ww,m", [(64, 6, 15, 3, 3000), (256, 9, 9, 5, 30000), (1024, 10, 7, 7, 80000),
                                         (2048, 8, 9, 5, 40000)])
def test_wkernel_image_shapes(oracle_mod, prec, n, nw, W, Ww, m):
    """Other sizes, uv supports (the 7-, 9- and 15-tap register classes) and w-supports."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = _random_ds(300 + n + Ww, m, n, nw, W, prec, wscale=500.0)
    img = ws.image(*_dev(ds, torch), ds.freq_hz, n=n, pixel_rad=ds.pixel_rad, n_wplanes=nw, support=W,
                   beta=ds.beta, w_support=Ww).cpu().numpy()
    d64 = ds.as_precision("f64")
    ref = oracle_mod.wstack_image(d64.uvw_m, d64.vis, d64.weights, d64.freq_hz, _wprm(oracle_mod, d64, Ww))
    _check(oracle_mod, img, ref, n, W, ds.beta, TOL[prec], full=(prec == "f64" and W <= 7),
           tag=f"wkernel {prec} n={n} W={W} Ww={Ww}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_wkernel_grid_and_batch(oracle_mod, prec):
    """The gridding step alone (each plane holds the rows whose w-taps reach it, weighted by
    the w-kernel) and two channels in one batch call against single-channel oracle images."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    n, nw, W, Ww, m = 256, 7, 7, 3, 20000
    ds = _random_ds(41, m, n, nw, W, prec, wscale=400.0)
    d64 = ds.as_precision("f64")
    half = m // 2
    with ws.Plan(n, ds.pixel_rad, nw, W, ds.beta, prec, max_vis=m, max_channels=2, w_support=Ww) as p:
        u, v, w = _dev(ds, torch)
        g = p.grid(u, v, w, ds.freq_hz).cpu().numpy()
        two = p.image_batch(u, v, w, [half, m - half], [ds.freq_hz, 0.8 * ds.freq_hz]).cpu().numpy()
    gref = oracle_mod.grid_stack(d64.uvw_m, d64.vis, d64.weights, d64.freq_hz, _wprm(oracle_mod, d64, Ww))
    assert np.max(np.abs(g - gref)) <= (1e-12 if prec == "f64" else 2e-6) * np.max(np.abs(gref))
    assert np.array_equal(np.abs(gref) > 0, np.abs(g) > 0)
    for c, (sl, f) in enumerate(((slice(0, half), d64.freq_hz), (slice(half, m), 0.8 * d64.freq_hz))):
        ref = oracle_mod.wstack_image(d64.uvw_m[sl], d64.vis[sl], d64.weights[sl], f, _wprm(oracle_mod, d64, Ww))
        _check(oracle_mod, two[c], ref, n, W, ds.beta, TOL[prec], full=(prec == "f64"), tag=f"wkernel batch ch{c}")


def test_wkernel_fixed_range_clamps_and_degenerate_range(oracle_mod):
    """A fixed range narrower than the data (rows beyond it at the end plane coordinates), and a
    range of zero width (every row at one w: its taps at z = h on planes 0 .. Ww - 1)."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = _random_ds(71, 20000, 256, 8, 7, "f64", wscale=2000.0)
    wr = (-400.0, 900.0)
    img = ws.image(*_dev(ds, torch), ds.freq_hz, n=256, pixel_rad=ds.pixel_rad, n_wplanes=8, support=7,
                   beta=ds.beta, w_support=5, w_range=wr).cpu().numpy()
    ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, _wprm(oracle_mod, ds, 5, w_range=wr))
    _check(oracle_mod, img, ref, 256, 7, ds.beta, 1e-12, full=True, tag="wkernel fixed range")
    flat = ds.subset(slice(0, 5000))
    flat.uvw_m = flat.uvw_m.copy()
    flat.uvw_m[:, 2] = 3.0
    img = ws.image(*_dev(flat, torch), flat.freq_hz, n=256, pixel_rad=flat.pixel_rad, n_wplanes=8, support=7,
                   beta=flat.beta, w_support=5).cpu().numpy()
    ref = oracle_mod.wstack_image(flat.uvw_m, flat.vis, flat.weights, flat.freq_hz, _wprm(oracle_mod, flat, 5))
    _check(oracle_mod, img, ref, 256, 7, flat.beta, 1e-12, full=True, tag="wkernel zero-width range")


def test_wkernel_closer_to_the_dft_on_the_gpu(oracle_mod, c1):
    """What the variant is for: at the same 8 planes, the GPU's w-kernel image (Ww = 7) is
    within 1e-6 of the direct DFT of Eq. 1 on the inner half, the nearest-plane one is not."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = c1
    n = ds.n
    rows = np.arange(n // 4, 3 * n // 4, 4)
    cols = np.arange(n // 4 + 1, 3 * n // 4, 4)
    Dd = oracle_mod.dft_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, n, ds.pixel_rad, pixels=(rows, cols))
    kw = dict(n=n, pixel_rad=ds.pixel_rad, n_wplanes=ds.n_wplanes, support=ds.support, beta=ds.beta)
    near = ws.image(*_dev(ds, torch), ds.freq_hz, **kw).cpu().numpy()[np.ix_(rows, cols)]
    wk = ws.image(*_dev(ds, torch), ds.freq_hz, w_support=7, **kw).cpu().numpy()[np.ix_(rows, cols)]
    e_near, e_wk = _errs(near, Dd)[0], _errs(wk, Dd)[0]
    print(f"vs DFT (inner half): nearest plane {e_near:.2e}, w-kernel 7 {e_wk:.2e}")
    assert e_wk < 1e-6 < e_near


def test_wkernel_prediction_rejected():
    """The prediction is the transpose of nearest-plane imaging only: a w-kernel plan refuses it."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = _random_ds(5, 100, 64, 6, 7, "f32")
    with ws.Plan(64, ds.pixel_rad, 6, 7, precision="f32", max_vis=ds.m, w_support=3) as p:
        u, _, w = _dev(ds, torch)
        with pytest.raises(ws.WsimgError):
            p.predict(u, w, ds.freq_hz, torch.zeros((64, 64), dtype=torch.float32, device=u.device))
