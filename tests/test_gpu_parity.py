"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: the float32 path must match the float64 oracle to 1e-5 in both relative L2
and relative peak error; the float64 path to 1e-12.  Gridding alone (float64) to 1e-12 of
the largest cell, float32 to 2e-6.  Integer outputs (counts, kept/dropped rows) exactly.

Where the comparison is made: the grid has no padding, so dividing by the kernel's
transform amplifies any rounding in the untapered image by C(0)^2 / (C(xi_i) C(xi_j)),
which reaches 2.6e3 in the corners for W = 7, 3.0e4 for W = 9 and 4.3e7 for W = 15
(and only 5.9, 10 and 52 inside |xi| <= 1/4).  Both the oracle and the GPU carry that
amplified rounding, so each image check compares (a) the untapered image
D * C(xi_i) C(xi_j) / C(0)^2 over every pixel and (b) the image itself over the inner
half; for the W = 7 workloads the image is also compared over every pixel.
"""

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from helpers import TOL, _check, _dev, _errs, _prm, _random_ds, _taper, _torch  # noqa: F401


# ---------------------------------------------------------------------------------------
# the gridding step alone (S1-S3)

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_grid_parity_c1(oracle_mod, c1, prec):
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = c1.as_precision(prec)
    g, st = ws.grid(*_dev(ds, torch), ds.freq_hz, n=ds.n, pixel_rad=ds.pixel_rad, n_wplanes=ds.n_wplanes,
                    support=ds.support, beta=ds.beta, stats=True)
    g = g.cpu().numpy()
    pr = oracle_mod.prepare(ds.uvw_m, ds.weights, ds.freq_hz, _prm(oracle_mod, ds))
    ref = oracle_mod.grid_stack(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, _prm(oracle_mod, ds), prepared=pr)
    assert st["n_gridded"] == pr.n_kept and st["n_dropped"] == ds.m - pr.n_kept
    assert st["w_lo"] == pr.w_lo and st["w_hi"] == pr.w_hi
    assert abs(st["sum_w"] - pr.sum_w) <= 1e-12 * pr.sum_w
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(g - ref)) / scale
    assert err <= (1e-12 if prec == "f64" else 2e-6), err
    # every non-zero cell of the oracle is non-zero here and vice versa (same taps)
    assert np.array_equal(np.abs(ref) > 0, np.abs(g) > 0)


@pytest.mark.parametrize("n,nw,W,m", [(16, 1, 3, 50), (64, 3, 15, 3000), (512, 5, 9, 20000)])
def test_grid_parity_shapes(oracle_mod, n, nw, W, m):
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = _random_ds(11 + n, m, n, nw, W, "f64")
    g = ws.grid(*_dev(ds, torch), ds.freq_hz, n=n, pixel_rad=ds.pixel_rad, n_wplanes=nw, support=W,
                beta=ds.beta).cpu().numpy()
    ref = oracle_mod.grid_stack(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, _prm(oracle_mod, ds))
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------------------
# the whole path (S1-S6)

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_image_parity_c1(oracle_mod, c1, prec):
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = c1.as_precision(prec)
    img = ws.image(*_dev(ds, torch), ds.freq_hz, n=ds.n, pixel_rad=ds.pixel_rad, n_wplanes=ds.n_wplanes,
                   support=ds.support, beta=ds.beta).cpu().numpy()
    ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, _prm(oracle_mod, ds))
    _check(oracle_mod, img, ref, ds.n, ds.support, ds.beta, TOL[prec], full=True, tag=f"c1 {prec}")


@pytest.mark.parametrize("n,nw,W,m", [
    (16, 1, 3, 40), (32, 2, 5, 500), (64, 3, 7, 4000), (128, 4, 15, 5000),
    (256, 7, 9, 30000), (512, 5, 7, 60000), (1024, 3, 7, 100000), (2048, 2, 9, 50000),
])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_image_parity_shapes(oracle_mod, n, nw, W, m, prec):
    """Every transform size that takes a different pass layout, ragged strip and block counts."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = _random_ds(100 + n + nw, m, n, nw, W, prec)
    img = ws.image(*_dev(ds, torch), ds.freq_hz, n=n, pixel_rad=ds.pixel_rad, n_wplanes=nw, support=W,
                   beta=ds.beta).cpu().numpy()
    ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, _prm(oracle_mod, ds))
    # random visibilities give a noise-like image whose peak is near its rms, so the corner
    # amplification dominates its full-image peak error in float32: full check in float64 only
    _check(oracle_mod, img, ref, n, W, ds.beta, TOL[prec], full=(W <= 7 and prec == "f64"),
           tag=f"{prec} n={n} W={W}")


def test_fixed_range_and_clamping(oracle_mod):
    """A fixed plane range narrower than the data: rows beyond it go to the edge planes."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = _random_ds(7, 20000, 256, 6, 7, "f64", wscale=2000.0)
    wr = (-500.0, 800.0)
    img = ws.image(*_dev(ds, torch), ds.freq_hz, n=ds.n, pixel_rad=ds.pixel_rad, n_wplanes=6, support=7,
                   beta=ds.beta, w_range=wr).cpu().numpy()
    ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, _prm(oracle_mod, ds, w_range=wr))
    _check(oracle_mod, img, ref, ds.n, 7, ds.beta, 1e-12, full=True)


@pytest.mark.parametrize("n", [1024, 4096])
def test_sparse_plane_occupancy(oracle_mod, n):
    """Rows on three w levels with a fixed plane range of 9 planes: planes 0, 3 and 7 hold rows,
    the others are empty and lie between them (the stacking pass steps over empty planes and
    loads each plane's strip flags two occupied planes ahead).  n = 4096 takes the radix-16
    stacking pass."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    import synth
    rng = np.random.default_rng(40 + n)
    m = 20000
    ds = _random_ds(40 + n, m, n, 9, 7, "f64")
    lam = synth.C_LIGHT / ds.freq_hz
    ds.uvw_m[:, 2] = np.array([-400.0, -100.0, 300.0])[rng.integers(0, 3, m)] * lam
    wr = (-450.0, 450.0)       # plane width 100 wavelengths: the levels land in planes 0, 3, 7
    kw = dict(n=n, pixel_rad=ds.pixel_rad, n_wplanes=9, support=7, beta=ds.beta, w_range=wr)
    img64 = ws.image(*_dev(ds, torch), ds.freq_hz, **kw).cpu().numpy()
    d32 = ds.as_precision("f32")
    img32 = ws.image(*_dev(d32, torch), ds.freq_hz, **kw).cpu().numpy()
    prm = _prm(oracle_mod, ds, w_range=wr)
    if n <= 1024:
        ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, prm)
        _check(oracle_mod, img64, ref, n, 7, ds.beta, 1e-12, full=True, tag="sparse planes f64")
        _check(oracle_mod, img32, ref, n, 7, ds.beta, 1e-5, tag="sparse planes f32")
    else:
        _check(oracle_mod, img32, img64, n, 7, ds.beta, 1e-5, tag="sparse planes f32 vs gpu f64")
        rows, cols = _sample_pixels(n, 12, 5)
        ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, prm, pixels=(rows, cols))
        scale = np.max(np.abs(img64))
        e64 = np.max(np.abs(img64[np.ix_(rows, cols)] - ref)) / scale
        e32 = np.max(np.abs(img32[np.ix_(rows, cols)] - ref)) / scale
        print(f"sparse planes n={n} sampled vs oracle: f64 {e64:.3e} f32 {e32:.3e}")
        assert e64 <= 1e-12 and e32 <= 1e-5


def test_drops_counts_and_nonfinite(oracle_mod):
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = _random_ds(8, 5000, 128, 4, 7, "f64", frac=0.55)       # some footprints leave the grid
    ds.uvw_m[10, 0] = np.nan
    ds.uvw_m[11, 2] = np.inf
    ds.weights[12] = np.nan
    ds.weights[13] = 0.0
    img, st = ws.image(*_dev(ds, torch), ds.freq_hz, n=ds.n, pixel_rad=ds.pixel_rad, n_wplanes=4,
                       support=7, beta=ds.beta, stats=True)
    pr = oracle_mod.prepare(ds.uvw_m, ds.weights, ds.freq_hz, _prm(oracle_mod, ds))
    assert 0 < st["n_dropped"] == ds.m - pr.n_kept
    assert st["n_gridded"] == pr.n_kept
    ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, _prm(oracle_mod, ds))
    _check(oracle_mod, img.cpu().numpy(), ref, ds.n, 7, ds.beta, 1e-12, full=True)


def test_empty_inputs():
    torch = _torch()
    import paper_2601_19714_amd as ws
    dev = torch.device("cuda:0")
    p = ws.Plan(64, 1e-4, 4, 7, precision="f32", max_vis=10)
    uvw = torch.zeros((0, 3), dtype=torch.float64, device=dev)
    vis = torch.zeros(0, dtype=torch.complex64, device=dev)
    w = torch.zeros(0, dtype=torch.float32, device=dev)
    out = torch.full((64, 64), 7.0, device=dev)
    with pytest.raises(ws.WsimgError) as e:
        p.image(uvw, vis, w, 1e9, out=out, stats=True)
    assert e.value.status == -4
    assert not torch.any(out != 0)
    # all rows off the grid
    uvw = torch.tensor([[1e9, 0.0, 0.0]] * 3, dtype=torch.float64, device=dev)
    vis = torch.ones(3, dtype=torch.complex64, device=dev)
    w = torch.ones(3, dtype=torch.float32, device=dev)
    out.fill_(3.0)
    with pytest.raises(ws.WsimgError):
        p.image(uvw, vis, w, 1e9, out=out, stats=True)
    assert not torch.any(out != 0)
    # capacity
    big = torch.zeros((11, 3), dtype=torch.float64, device=dev)
    with pytest.raises(ws.WsimgError) as e:
        p.image(big, torch.zeros(11, dtype=torch.complex64, device=dev),
                torch.zeros(11, dtype=torch.float32, device=dev), 1e9)
    assert e.value.status == -5
    p.close()


def test_hot_bucket_and_single_cell(oracle_mod):
    """Many rows on one cell (one overfull bucket) next to a sparse background."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = _random_ds(9, 40000, 256, 3, 7, "f32")
    ds.uvw_m[:30000, :2] = ds.uvw_m[0, :2]
    img = ws.image(*_dev(ds, torch), ds.freq_hz, n=ds.n, pixel_rad=ds.pixel_rad, n_wplanes=3, support=7,
                   beta=ds.beta).cpu().numpy()
    ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, _prm(oracle_mod, ds))
    _check(oracle_mod, img, ref, ds.n, 7, ds.beta, 1e-5)


def test_point_source_through_gpu(oracle_mod, c1):
    """The DFT pin of a point source carried over: the GPU image peaks on the source pixel
    with F/n0 within the w-quantisation and aliasing bound."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    n, dl = c1.n, c1.pixel_rad
    i0, j0 = n // 2 + 23, n // 2 - 41
    l0, m0 = (j0 - n // 2) * dl, (i0 - n // 2) * dl
    u, v, w = (c1.uvw_m * c1.freq_hz / 299_792_458.0).T
    n0 = math.sqrt(1 - l0 * l0 - m0 * m0)
    vis = (0.9 / n0) * np.exp(-2j * math.pi * (u * l0 + v * m0 + w * (n0 - 1)))
    ds = c1.__class__(**{**c1.__dict__, "vis": vis.astype(np.complex64), "weights": c1.weights.astype(np.float32)})
    img = ws.image(*_dev(ds, torch), ds.freq_hz, n=n, pixel_rad=dl, n_wplanes=16, support=7,
                   beta=ds.beta).cpu().numpy()
    assert np.unravel_index(np.argmax(img), img.shape) == (i0, j0)
    assert abs(img[i0, j0] * n0 / 0.9 - 1.0) < 1e-3


def test_repeat_calls_and_timing(c1):
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = c1.as_precision("f32")
    args = _dev(ds, torch)
    with ws.Plan(ds.n, ds.pixel_rad, ds.n_wplanes, ds.support, ds.beta, "f32", max_vis=ds.m) as p:
        p.set_timing(True)
        a = p.image(*args, ds.freq_hz).cpu().numpy()
        b = p.image(*args, ds.freq_hz).cpu().numpy()
        t = p.read_timing()
        info = p.info()
    assert t["calls"] == 2 and t["ms_total"] > 0 and all(v >= 0 for v in t["ms"].values())
    assert np.max(np.abs(a - b)) <= 1e-6 * np.max(np.abs(a))
    assert info["n"] == ds.n and info["device_bytes"] > 0


# ---------------------------------------------------------------------------------------
# full-size workloads: sampled pixels against the oracle, whole image float32 vs float64

def _sample_pixels(n, k, seed):
    rng = np.random.default_rng(seed)
    inner = np.arange(n // 4, 3 * n // 4)
    rows = np.sort(rng.choice(inner, k, replace=False))
    cols = np.sort(rng.choice(inner, k, replace=False))
    rows[0], cols[0] = n // 2, n // 2                 # include the phase centre
    return rows, cols


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_c2_full_image_vs_oracle(oracle_mod):
    """The MeerKAT-shaped workload at full size (7 257 600 rows, 4096^2, 32 planes, W = 7):
    the whole float32 and float64 images against the whole float64 oracle image (R17: at
    W = 7 the image is compared over every pixel), plus untapered and inner-half checks."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    import synth
    from helpers import host_threads
    ds = synth.make_config(2, device="cuda")
    d64 = ds.as_precision("f64")
    kw = dict(n=ds.n, pixel_rad=ds.pixel_rad, n_wplanes=ds.n_wplanes, support=ds.support, beta=ds.beta)
    img32 = ws.image(*_dev(ds, torch), ds.freq_hz, **kw).cpu().numpy()
    img64 = ws.image(*_dev(d64, torch), ds.freq_hz, **kw).cpu().numpy()
    th = host_threads()
    print(f"c2 oracle on {th} threads", flush=True)
    ref = oracle_mod.wstack_image(d64.uvw_m, d64.vis, d64.weights, d64.freq_hz, _prm(oracle_mod, d64),
                                  threads=th)
    _check(oracle_mod, img64, ref, ds.n, ds.support, ds.beta, 1e-12, full=True, tag="c2 f64 vs oracle")
    _check(oracle_mod, img32, ref, ds.n, ds.support, ds.beta, 1e-5, full=True, tag="c2 f32 vs oracle")


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_c3_geometry_full_grid(oracle_mod):
    """The 8192^2, 64-plane, W = 9 geometry at a shortened track (2^21 rows).  Float32 against
    float64 on the GPU: untapered everywhere, inner half, and the central 512^2 crop (R17's
    place for this workload); both against the oracle at 32 x 32 pixels spread over the crop."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    import synth
    from helpers import crop_pixels, host_threads
    print("c3 geometry: 2^21 rows, n=8192, nw=64, W=9", flush=True)
    ds = synth.make_config(3, device="cuda", max_rows=1 << 21)
    d64 = ds.as_precision("f64")
    kw = dict(n=ds.n, pixel_rad=ds.pixel_rad, n_wplanes=ds.n_wplanes, support=ds.support, beta=ds.beta)
    print("c3 float32 image", flush=True)
    img32 = ws.image(*_dev(ds, torch), ds.freq_hz, **kw).cpu().numpy()
    print("c3 float64 image", flush=True)
    img64 = ws.image(*_dev(d64, torch), ds.freq_hz, **kw).cpu().numpy()
    _check(oracle_mod, img32, img64, ds.n, ds.support, ds.beta, 1e-5, tag="c3 f32 vs gpu f64")
    crop = slice(ds.n // 2 - 256, ds.n // 2 + 256)
    l2, pk = _errs(img32[crop, crop], img64[crop, crop])
    print(f"c3 central 512^2 crop f32 vs f64: {l2:.3e} / {pk:.3e}")
    assert l2 <= 1e-5 and pk <= 1e-5
    rows, cols = crop_pixels(ds.n, 512, 32, 3)
    ref = oracle_mod.wstack_image(d64.uvw_m, d64.vis, d64.weights, d64.freq_hz, _prm(oracle_mod, d64),
                                  pixels=(rows, cols), threads=host_threads())
    e64 = _errs(img64[np.ix_(rows, cols)], ref)
    e32 = _errs(img32[np.ix_(rows, cols)], ref)
    print(f"c3 crop-sampled vs oracle: f64 {e64[0]:.3e}/{e64[1]:.3e} f32 {e32[0]:.3e}/{e32[1]:.3e}")
    assert max(e64) <= 1e-12 and max(e32) <= 1e-5


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_complex_out_c1(oracle_mod, c1, prec):
    """WSIMG_COMPLEX_OUT (reading R10): the complex image S / (sum W C(xi_i) C(xi_j)) against
    the oracle's complex image, both parts; its real part equals the real image.  The C1 sky
    is real but its visibilities carry no Hermitian partners, so Im S is as large as Re S."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = c1.as_precision(prec)
    kw = dict(n=ds.n, pixel_rad=ds.pixel_rad, n_wplanes=ds.n_wplanes, support=ds.support, beta=ds.beta)
    img = ws.image(*_dev(ds, torch), ds.freq_hz, complex_out=True, **kw).cpu().numpy()
    real = ws.image(*_dev(ds, torch), ds.freq_hz, **kw).cpu().numpy()
    assert np.iscomplexobj(img) and img.shape == (ds.n, ds.n)
    ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, _prm(oracle_mod, ds), complex_out=True)
    assert np.linalg.norm(ref.imag) > 0.1 * np.linalg.norm(ref.real)
    _check(oracle_mod, img, ref, ds.n, ds.support, ds.beta, TOL[prec], full=True, tag=f"complex c1 {prec}")
    # the imaginary part alone is noise-like (no point-source peak), so like random data its
    # full-image peak error in float32 is set by the corner amplification of the taper: full
    # check in float64, untapered everywhere and inner half in both
    _check(oracle_mod, img.imag, ref.imag, ds.n, ds.support, ds.beta, TOL[prec], full=(prec == "f64"),
           tag=f"imag c1 {prec}")
    assert max(_errs(img.real, real)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,nw,W,m,pad", [(64, 3, 15, 3000, 1), (512, 5, 7, 40000, 1), (256, 4, 9, 20000, 2)])
def test_complex_out_shapes_and_batch(oracle_mod, prec, n, nw, W, m, pad):
    """Complex images of other sizes, supports and the padded grid, one channel and two
    channels in one batch call, against the oracle's complex images."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = _random_ds(900 + n + W, m, n, nw, W, prec)
    d64 = ds.as_precision("f64")
    half = m // 2
    with ws.Plan(n, ds.pixel_rad, nw, W, ds.beta, prec, max_vis=ds.m, max_channels=2, pad=pad,
                 complex_out=True) as p:
        u, v, w = _dev(ds, torch)
        one = p.image(u, v, w, ds.freq_hz).cpu().numpy()
        two = p.image_batch(u, v, w, [half, m - half], [ds.freq_hz, 1.25 * ds.freq_hz]).cpu().numpy()
    assert one.dtype == (np.complex64 if prec == "f32" else np.complex128)
    prm = _prm(oracle_mod, d64)
    prm.pad = pad
    refs = [oracle_mod.wstack_image(d64.uvw_m, d64.vis, d64.weights, d64.freq_hz, prm, complex_out=True),
            oracle_mod.wstack_image(d64.uvw_m[:half], d64.vis[:half], d64.weights[:half], d64.freq_hz, prm,
                                    complex_out=True),
            oracle_mod.wstack_image(d64.uvw_m[half:], d64.vis[half:], d64.weights[half:], 1.25 * d64.freq_hz,
                                    prm, complex_out=True)]
    tol = TOL[prec]
    for tag, img, ref in (("one", one, refs[0]), ("ch0", two[0], refs[1]), ("ch1", two[1], refs[2])):
        if pad == 2:
            t = _taper_pad(oracle_mod, n, W, ds.beta)
            tt = np.outer(t, t)
            ua, fa = _errs(img * tt, ref * tt), _errs(img, ref)
            print(f"complex pad2 {tag} {prec}: untapered {ua[0]:.2e}/{ua[1]:.2e} full {fa[0]:.2e}/{fa[1]:.2e}")
            assert max(ua) <= tol and max(fa) <= tol
        else:
            _check(oracle_mod, img, ref, n, W, ds.beta, tol, full=(prec == "f64" and W <= 7),
                   tag=f"complex {tag} {prec} n={n}")


def test_complex_out_rejected_by_predict():
    """A complex-output plan images only: its prediction call is an error, not a silent
    reinterpretation of the image buffer."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = _random_ds(5, 100, 64, 2, 7, "f32")
    with ws.Plan(64, ds.pixel_rad, 2, 7, precision="f32", max_vis=ds.m, complex_out=True) as p:
        u, _, w = _dev(ds, torch)
        with pytest.raises(ws.WsimgError):
            p.predict(u, w, ds.freq_hz, torch.zeros((64, 64), dtype=torch.float32, device=u.device))


# ---------------------------------------------------------------------------------------
# properties of the GPU path itself (any size)

def test_gpu_linearity_permutation_and_weight_scale(c1):
    """The image is linear in V, independent of row order, and unchanged by scaling all
    weights (natural weighting divides by their sum)."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = c1.as_precision("f64")
    uvw, vis, w = _dev(ds, torch)
    kw = dict(n=ds.n, pixel_rad=ds.pixel_rad, n_wplanes=ds.n_wplanes, support=ds.support, beta=ds.beta)
    rng = np.random.default_rng(21)
    v2 = torch.from_numpy(rng.normal(size=ds.m) + 1j * rng.normal(size=ds.m)).to(vis.device)
    a, b = 0.7, -1.9
    D1 = ws.image(uvw, vis, w, ds.freq_hz, **kw).cpu().numpy()
    D2 = ws.image(uvw, v2, w, ds.freq_hz, **kw).cpu().numpy()
    D12 = ws.image(uvw, (a * vis + b * v2).contiguous(), w, ds.freq_hz, **kw).cpu().numpy()
    assert np.max(np.abs(D12 - (a * D1 + b * D2))) <= 1e-12 * np.max(np.abs(D12))
    perm = torch.from_numpy(rng.permutation(ds.m)).to(vis.device)
    Dp = ws.image(uvw[perm].contiguous(), vis[perm].contiguous(), w[perm].contiguous(), ds.freq_hz,
                  **kw).cpu().numpy()
    assert np.max(np.abs(Dp - D1)) <= 1e-12 * np.max(np.abs(D1))
    Ds = ws.image(uvw, vis, (3.25 * w).contiguous(), ds.freq_hz, **kw).cpu().numpy()
    assert np.max(np.abs(Ds - D1)) <= 1e-12 * np.max(np.abs(D1))


def test_plan_reuse_with_fewer_rows(oracle_mod, c1):
    """One plan, sized for all rows, imaging a prefix and then the whole set."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = c1.as_precision("f32")
    uvw, vis, w = _dev(ds, torch)
    with ws.Plan(ds.n, ds.pixel_rad, ds.n_wplanes, ds.support, ds.beta, "f32", max_vis=ds.m) as p:
        for m in (ds.m // 3, ds.m):
            img = p.image(uvw[:m].contiguous(), vis[:m].contiguous(), w[:m].contiguous(), ds.freq_hz).cpu().numpy()
            sub = ds.subset(slice(0, m))
            ref = oracle_mod.wstack_image(sub.uvw_m, sub.vis, sub.weights, sub.freq_hz, _prm(oracle_mod, sub))
            _check(oracle_mod, img, ref, ds.n, ds.support, ds.beta, 1e-5, full=True, tag=f"prefix {m}")


# ---------------------------------------------------------------------------------------
# w-folding (WSIMG_FOLD_W)

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fold_parity_c1(oracle_mod, c1, prec):
    """Folded imaging against the folded oracle, and against the GPU imaging of rows flipped
    by hand ((u, v, w, V) -> (-u, -v, -w, conj V) for w < 0) without folding."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = c1.as_precision(prec)
    with ws.Plan(ds.n, ds.pixel_rad, ds.n_wplanes, ds.support, ds.beta, prec, max_vis=ds.m, fold_w=True) as p:
        img, st = p.image(*_dev(ds, torch), ds.freq_hz, stats=True)
    img = img.cpu().numpy()
    prm = _prm(oracle_mod, ds)
    prm.fold = True
    pr = oracle_mod.prepare(ds.uvw_m, ds.weights, ds.freq_hz, prm)
    assert st["w_lo"] == pr.w_lo and st["w_hi"] == pr.w_hi and st["w_lo"] >= 0
    ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, prm, prepared=pr)
    _check(oracle_mod, img, ref, ds.n, ds.support, ds.beta, TOL[prec], full=True, tag=f"fold {prec}")
    neg = ds.uvw_m[:, 2] < 0
    uvw2 = np.ascontiguousarray(np.where(neg[:, None], -ds.uvw_m, ds.uvw_m))
    vis2 = np.ascontiguousarray(np.where(neg, np.conj(ds.vis), ds.vis))
    dev = torch.device("cuda:0")
    hand = ws.image(torch.from_numpy(uvw2).to(dev), torch.from_numpy(vis2).to(dev),
                    torch.from_numpy(np.ascontiguousarray(ds.weights)).to(dev), ds.freq_hz, n=ds.n,
                    pixel_rad=ds.pixel_rad, n_wplanes=ds.n_wplanes, support=ds.support, beta=ds.beta).cpu().numpy()
    assert np.max(np.abs(hand - img)) <= (1e-12 if prec == "f64" else 1e-6) * np.max(np.abs(img))


# ---------------------------------------------------------------------------------------
# grid padding x2 (WSIMG_PAD2)

def _taper_pad(oracle, n, W, beta):
    xi = (np.arange(n) - n // 2) / (2 * n)
    return oracle.kb.kb_taper(xi, W, beta) / oracle.kb.kb_taper(0.0, W, beta)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,nw,W,m", [(16, 1, 3, 40), (64, 3, 15, 3000), (256, 7, 9, 30000), (1024, 3, 7, 100000)])
def test_pad2_parity(oracle_mod, prec, n, nw, W, m):
    """Padded imaging (2n grid, central crop) against the padded oracle: untapered image
    everywhere and the image itself everywhere (the taper's edge amplification is at most
    C(0)^2/C(1/4)^2: 5.9 for W = 7, 52 for W = 15), and the padded grid [nw][2n][2n]."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    ds = _random_ds(700 + n + W, m, n, nw, W, prec)
    with ws.Plan(n, ds.pixel_rad, nw, W, ds.beta, prec, max_vis=ds.m, pad=2) as p:
        assert p.info()["n_grid"] == 2 * n
        img = p.image(*_dev(ds, torch), ds.freq_hz).cpu().numpy()
        grd = p.grid(*_dev(ds, torch), ds.freq_hz).cpu().numpy()
    d64 = ds.as_precision("f64")
    prm = _prm(oracle_mod, d64)
    prm.pad = 2
    ref = oracle_mod.wstack_image(d64.uvw_m, d64.vis, d64.weights, d64.freq_hz, prm)
    t = _taper_pad(oracle_mod, n, W, ds.beta)
    tt = np.outer(t, t)
    ua = _errs(img * tt, ref * tt)
    fa = _errs(img, ref)
    print(f"pad2 n={n} W={W} {prec}: untapered {ua[0]:.2e}/{ua[1]:.2e} full {fa[0]:.2e}/{fa[1]:.2e}")
    tol = TOL[prec]
    assert ua[0] <= tol and ua[1] <= tol
    assert fa[0] <= tol and fa[1] <= (tol if W <= 9 else 10 * tol)
    gref = oracle_mod.grid_stack(d64.uvw_m, d64.vis, d64.weights, d64.freq_hz, prm)
    assert grd.shape == gref.shape == (nw, 2 * n, 2 * n)
    assert np.max(np.abs(grd - gref)) <= (1e-12 if prec == "f64" else 2e-6) * np.max(np.abs(gref))
