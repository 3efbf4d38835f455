"""Shared pieces of the GPU parity tests: device copies, error norms, taper-aware checks."""

import numpy as np
import pytest

TOL = {"f32": 1e-5, "f64": 1e-12}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(ds, torch):
    dev = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(ds.uvw_m)).to(dev),
            torch.from_numpy(np.ascontiguousarray(ds.vis)).to(dev),
            torch.from_numpy(np.ascontiguousarray(ds.weights)).to(dev))


def _errs(a, ref):
    d = a - ref
    return (float(np.linalg.norm(d) / np.linalg.norm(ref)), float(np.max(np.abs(d)) / np.max(np.abs(ref))))


def _taper(oracle, n, W, beta, idx=None):
    idx = np.arange(n) if idx is None else np.asarray(idx)
    xi = (idx - n // 2) / n
    return oracle.kb.kb_taper(xi, W, beta) / oracle.kb.kb_taper(0.0, W, beta)


def _check(oracle, img, ref, n, W, beta, tol, rows=None, cols=None, full=False, tag=""):
    """(a) untapered everywhere, (b) image on the inner half, (c) image everywhere if full."""
    rows = np.arange(n) if rows is None else np.asarray(rows)
    cols = np.arange(n) if cols is None else np.asarray(cols)
    t = np.outer(_taper(oracle, n, W, beta, rows), _taper(oracle, n, W, beta, cols))
    ua = _errs(img * t, ref * t)
    ri = (np.abs(rows - n // 2) <= n // 4)
    ci = (np.abs(cols - n // 2) <= n // 4)
    ia = _errs(img[np.ix_(ri, ci)], ref[np.ix_(ri, ci)])
    fa = _errs(img, ref)
    print(f"{tag} untapered {ua[0]:.2e}/{ua[1]:.2e} inner {ia[0]:.2e}/{ia[1]:.2e} full {fa[0]:.2e}/{fa[1]:.2e}")
    assert ua[0] <= tol and ua[1] <= tol, ("untapered", ua)
    assert ia[0] <= tol and ia[1] <= tol, ("inner half", ia)
    if full:
        assert fa[0] <= tol and fa[1] <= tol, ("full image", fa)


def _prm(oracle, ds, nw=None, w_range=None):
    lo, hi = (None, None) if w_range is None else w_range
    return oracle.Params(ds.n, ds.pixel_rad, ds.n_wplanes if nw is None else nw, ds.support, ds.beta, lo, hi)


def _random_ds(seed, m, n, nw, W, prec, frac=0.4, wscale=300.0, dl=None):
    """A random visibility set whose footprints cover most of an n x n grid."""
    import synth
    rng = np.random.default_rng(seed)
    dl = dl if dl is not None else 2.0 / (n * 60.0)        # small field
    freq = 1.0e9
    lam = synth.C_LIGHT / freq
    du = 1.0 / (n * dl)
    uv = rng.uniform(-frac * n, frac * n, size=(m, 2)) * du * lam
    w = rng.normal(0, 1, m) * wscale * lam
    uvw = np.column_stack([uv, w])
    vis = rng.normal(size=m) + 1j * rng.normal(size=m)
    wts = rng.uniform(0.2, 2.0, m)
    ds = synth.Dataset("random", uvw, vis, wts, freq, n, dl, nw, W, 2.34 * W)
    return ds.as_precision(prec)


def host_threads(cap=16):
    """Threads for oracle work on the host: the cores this process may run on, at most cap
    (a GPU machine gives one GPU's share of its cores)."""
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def crop_pixels(n, side, k, seed):
    """k x k pixel rows/cols spread over the central side x side crop (the centre included)."""
    rng = np.random.default_rng(seed)
    lo = n // 2 - side // 2
    rows = np.sort(rng.choice(np.arange(lo, lo + side), k, replace=False))
    cols = np.sort(rng.choice(np.arange(lo, lo + side), k, replace=False))
    rows[0], cols[0] = n // 2, n // 2
    return np.unique(rows), np.unique(cols)
