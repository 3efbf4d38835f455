"""Seeded synthetic visibility sets shaped like the paper's workloads.

Geometry follows the textbook relations for an east-north-up (ENU) array
(Thompson, Moran & Swenson, ch. 4): baselines are rotated into the
equatorial (X, Y, Z) frame at the array latitude, then projected onto
(u, v, w) for each hour angle H and the phase-centre declination.

Visibilities of a sky of point (and optionally Gaussian) sources are the
forward measurement equation (Eq. 1 of the paper):
    V(u,v,w) = sum_s (F_s / n_s) exp(-2 pi i (u l_s + v m_s + w (n_s - 1)))
with n_s = sqrt(1 - l_s^2 - m_s^2).  Gaussian sources are given the flat-sky
amplitude factor exp(-2 pi^2 sigma_s^2 (u^2 + v^2)).

Every random draw comes from ``numpy.random.default_rng(seed)``; the sum over
sources runs in float64 through torch (on the CPU or on a GPU) only because it
is the one large contraction here.  Rows are stored time-major (all
baselines of time step 0, then time step 1, ...), as a measurement set is read.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

C_LIGHT = 299_792_458.0          # m/s
ARCSEC = math.pi / (180.0 * 3600.0)
HOUR_RAD = 2.0 * math.pi / 24.0  # hour angle: 1 h = 15 deg


@dataclasses.dataclass
class Dataset:
    """One channel of visibilities plus the imaging parameters of its workload."""

    name: str
    uvw_m: np.ndarray          # (M, 3) float64, metres
    vis: np.ndarray            # (M,) complex128 or complex64
    weights: np.ndarray        # (M,) float64 or float32
    freq_hz: float
    n: int                     # image side = grid side
    pixel_rad: float
    n_wplanes: int
    support: int
    beta: float
    sources: Dict[str, np.ndarray] = dataclasses.field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.uvw_m.shape[0])

    def as_precision(self, precision: str) -> "Dataset":
        """Return a copy whose vis/weights carry the dtype of ``precision``.

        'f64' -> complex128/float64, 'f32' -> complex64/float32.  uvw stays float64.
        """
        if precision == "f64":
            cv, fw = np.complex128, np.float64
        elif precision == "f32":
            cv, fw = np.complex64, np.float32
        else:
            raise ValueError(precision)
        return dataclasses.replace(self, vis=self.vis.astype(cv), weights=self.weights.astype(fw))

    def subset(self, idx) -> "Dataset":
        return dataclasses.replace(self, uvw_m=np.ascontiguousarray(self.uvw_m[idx]),
                                   vis=np.ascontiguousarray(self.vis[idx]),
                                   weights=np.ascontiguousarray(self.weights[idx]))


# ---------------------------------------------------------------------------
# array geometry

def antenna_layout(kind: str, rng: np.random.Generator, **kw) -> np.ndarray:
    """Antenna (station) positions as ENU metres, height 0, shape (n, 3)."""
    if kind == "disk":
        n, radius = kw["n"], kw["radius_m"]
        r = radius * np.sqrt(rng.random(n))
        th = 2.0 * math.pi * rng.random(n)
    elif kind == "core+outliers":
        nc, rc = kw["n_core"], kw["core_radius_m"]
        no, r0, r1 = kw["n_out"], kw["out_r0_m"], kw["out_r1_m"]
        r = np.concatenate([rc * np.sqrt(rng.random(nc)),
                            np.exp(rng.uniform(math.log(r0), math.log(r1), no))])
        th = 2.0 * math.pi * rng.random(nc + no)
    elif kind == "logradial":
        n, r0, r1 = kw["n"], kw["r0_m"], kw["r1_m"]
        r = np.exp(rng.uniform(math.log(r0), math.log(r1), n))
        th = 2.0 * math.pi * rng.random(n)
    else:
        raise ValueError(kind)
    enu = np.zeros((r.size, 3))
    enu[:, 0] = r * np.cos(th)
    enu[:, 1] = r * np.sin(th)
    return enu


def baselines_xyz(enu: np.ndarray, lat_rad: float) -> np.ndarray:
    """All pairs a1 < a2, b = a2 - a1, rotated to the equatorial frame (X, Y, Z)."""
    a1, a2 = np.triu_indices(enu.shape[0], k=1)
    d = enu[a2] - enu[a1]
    e, nn, up = d[:, 0], d[:, 1], d[:, 2]
    sphi, cphi = math.sin(lat_rad), math.cos(lat_rad)
    x = -sphi * nn + cphi * up
    y = e
    z = cphi * nn + sphi * up
    return np.stack([x, y, z], axis=1)


def uvw_track(bxyz: np.ndarray, dec_rad: float, ha_rad: np.ndarray,
              max_rows: Optional[int] = None) -> np.ndarray:
    """(u, v, w) in metres for every (time, baseline), time-major, shape (T*B, 3)."""
    nb = bxyz.shape[0]
    rows = ha_rad.size * nb if max_rows is None else min(max_rows, ha_rad.size * nb)
    out = np.empty((rows, 3))
    sd, cd = math.sin(dec_rad), math.cos(dec_rad)
    X, Y, Z = bxyz[:, 0], bxyz[:, 1], bxyz[:, 2]
    step = max(1, (1 << 22) // nb)
    for t0 in range(0, ha_rad.size, step):
        r0 = t0 * nb
        if r0 >= rows:
            break
        h = ha_rad[t0:t0 + step][:, None]
        sh, ch = np.sin(h), np.cos(h)
        u = sh * X + ch * Y
        v = -sd * ch * X + sd * sh * Y + cd * Z
        w = cd * ch * X - cd * sh * Y + sd * Z
        blk = np.stack([u, v, w], axis=2).reshape(-1, 3)
        r1 = min(rows, r0 + blk.shape[0])
        out[r0:r1] = blk[: r1 - r0]
    return out


# ---------------------------------------------------------------------------
# sky model and forward prediction

def _powerlaw_fluxes(rng, n, smin, smax, index=-1.5):
    """Draw n fluxes from dN/dS ~ S^index on [smin, smax] by inverse CDF."""
    a = index + 1.0                       # -0.5 for index -1.5
    u = rng.random(n)
    lo, hi = smin ** a, smax ** a
    return (lo + u * (hi - lo)) ** (1.0 / a)


def predict_point_sources(uvw_m: np.ndarray, freq_hz: float, l: np.ndarray, m: np.ndarray,
                          flux: np.ndarray, gauss_sigma_rad: Optional[np.ndarray] = None,
                          device: str = "cpu", chunk: Optional[int] = None) -> np.ndarray:
    """Forward measurement equation for a list of sources, float64, complex128 out."""
    import torch

    M = uvw_m.shape[0]
    S = l.size
    out = np.zeros(M, dtype=np.complex128)
    if M == 0 or S == 0:
        return out
    dev = torch.device(device)
    n = np.sqrt(1.0 - l * l - m * m)
    A = torch.tensor(np.stack([l, m, n - 1.0]), dtype=torch.float64, device=dev)   # (3, S)
    amp = torch.tensor(flux / n, dtype=torch.float64, device=dev)                    # (S,)
    gs = None
    if gauss_sigma_rad is not None:
        gs = torch.tensor(gauss_sigma_rad, dtype=torch.float64, device=dev)
    if chunk is None:
        chunk = max(1024, (1 << 24 if dev.type == "cuda" else 1 << 21) // S)
    scale = freq_hz / C_LIGHT
    for c0 in range(0, M, chunk):
        c1 = min(M, c0 + chunk)
        uvw = torch.tensor(uvw_m[c0:c1], dtype=torch.float64, device=dev) * scale   # wavelengths
        cyc = uvw @ A                                                               # (C, S)
        cyc = cyc - torch.round(cyc)
        ph = (-2.0 * math.pi) * cyc
        a = amp.expand_as(cyc)
        if gs is not None:
            uv2 = (uvw[:, 0] ** 2 + uvw[:, 1] ** 2)[:, None]
            a = a * torch.exp(-2.0 * math.pi ** 2 * gs[None, :] ** 2 * uv2)
        re = (a * torch.cos(ph)).sum(dim=1)
        im = (a * torch.sin(ph)).sum(dim=1)
        out[c0:c1].real = re.cpu().numpy()
        out[c0:c1].imag = im.cpu().numpy()
    return out


# ---------------------------------------------------------------------------
# the five workloads

CONFIGS: Dict[int, dict] = {
    1: dict(name="c1_plain_f64", layout=("disk", dict(n=64, radius_m=2000.0)),
            lat_deg=-30.0, dec_deg=-30.0,
            ha=("linspace", -2.0, 2.0, 50), freq_hz=1.4e9,
            n=256, pixel_arcsec=2.0, n_wplanes=8, support=7,
            sky=dict(n_points=20, flux=("uniform", 0.1, 1.0)), noise=0.01, precision="f64"),
    2: dict(name="c2_meerkat_f32", layout=("core+outliers", dict(n_core=44, core_radius_m=500.0,
                                                                 n_out=20, out_r0_m=500.0, out_r1_m=4000.0)),
            lat_deg=-30.7, dec_deg=-30.0,
            ha=("steps", 8.0, 3600), freq_hz=1.4e9,
            n=4096, pixel_arcsec=1.5, n_wplanes=32, support=7,
            sky=dict(n_points=200, flux=("powerlaw", 1e-3, 1.0)), noise=1e-3, precision="f32"),
    3: dict(name="c3_lofar_f32", layout=("logradial", dict(n=60, r0_m=50.0, r1_m=100_000.0)),
            lat_deg=52.9, dec_deg=60.0,
            ha=("steps", 8.0, 37915), max_rows=1 << 26, freq_hz=150e6,
            n=8192, pixel_arcsec=1.0, n_wplanes=64, support=9,
            sky=dict(n_points=1000, flux=("powerlaw", 1e-3, 1.0),
                     n_gauss=10, gauss_flux=("uniform", 0.05, 0.5), gauss_sigma_px=(3.0, 20.0)),
            noise=1e-3, precision="f32"),
    4: dict(name="c4_batched_f32", layout_of=2,
            lat_deg=-30.7, dec_deg=-30.0,
            ha=("steps", 8.0, 496), freq_hz=None, channels=(856e6, 1712e6, 64), flag_max=0.6,
            n=1024, pixel_arcsec=2.0, n_wplanes=16, support=7,
            sky=dict(n_points=200, flux=("powerlaw", 1e-3, 1.0)), noise=1e-3, precision="f32"),
    5: dict(name="c5_adjoint_f32", layout_of=2,
            lat_deg=-30.7, dec_deg=-30.0,
            ha=("steps", 8.0, 1984), freq_hz=1.4e9,
            n=2048, pixel_arcsec=1.5, n_wplanes=16, support=7,
            sky=dict(n_points=50, flux=("uniform", 0.1, 1.0)), noise=1e-2, precision="f32"),
}


def config_spec(i: int) -> dict:
    return dict(CONFIGS[i])


def _hour_angles(spec) -> np.ndarray:
    kind = spec[0]
    if kind == "linspace":
        _, h0, h1, nt = spec
        return np.linspace(h0, h1, nt) * HOUR_RAD
    if kind == "steps":
        _, hours, nt = spec
        dt = hours / nt
        return (-hours / 2.0 + (np.arange(nt) + 0.5) * dt) * HOUR_RAD
    raise ValueError(kind)


def _layout_for(i: int) -> np.ndarray:
    spec = CONFIGS[i]
    src = spec.get("layout_of", i)
    kind, kw = CONFIGS[src]["layout"]
    return antenna_layout(kind, np.random.default_rng(1000 + src), **kw)


def _sky(spec, rng, fov_rad, pixel_rad):
    sky = spec["sky"]
    ns = sky["n_points"]
    half = 0.4 * fov_rad
    l = rng.uniform(-half, half, ns)
    m = rng.uniform(-half, half, ns)
    fk = sky["flux"]
    if fk[0] == "uniform":
        f = rng.uniform(fk[1], fk[2], ns)
    else:
        f = _powerlaw_fluxes(rng, ns, fk[1], fk[2])
    sig = np.zeros(ns)
    ng = sky.get("n_gauss", 0)
    if ng:
        lg = rng.uniform(-half, half, ng)
        mg = rng.uniform(-half, half, ng)
        gf = rng.uniform(sky["gauss_flux"][1], sky["gauss_flux"][2], ng)
        gs = rng.uniform(*sky["gauss_sigma_px"], ng) * pixel_rad
        l, m, f = np.concatenate([l, lg]), np.concatenate([m, mg]), np.concatenate([f, gf])
        sig = np.concatenate([sig, gs])
    return dict(l=l, m=m, flux=f, sigma=sig)


def make_config(i: int, device: str = "cpu", max_rows: Optional[int] = None,
                noise: bool = True, geometry_only: bool = False) -> Dataset:
    """Build workload ``i`` (1, 2, 3 or 5) exactly as seeded: default_rng(1000 + i).

    ``max_rows`` truncates the time-major rows (a shorter track of the same array).
    ``geometry_only`` leaves the visibilities zero (uvw, weights and the imaging parameters
    are the workload's own; the sky is still drawn, so nothing else changes).
    """
    if i == 4:
        raise ValueError("config 4 is multi-channel: use make_channels()")
    spec = CONFIGS[i]
    rng = np.random.default_rng(1000 + i)
    if "layout_of" in spec:
        enu = _layout_for(i)
    else:
        # the layout is the first draw of this workload's own stream
        kind, kw = spec["layout"]
        enu = antenna_layout(kind, rng, **kw)
    lat = math.radians(spec["lat_deg"])
    dec = math.radians(spec["dec_deg"])
    bxyz = baselines_xyz(enu, lat)
    rows = spec.get("max_rows")
    if max_rows is not None:
        rows = max_rows if rows is None else min(rows, max_rows)
    uvw = uvw_track(bxyz, dec, _hour_angles(spec["ha"]), rows)
    pixel = spec["pixel_arcsec"] * ARCSEC
    n = spec["n"]
    src = _sky(spec, rng, n * pixel, pixel)
    sig = src["sigma"] if np.any(src["sigma"] > 0) else None
    if geometry_only:
        vis = np.zeros(uvw.shape[0], dtype=np.complex128)
    else:
        vis = predict_point_sources(uvw, spec["freq_hz"], src["l"], src["m"], src["flux"], sig, device)
    if noise and spec["noise"] > 0 and not geometry_only:
        nz = rng.standard_normal((uvw.shape[0], 2)) * spec["noise"]
        vis = vis + (nz[:, 0] + 1j * nz[:, 1])
    w = np.ones(uvw.shape[0])
    ds = Dataset(name=spec["name"], uvw_m=uvw, vis=vis, weights=w, freq_hz=float(spec["freq_hz"]),
                 n=n, pixel_rad=pixel, n_wplanes=spec["n_wplanes"], support=spec["support"],
                 beta=2.34 * spec["support"], sources=src)
    return ds.as_precision(spec["precision"])


def make_channels(device: str = "cpu", n_channels: Optional[int] = None) -> List[Dataset]:
    """Workload 4: many channels of one track, each thinned by its own random flagging."""
    spec = CONFIGS[4]
    rng = np.random.default_rng(1004)
    enu = _layout_for(4)
    bxyz = baselines_xyz(enu, math.radians(spec["lat_deg"]))
    uvw = uvw_track(bxyz, math.radians(spec["dec_deg"]), _hour_angles(spec["ha"]))
    pixel = spec["pixel_arcsec"] * ARCSEC
    n = spec["n"]
    src = _sky(spec, rng, n * pixel, pixel)
    f0, f1, nc = spec["channels"]
    freqs = np.linspace(f0, f1, nc)
    if n_channels is not None:
        freqs = freqs[:n_channels]
    out = []
    m0 = uvw.shape[0]
    for c, f in enumerate(freqs):
        frac = rng.uniform(0.0, spec["flag_max"])
        drop = rng.choice(m0, size=int(math.floor(frac * m0)), replace=False)
        keep = np.ones(m0, dtype=bool)
        keep[drop] = False
        u = np.ascontiguousarray(uvw[keep])
        v = predict_point_sources(u, f, src["l"], src["m"], src["flux"], None, device)
        nz = rng.standard_normal((u.shape[0], 2)) * spec["noise"]
        v = v + (nz[:, 0] + 1j * nz[:, 1])
        ds = Dataset(name=f"{spec['name']}_ch{c}", uvw_m=u, vis=v, weights=np.ones(u.shape[0]),
                     freq_hz=float(f), n=n, pixel_rad=pixel, n_wplanes=spec["n_wplanes"],
                     support=spec["support"], beta=2.34 * spec["support"], sources=src)
        out.append(ds.as_precision("f32"))
    return out


def stack_channels(channels: List[Dataset]):
    """Concatenate channel datasets row-wise: (uvw_m, vis, weights, row_counts, freqs_hz)."""
    uvw = np.concatenate([c.uvw_m for c in channels], axis=0)
    vis = np.concatenate([c.vis for c in channels])
    wts = np.concatenate([c.weights for c in channels])
    counts = [int(c.uvw_m.shape[0]) for c in channels]
    freqs = [float(c.freq_hz) for c in channels]
    return uvw, vis, wts, counts, freqs


def sky_image(ds: Dataset, field_amp: float = 0.05, field_sigma_frac: float = 0.125,
              seed: int = 1105) -> np.ndarray:
    """A dataset's sky as an [n, n] float64 image (row i: m = (i - n/2) dl; column j: l):
    each source's flux at its nearest pixel, plus a smooth Gaussian field of peak field_amp
    and width field_sigma_frac * n pixels at a seeded offset from the centre."""
    n, dl = ds.n, ds.pixel_rad
    img = np.zeros((n, n))
    src = ds.sources
    if src and len(src.get("l", [])):
        j = np.rint(np.asarray(src["l"]) / dl + n // 2).astype(np.int64)
        i = np.rint(np.asarray(src["m"]) / dl + n // 2).astype(np.int64)
        ok = (i >= 0) & (i < n) & (j >= 0) & (j < n)
        np.add.at(img, (i[ok], j[ok]), np.asarray(src["flux"])[ok])
    rng = np.random.default_rng(seed)
    ci, cj = n // 2 + rng.uniform(-0.1, 0.1, 2) * n
    sig = field_sigma_frac * n
    ii = np.arange(n)[:, None]
    jj = np.arange(n)[None, :]
    img += field_amp * np.exp(-((ii - ci) ** 2 + (jj - cj) ** 2) / (2.0 * sig * sig))
    return img
