"""The allocation-free entry point (wsimg_image_noalloc, through the C ABI) against the plan
entry point wsimg_image and the float64 oracle, on consecutive calls that reuse the static
scratch array: the full 256^2 plain-method workload, then fewer rows (the array keeps the
first call's contents), then a smaller image of another support (the tables change).

Bar: the same as every image parity test, float64 1e-12 and float32 1e-5 in relative L2 and
relative peak error, untapered everywhere, on the inner half and (support 7) everywhere."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from helpers import TOL, _check, _dev, _prm, _random_ds, _torch  # noqa: E402


def _noalloc(ws, torch, d):
    u, v, w = _dev(d, torch)
    rdt = torch.float32 if d.vis.dtype == np.complex64 else torch.float64
    out = torch.full((d.n, d.n), float("nan"), dtype=rdt, device=u.device)
    img, st = ws.image_noalloc(u, v, w, d.freq_hz, out, n=d.n, pixel_rad=d.pixel_rad, n_wplanes=d.n_wplanes,
                               support=d.support, beta=d.beta, stats=True)
    plan = ws.image(u, v, w, d.freq_hz, n=d.n, pixel_rad=d.pixel_rad, n_wplanes=d.n_wplanes,
                    support=d.support, beta=d.beta, stats=True)
    return img.cpu().numpy(), st, plan[0].cpu().numpy(), plan[1]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_against_plan_and_oracle(oracle_mod, c1, prec):
    torch = _torch()
    import paper_2601_19714_amd as ws
    full = c1.as_precision(prec)
    cases = [("c1 all rows", full), ("c1 first 30000 rows", full.subset(slice(0, 30000))),
             ("128^2 support 9", _random_ds(41, 5000, 128, 3, 9, prec))]
    for tag, d in cases:
        print(f"noalloc {prec}: {tag} (m={d.m}, n={d.n}, W={d.support})", flush=True)
        img, st, ref_plan, st_plan = _noalloc(ws, torch, d)
        assert np.all(np.isfinite(img))
        for k in ("n_in", "n_gridded", "n_dropped", "n_strips_occupied", "n_planes_occupied"):
            assert st[k] == st_plan[k], k
        assert st["w_lo"] == st_plan["w_lo"] and st["w_hi"] == st_plan["w_hi"]
        ref = oracle_mod.wstack_image(d.uvw_m, d.vis, d.weights, d.freq_hz, _prm(oracle_mod, d))
        full_ok = d.support <= 7 and (prec == "f64" or tag.startswith("c1"))
        _check(oracle_mod, img, ref_plan, d.n, d.support, d.beta, TOL[prec], full=full_ok, tag=f"{tag} vs plan")
        _check(oracle_mod, img, ref, d.n, d.support, d.beta, TOL[prec], full=full_ok, tag=f"{tag} vs oracle")
