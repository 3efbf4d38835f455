"""Batched channels (wsimg_image_batch): many channels of one geometry in one call.

Each channel's image must equal what the oracle makes from that channel alone (the float32
bar of 1e-5, taper-aware as in the single-channel tests) and, to rounding of the float64
grid accumulation order, what a single-channel call makes.  The workload is the 64-channel
MeerKAT-shaped set: 856-1712 MHz, each channel thinned by 0-60 % random flagging, 1024^2
images, 16 w-planes, support 7.
"""

import dataclasses

import numpy as np
import pytest

from helpers import TOL, _check, _prm, _random_ds, _torch

pytestmark = pytest.mark.gpu


def _to(torch, *arrays):
    dev = torch.device("cuda:0")
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrays]


@pytest.fixture(scope="module")
def c4():
    torch = _torch()
    import synth
    chans = synth.make_channels(device="cuda", n_channels=None)
    uvw, vis, wts, counts, freqs = synth.stack_channels(chans)
    return chans, _to(torch, uvw, vis, wts), counts, freqs


@pytest.fixture(scope="module")
def c4_images(c4):
    import paper_2601_19714_amd as ws
    chans, (u, v, w), counts, freqs = c4
    ds = chans[0]
    with ws.Plan(ds.n, ds.pixel_rad, ds.n_wplanes, ds.support, ds.beta, "f32", max_vis=sum(counts),
                 max_channels=len(counts)) as p:
        imgs, st = p.image_batch(u, v, w, counts, freqs, stats=True)
        info = p.info()
    return imgs.cpu().numpy(), st, info


def test_c4_shape_and_stats(c4, c4_images):
    chans, _, counts, freqs = c4
    imgs, st, info = c4_images
    assert len(counts) == 64 and imgs.shape == (64, 1024, 1024)
    assert info["max_channels"] == 64
    assert 0.39e6 <= min(counts) and max(counts) <= 1.0e6
    for c, s in enumerate(st):
        assert s["n_in"] == counts[c]
        assert s["n_gridded"] + s["n_dropped"] == counts[c]
        assert s["sum_w"] == s["n_gridded"]                  # unit weights
        assert s["n_planes_occupied"] >= 1
    assert np.all(np.isfinite(imgs))


@pytest.mark.parametrize("c", [0, 21, 63])
def test_c4_channel_vs_oracle(oracle_mod, c4, c4_images, c):
    chans, _, _, _ = c4
    imgs, st, _ = c4_images
    ds = chans[c]
    pr = oracle_mod.prepare(ds.uvw_m, ds.weights, ds.freq_hz, _prm(oracle_mod, ds))
    assert st[c]["n_gridded"] == pr.n_kept
    assert st[c]["w_lo"] == pr.w_lo and st[c]["w_hi"] == pr.w_hi
    ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, _prm(oracle_mod, ds), prepared=pr)
    _check(oracle_mod, imgs[c], ref, ds.n, ds.support, ds.beta, TOL["f32"], full=True, tag=f"c4 ch{c}")


def test_c4_batch_equals_single_calls(c4, c4_images):
    torch = _torch()
    import paper_2601_19714_amd as ws
    chans, (u, v, w), counts, freqs = c4
    imgs, st, _ = c4_images
    ds = chans[0]
    off = np.concatenate([[0], np.cumsum(counts)])
    worst = 0.0
    with ws.Plan(ds.n, ds.pixel_rad, ds.n_wplanes, ds.support, ds.beta, "f32", max_vis=max(counts)) as p:
        for c in range(len(counts)):
            sl = slice(int(off[c]), int(off[c + 1]))
            one, s1 = p.image(u[sl], v[sl], w[sl], freqs[c], stats=True)
            one = one.cpu().numpy()
            for key in ("n_gridded", "n_dropped", "w_lo", "w_hi", "n_strips_occupied", "n_planes_occupied"):
                assert s1[key] == st[c][key], (c, key)
            assert s1["sum_w"] == st[c]["sum_w"]
            worst = max(worst, float(np.max(np.abs(one - imgs[c])) / np.max(np.abs(one))))
    torch.cuda.synchronize()
    print(f"batch vs single calls: worst peak-relative difference {worst:.2e}")
    assert worst <= 1e-6


def test_batch_edge_cases(oracle_mod):
    """Empty channels, a zero-weight channel, uneven sizes, f64, and the argument checks."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    n, nw, W = 64, 3, 7
    sets = [_random_ds(500 + i, m, n, nw, W, "f64") for i, m in enumerate([3000, 0, 17, 5000, 257])]
    sets[2] = dataclasses.replace(sets[2], weights=np.zeros(17))         # zero total weight
    sets = [dataclasses.replace(ds, freq_hz=1.0e9 * (1.0 + 0.1 * i)) for i, ds in enumerate(sets)]
    import synth
    uvw, vis, wts, counts, freqs = synth.stack_channels(sets)
    u, v, w = _to(torch, uvw, vis, wts)
    with ws.Plan(n, sets[0].pixel_rad, nw, W, sets[0].beta, "f64", max_vis=len(wts), max_channels=8) as p:
        with pytest.raises(ws.WsimgError) as ei:
            p.image_batch(u, v, w, counts, freqs, stats=True)
        assert ei.value.status == -4                                   # zero weight in channels 1, 2
        imgs = p.image_batch(u, v, w, counts, freqs).cpu().numpy()     # without stats: no error
        for c, ds in enumerate(sets):
            if c in (1, 2):
                assert np.all(imgs[c] == 0.0), c
                continue
            ref = oracle_mod.wstack_image(ds.uvw_m, ds.vis, ds.weights, ds.freq_hz, _prm(oracle_mod, ds))
            _check(oracle_mod, imgs[c], ref, n, W, ds.beta, TOL["f64"], full=False, tag=f"edge ch{c}")
        # one channel equals wsimg_image
        one = p.image(u[:3000], v[:3000], w[:3000], freqs[0]).cpu().numpy()
        assert np.max(np.abs(one - imgs[0])) <= 1e-12 * np.max(np.abs(one))
        # argument checks
        with pytest.raises(ws.WsimgError) as ei:
            p.image_batch(u, v, w, counts + [0] * 4, freqs + [1e9] * 4)       # 9 > max_channels
        assert ei.value.status == -1
        with pytest.raises(ws.WsimgError) as ei:
            p.image_batch(u, v, w, [len(wts)] + [0] * 4, [freqs[0], 1e9, -1.0, 1e9, 1e9])
        assert ei.value.status == -1                                   # negative frequency
    with ws.Plan(n, sets[0].pixel_rad, nw, W, sets[0].beta, "f64", max_vis=100, max_channels=8) as p:
        with pytest.raises(ws.WsimgError) as ei:
            p.image_batch(u, v, w, counts, freqs)
        assert ei.value.status == -5                                   # total rows > max_vis


def test_batch_graph_capture_and_replay(c4, c4_images):
    """The 64-channel call captured into a HIP graph (torch.cuda.graph over the plan's
    stream) and replayed three times, with eager calls on the same plan and host
    synchronisations between the replays: every replay matches the eager images."""
    torch = _torch()
    import paper_2601_19714_amd as ws
    chans, (u, v, w), counts, freqs = c4
    eager, _, _ = c4_images
    ds = chans[0]
    with ws.Plan(ds.n, ds.pixel_rad, ds.n_wplanes, ds.support, ds.beta, "f32", max_vis=sum(counts),
                 max_channels=len(counts)) as p:
        out = torch.empty((len(counts), ds.n, ds.n), dtype=torch.float32, device="cuda:0")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            p.image_batch(u, v, w, counts, freqs, out=out)          # warm-up off the capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            p.image_batch(u, v, w, counts, freqs, out=out)
        scale = np.max(np.abs(eager))
        for rep in range(3):
            out.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            err = float(np.max(np.abs(got - eager)) / scale)
            print(f"replay {rep}: peak-relative difference from eager {err:.2e}")
            assert err <= 1e-6, rep
            # eager work on the same plan between replays (other channel counts)
            half = sum(counts[:32])
            p.image_batch(u[:half], v[:half], w[:half], counts[:32], freqs[:32])
            torch.cuda.synchronize()
