"""Host replay of the imaging kernels' data-dependent index arithmetic, checked against the
allocation sizes the library reports for the same plan (wsimg_plan_query, no GPU needed).

Why: the 8192^2, 64-plane, W = 9 LOFAR-shaped geometry is the one workload whose scratch
buffers land on exact powers of two (2^21 rows: a 32 MiB record buffer), so an index one past
the last record that is harmless elsewhere (the allocation granule's slack absorbs it) would
leave the mapping there.  This file recomputes, from the same float64 row geometry and the same
keys as the kernels (fp contraction off there, plain IEEE operations in numpy here), every index
that depends on the data:

  * k_key / k_scatter: bucket key, counter replica, record position;
  * the counting-sort offsets and the record fields' bit widths (13-bit tap column,
    5-bit row-in-strip, 8192 origin bins);
  * k_occupancy: strip visits, heavy / light / split work-list entries against its capacity;
  * k_origin_sort: per-bucket origin histogram bins and destinations;
  * k_grid_rows (grid_strip): each work item's record range and bucket walk, the strip rows a
    record reaches, the LDS strip index of every tap, the write into the row-transformed planes;
  * k_adj_rows (degrid_strip): the same record ranges plus the input-row table;
  * k_stack_flags / k_cols_stack: strip-flag and plane reads, image writes;

and checks each against the plan's allocation: rows <= row_capacity (max_vis plus slack),
counters, work list, LDS bytes per work-group, planes of the intermediate.

The work-group shapes are mirrored here from the kernels' compile-time rules and compared with
what the library itself reports, so a drift between the two fails the test.
"""

import json
import math
import os

import numpy as np
import pytest


def _tuned_macros():
    """The -DNAME=VALUE flags of the autotuner's record, which the library build adds."""
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2601_19714_amd", "tuned.json")
    out = {}
    if os.path.exists(path):
        with open(path) as fh:
            for f in json.load(fh).get("flags", []):
                if f.startswith("-D") and "=" in f:
                    k, v = f[2:].split("=", 1)
                    out[k] = int(v)
    return out


TUNED = _tuned_macros()

C_LIGHT = 299_792_458.0
REPLICAS = 64                 # bucket counter replicas
KEY_ROWS = 8192               # rows per key block (replica = block mod 64; the scatter follows it)
ORIGIN_BINS = 8192            # LDS histogram of the origin sort
BIG_BUCKET = 16384            # buckets above this many records are origin-sorted first, from a list
HEAVY = 4096                  # record visits above which a strip goes to the front of the list
MIN_PART = 4096
MAX_PARTS = 32
MAX_SPLIT = 512
CHUNK_MAX = {"f32": TUNED.get("WSIMG_F32_GRID_CHUNK_MAX", 64),
             "f64": TUNED.get("WSIMG_F64_GRID_CHUNK_MAX", 16)}   # records per gridding work item
MAX_LDS = 160 * 1024
CUS = 256                     # MI355X compute units (the persistent grid's size)


PAD_SHIFT = 5                 # one LDS pad slot per 32 elements


def padded(e):
    """Padded LDS elements (one slot per 32), rounded up to an even count."""
    return (e + (e >> PAD_SHIFT) + 2) & ~1


def lds_pad(e):
    return e + (e >> PAD_SHIFT)


def shape(prec, log2n):
    """The kernels' compile-time work-group shapes for a (precision, grid side) pair."""
    f32 = prec == "f32"
    N = 1 << log2n
    lr1 = min(4, log2n - 1)
    lr2_f32 = TUNED.get(f"WSIMG_F32_LR2_N{log2n}", 4 if log2n == 12 else 3)
    lr2 = min(lr2_f32 if f32 else 3, log2n - 1)
    cap1 = 8192 if log2n >= 12 else 4096
    hs = TUNED.get(f"WSIMG_STRIP_ROWS_N{log2n}", 2)           # rows per strip below 4096^2 (0: by cells)
    h0 = hs if (log2n < 12 and hs > 0) else min(4, max(1, cap1 // N))
    H = min(h0, N // 2)
    nt1 = max(64, H * N >> lr1)
    pxa = 8192 if f32 else 4096                              # column-pass work-group pixels
    px2 = (65536 if f32 else 8192) if log2n == 13 else pxa   # layout block pixels
    B = max(1, min(px2 // N, N // 2))
    BA = min(max(1, pxa // N), B)
    bs0 = 1 if f32 else 0
    BS = BA if bs0 <= 0 else min(bs0, B)
    E2 = 1 << lr2
    nt2 = max(64, BS * N // E2)
    cb = 8 if f32 else 16
    lds1 = padded(H * N)
    lds2s = padded(BS * N)
    nm1_lds = lds2s * cb + 8 * E2 * nt2 + 4096 <= MAX_LDS
    lds2s_bytes = lds2s * cb + (8 * E2 * nt2 if nm1_lds else 0) + 4096
    return dict(N=N, H=H, log2H=H.bit_length() - 1, nt1=nt1, B=B, log2B=B.bit_length() - 1, BS=BS,
                E2=E2, nt2=nt2, lds1=lds1, lds1_bytes=lds1 * 16, lds2s_bytes=lds2s_bytes, cb=cb)


def walk_rows(W):
    """Register rows per gridding walk for the support class (W <= 7: 7 taps, W = 9: 9, else 15)."""
    wmax = 7 if W <= 7 else (9 if W == 9 else 15)
    fit = TUNED.get("WSIMG_WALK_VGPRS", 64) // (wmax * 4)
    return 8 if fit >= 8 else 4 if fit >= 4 else 2 if fit >= 2 else 1


def row_geometry(uvw, wt, freq, n, pixel, W):
    """The kernels' float64 row geometry, operation for operation."""
    du = 1.0 / (float(n) * pixel)
    half_n = float(n) / 2.0
    u = uvw[:, 0] * freq / C_LIGHT
    v = uvw[:, 1] * freq / C_LIGHT
    w = uvw[:, 2] * freq / C_LIGHT
    x = u / du + half_n
    y = v / du + half_n
    cx = np.floor(x + 0.5)
    cy = np.floor(y + 0.5)
    h = float((W - 1) // 2)
    fq, fp = cx - h, cy - h
    finite = np.isfinite(uvw).all(axis=1) & np.isfinite(wt)
    with np.errstate(invalid="ignore"):
        keep = finite & (fq >= 0) & (fq + (W - 1) <= n - 1) & (fp >= 0) & (fp + (W - 1) <= n - 1)
    return x, y, w, cx, cy, keep


def plane_index(w, w_lo, dw, nw):
    if dw == 0.0:
        return np.zeros(w.shape, dtype=np.int64)
    kf = np.floor((w - w_lo) / dw)
    k = np.where(kf >= 0.0, kf, 0.0)
    return np.minimum(k, nw - 1).astype(np.int64)


def frac_code(f):
    c = np.rint((f + 0.5) * 8388608.0)
    return np.clip(c, 0, 8388607).astype(np.int64)


def replay(uvw, wt, freq, prm, info, prec):
    """Recompute every data-dependent index and check it against the plan's allocations.
    Returns a dict of the extremes found (for the record)."""
    n, W, nw, pixel = info["n_grid"], prm["support"], prm["n_wplanes"], prm["pixel_rad"]
    log2n = n.bit_length() - 1
    sh = shape(prec, log2n)
    # the mirror agrees with the library
    assert info["strip_rows"] == sh["H"] and info["col_block"] == sh["B"]
    assert info["grid_threads"] == sh["nt1"] and info["stack_threads"] == sh["nt2"]
    assert info["stack_cols"] == sh["BS"] and info["stack_radix"] == sh["E2"]
    assert info["lds_grid_bytes"] == sh["lds1_bytes"] and info["lds_stack_bytes"] == sh["lds2s_bytes"]
    assert sh["lds1_bytes"] + 8 <= MAX_LDS and sh["lds2s_bytes"] <= MAX_LDS
    H, log2H, S = sh["H"], sh["log2H"], n // sh["H"]
    nb = nw * S
    assert info["n_buckets"] == nb
    ncnt = nb * REPLICAS
    half = (W - 1) // 2
    M = uvw.shape[0]
    assert M <= info["max_vis"] < info["row_capacity"]

    x, y, w, cx, cy, keep = row_geometry(uvw, wt, freq, n, pixel, W)
    sel = keep & (wt > 0)
    w_lo, w_hi = (float(w[sel].min()), float(w[sel].max())) if sel.any() else (0.0, 0.0)
    dw = (w_hi - w_lo) / nw
    rows = np.nonzero(keep)[0]
    n_kept = rows.size
    q0 = cx[rows].astype(np.int64) - half
    p0 = cy[rows].astype(np.int64) - half
    k = plane_index(w[rows], w_lo, dw, nw)
    # k_key: bucket key and counter replica of each kept row
    kk = k * S + (p0 >> log2H)
    assert kk.min() >= 0 and kk.max() < nb
    rep = (rows // KEY_ROWS) & (REPLICAS - 1)
    cidx = kk * REPLICAS + rep
    assert cidx.max() < ncnt
    counts = np.bincount(cidx, minlength=ncnt)
    offsets = np.concatenate([[0], np.cumsum(counts)])
    assert offsets[-1] == n_kept < 2 ** 32 and len(offsets) == ncnt + 1
    # k_scatter: position = offsets[counter] + rank (ranks: 0..count-1 in any order)
    order = np.argsort(cidx, kind="stable")
    pos = np.empty(n_kept, dtype=np.int64)
    pos[order] = np.arange(n_kept)
    assert pos.max() < n_kept <= info["row_capacity"]
    assert np.all(pos >= offsets[cidx]) and np.all(pos < offsets[cidx + 1])
    # record fields (float record: 13-bit tap column, 5-bit row in strip, 23-bit offsets)
    assert q0.min() >= 0 and q0.max() < (1 << 13 if prec == "f32" else 1 << 16)
    pr = p0 & (H - 1)
    assert pr.max() < 32
    if prec == "f32":
        ux = frac_code(x[rows] - cx[rows])
        uy = frac_code(y[rows] - cy[rows])
        assert ux.max() < (1 << 23) and uy.max() < (1 << 23)
    # records in bucket order
    by_pos = np.empty(n_kept, dtype=np.int64)
    by_pos[pos] = np.arange(n_kept)
    bucket_of_rec = kk[by_pos]
    bstart = offsets[np.arange(nb + 1) * REPLICAS]            # bucket b = [bstart[b], bstart[b+1])
    # k_occupancy's big-bucket list fits its capacity (row capacity / BIG_BUCKET + 1 entries)
    n_big = int((np.diff(bstart) > BIG_BUCKET).sum())
    assert n_big < info["row_capacity"] // BIG_BUCKET + 1
    # decoding p0 from the bucket's strip and the stored row-in-strip gives the row's own p0
    strip_of_rec = bucket_of_rec % S
    assert np.array_equal((strip_of_rec << log2H) + pr[by_pos], p0[by_pos])

    # k_origin_sort: origin bins and destinations inside each bucket
    origin = (q0 << log2H) | pr
    assert origin.max() < ORIGIN_BINS
    o_rec = origin[by_pos]
    srt = np.lexsort((o_rec, bucket_of_rec))       # (bucket, origin) order, stable
    dest = np.empty(n_kept, dtype=np.int64)
    dest[srt] = np.arange(n_kept)
    b_of = bucket_of_rec
    assert np.all(dest >= bstart[b_of]) and np.all(dest < bstart[b_of + 1])

    # k_occupancy: strip visits, work-list entries
    kb = np.repeat(np.arange(nw), S)
    sidx = np.tile(np.arange(S), nw)
    slo = np.maximum(0, ((sidx << log2H) - (W - 1)) >> log2H)
    base = kb * S
    vbeg = bstart[base + slo]
    vend = bstart[base + sidx + 1]
    visits = vend - vbeg
    occ = visits > 0
    visits_call = M * ((W + H - 2) // H + 1)
    persist = CUS * max(1, MAX_LDS // sh["lds1_bytes"])
    share = max(MIN_PART, visits_call // persist)
    heavy = occ & (visits > HEAVY)
    split = heavy & (visits > 2 * share)
    parts = np.where(split, np.minimum(MAX_PARTS, -(-visits // share)), 1)
    # at most MAX_SPLIT strips get parts (whichever take the slots first): bound the entries by
    # giving the slots to the strips with the most parts
    extra = np.sort((parts - 1)[split])[::-1][:MAX_SPLIT].sum()
    entries = int(occ.sum() + extra)
    assert entries <= info["list_capacity"]

    # k_grid_rows: every work item of every entry, the records it fetches and the bucket walk
    NT = sh["nt1"]
    RW = min(walk_rows(W), H)
    NG = H // RW
    ent = np.nonzero(occ)[0]
    max_fetch = -1
    for e in ent:
        b0, b1 = int(vbeg[e]), int(vend[e])
        plist = [(b0, b1)]
        if split[e]:
            P = int(parts[e])
            L = b1 - b0
            plist = [(b0 + L * p // P, b0 + L * (p + 1) // P) for p in range(P)]
        for pb, pe in plist:
            nv = pe - pb
            if nv <= 0:
                continue
            chunk = min(max(-(-(nv * NG) // NT), 1), CHUNK_MAX[prec])
            items = -(-nv // chunk)
            last_r = pb + (items - 1) * chunk
            re = min(last_r + chunk, pe)
            max_fetch = max(max_fetch, re - 1)
    assert max_fetch < n_kept <= info["row_capacity"]
    # the walk's bucket pointer never passes strip s: every record in [vbeg, vend) of strip s
    # lies in a bucket s_lo..s of the same plane
    rec_b = np.searchsorted(bstart, np.arange(n_kept), side="right") - 1
    assert np.array_equal(rec_b, bucket_of_rec)
    # LDS strip indices of every tap a record adds in the strips it reaches (rows b in [0, W)):
    # row in strip in [0, H), column (q0 + a + n/2) mod n
    lmax = lds_pad((H - 1) * n + (n - 1))
    assert lmax < sh["lds1"]
    # the float strip is rewritten as float32 pairs in the same LDS
    assert lds_pad(H * n - 1) < 2 * sh["lds1"]
    # write into the row-transformed planes: [plane][column block][row'][B]
    B, log2B = sh["B"], sh["log2B"]
    n_img = prm["n"]
    pe_ = n * n_img
    jb_max = (H * n_img - 1) >> (log2H + log2B)
    dst_max = (nw - 1) * pe_ + ((jb_max << log2n) + n - 1) * B + (B - 1)
    assert dst_max < nw * pe_
    # split slots
    assert MAX_SPLIT * sh["lds1"] * 16 <= info["device_bytes"]

    # k_cols_stack: reads of one plane block, strip flags, image writes
    E, NT2, BS = sh["E2"], sh["nt2"], sh["BS"]
    nr = n // E
    NBs = n_img // BS
    crop = (n - n_img) // 2
    j0_max = (NBs - 1) * BS
    toff_max = ((min(NT2, BS * n // E) - 1) // BS) * B + (BS - 1)
    rd_max = (nw - 1) * pe_ + (j0_max >> log2B) * B * n + (j0_max & (B - 1)) + (E - 1) * nr * B + toff_max
    assert rd_max < nw * pe_
    assert ((min(NT2, BS * n // E) - 1) // BS) < nr          # flag word index within a plane
    assert (nr * E - 1) >> log2H < S                        # k_stack_flags: strip of the last row
    assert crop >= 0 and (n_img - 1) * n_img + (n_img - 1) < n_img * n_img

    return dict(n_kept=int(n_kept), buckets=int(nb), occupied=int(occ.sum()), list_entries=entries,
                max_fetch=int(max_fetch), max_origin=int(origin.max()), max_q0=int(q0.max()),
                w_lo=w_lo, w_hi=w_hi, heavy=int(heavy.sum()), split=int(split.sum()))


def pipelined_walk_overread(vbeg, vend, NT):
    """The largest record index a walk that fetches record r + 1 before it decodes record r,
    with no guard on the last record of its chunk, would touch: the end of the last chunk."""
    mx = -1
    for b0, b1 in zip(vbeg, vend):
        nv = int(b1 - b0)
        if nv <= 0:
            continue
        chunk = min(max(nv // NT, 1), 16)       # that walk's chunks: at most 16 records
        items = -(-nv // chunk)
        re = min(int(b0) + items * chunk, int(b1))
        mx = max(mx, re)          # one past the last record of the last chunk
    return mx


@pytest.fixture(scope="module")
def lib():
    import paper_2601_19714_amd as ws
    from paper_2601_19714_amd import _lib
    if not __import__("os").path.exists(_lib.LIB_PATH):
        from paper_2601_19714_amd import build
        build.build()
    return ws


def _prm(ds):
    return dict(n=ds.n, n_wplanes=ds.n_wplanes, support=ds.support, pixel_rad=ds.pixel_rad)


@pytest.mark.parametrize("log2n", list(range(4, 14)))
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_shape_mirror_matches_library(lib, prec, log2n):
    """The work-group shapes above are the library's, for every grid size and both precisions."""
    n = 1 << log2n
    W = 3 if n < 64 else 7
    info = lib.query(n, 1e-6, 4, W, precision=prec, max_vis=1000)
    sh = shape(prec, log2n)
    assert (info["strip_rows"], info["col_block"], info["grid_threads"], info["stack_threads"],
            info["stack_cols"], info["stack_radix"], info["lds_grid_bytes"], info["lds_stack_bytes"]) == \
           (sh["H"], sh["B"], sh["nt1"], sh["nt2"], sh["BS"], sh["E2"], sh["lds1_bytes"], sh["lds2s_bytes"])
    assert info["row_capacity"] > info["max_vis"]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_replay_lofar_geometry_2p21(lib, prec):
    """The 8192^2, 64-plane, W = 9 workload at 2^21 rows (the GPU parity test's size)."""
    import synth
    ds = synth.make_config(3, max_rows=1 << 21, geometry_only=True)
    info = lib.query(ds.n, ds.pixel_rad, ds.n_wplanes, ds.support, precision=prec, max_vis=ds.m)
    r = replay(ds.uvw_m, ds.weights.astype(np.float64), ds.freq_hz, _prm(ds), info, prec)
    print(prec, r)
    assert r["n_kept"] == ds.m          # every row of this track lands on the grid


def test_replay_meerkat_geometry():
    """The 4096^2, 32-plane, W = 7 workload (two-row strips)."""
    import paper_2601_19714_amd as ws
    import synth
    ds = synth.make_config(2, geometry_only=True)
    info = ws.query(ds.n, ds.pixel_rad, ds.n_wplanes, ds.support, precision="f32", max_vis=ds.m)
    r = replay(ds.uvw_m, ds.weights.astype(np.float64), ds.freq_hz, _prm(ds), info, "f32")
    print(r)


@pytest.mark.slow
def test_replay_lofar_geometry_full():
    """The whole 2^26-row LOFAR-shaped track."""
    import paper_2601_19714_amd as ws
    import synth
    ds = synth.make_config(3, geometry_only=True)
    info = ws.query(ds.n, ds.pixel_rad, ds.n_wplanes, ds.support, precision="f32", max_vis=ds.m)
    r = replay(ds.uvw_m, ds.weights.astype(np.float64), ds.freq_hz, _prm(ds), info, "f32")
    print(r)


def test_one_record_overread_lands_on_the_allocation_end():
    """Why a record buffer of exactly 16 * max_vis bytes was a hazard at this geometry: a walk
    that prefetches record r + 1 without a guard reads index n_kept at the end of the last
    chunk of the last occupied strip.  At 2^21 rows (all kept) that is byte 2^25, the first
    byte past a 32 MiB buffer, i.e. past a 2 MiB allocation granule boundary; on the
    MeerKAT-shaped workload (7 257 600 rows) the same byte lies inside the buffer's last
    2 MiB granule.  The library's row buffers now carry slack beyond max_vis."""
    import paper_2601_19714_amd as ws
    import synth
    granule = 2 << 20
    for cfg, rows in ((3, 1 << 21), (2, None)):
        ds = synth.make_config(cfg, max_rows=rows, geometry_only=True)
        n, W = ds.n, ds.support
        sh = shape("f32", n.bit_length() - 1)
        x, y, w, cx, cy, keep = row_geometry(ds.uvw_m, ds.weights.astype(np.float64), ds.freq_hz, n,
                                             ds.pixel_rad, W)
        n_kept = int(keep.sum())
        # strip ranges from the same keys as the replay
        rows_k = np.nonzero(keep)[0]
        sel = keep
        w_lo, w_hi = float(w[sel].min()), float(w[sel].max())
        k = plane_index(w[rows_k], w_lo, (w_hi - w_lo) / ds.n_wplanes, ds.n_wplanes)
        S = n // sh["H"]
        kk = k * S + ((cy[rows_k].astype(np.int64) - (W - 1) // 2) >> sh["log2H"])
        bstart = np.concatenate([[0], np.cumsum(np.bincount(kk, minlength=ds.n_wplanes * S))])
        sidx = np.tile(np.arange(S), ds.n_wplanes)
        base = np.repeat(np.arange(ds.n_wplanes), S) * S
        slo = np.maximum(0, ((sidx << sh["log2H"]) - (W - 1)) >> sh["log2H"])
        top = pipelined_walk_overread(bstart[base + slo], bstart[base + sidx + 1], sh["nt1"])
        assert top == n_kept == ds.m
        exact = 16 * ds.m
        byte = 16 * top
        if cfg == 3:
            assert byte == exact and exact % granule == 0     # first byte of the next granule
        else:
            assert byte == exact and exact % granule != 0     # inside the last granule
        info = ws.query(n, ds.pixel_rad, ds.n_wplanes, W, precision="f32", max_vis=ds.m)
        assert top < info["row_capacity"]
