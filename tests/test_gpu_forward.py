"""GPU parity of rich_propagate / rich_propagate_batch against the FP64 oracle (through the C ABI)."""

import numpy as np
import pytest

from paper_2309_12496_amd import inputs as I
from parity import compare, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2309_12496_amd import rich
    return rich


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    return oracle


@pytest.fixture(scope="module")
def c1(R, orc):
    cfg = I.config(1)
    return cfg, R.Scene(cfg["scene"]), orc.Scene(cfg["scene"])


@pytest.fixture(scope="module")
def c2(R, orc):
    cfg = I.config(2)
    return cfg, R.Scene(cfg["scene"]), orc.Scene(cfg["scene"])


def _hist_counts_consistent(out, nx, ny):
    fate = to_np(out["fate"])
    pix = to_np(out["pixel"])
    hist = to_np(out["histogram"]).astype(np.int64)
    counts = to_np(out["fate_counts"])
    assert counts.sum() == len(fate)
    assert np.array_equal(counts, np.bincount(fate, minlength=7))
    assert np.array_equal(hist, np.bincount(pix[fate == 0], minlength=nx * ny))


def test_c1_all_photons(R, orc, c1):
    cfg, gs, os_ = c1
    n = cfg["n_photons"]
    out = R.propagate(gs, cfg["source"], n, cfg["seed"])
    ref = orc.propagate(os_, cfg["source"], n, cfg["seed"])
    rep = compare(out, ref, label="C1")
    _hist_counts_consistent(out, gs.nx, gs.ny)
    assert gs.status() == 0
    print(rep)


@pytest.mark.parametrize("n,first", [(1, 0), (63, 5), (257, 1000), (4097, 123456789)])
def test_c1_ragged_sizes_and_offsets(R, orc, c1, n, first):
    cfg, gs, os_ = c1
    out = R.propagate(gs, cfg["source"], n, cfg["seed"], first_id=first)
    ref = orc.propagate(os_, cfg["source"], n, cfg["seed"], first_id=first)
    compare(out, ref, min_agree=1.0 if n < 1000 else 0.9999, label=f"C1 n={n} first={first}")


@pytest.mark.parametrize("first,seed", [(2**63 + 12345, None), (2**64 - 2000, None), (0, 2**64 - 1), (77, 2**32)])
def test_extreme_ids_and_seeds(R, orc, c1, first, seed):
    """Photon ids and seeds that use both 32-bit halves of the Philox counter and key (ids up to 2^64 - 1001)."""
    cfg, gs, os_ = c1
    seed = cfg["seed"] if seed is None else seed
    n = 1000
    out = R.propagate(gs, cfg["source"], n, seed, first_id=first)
    ref = orc.propagate(os_, cfg["source"], n, seed, first_id=first)
    # 1000 photons: a single explained disagreement is already 1e-3, so only explained ones are allowed
    compare(out, ref, min_agree=0.99, label=f"C1 first={first} seed={seed}")


@pytest.mark.parametrize("n,first,prefilter", [(1, 0, False), (63, 7, False), (1025, 1000, False), (3000, 123457, False),
                                                (8193, 3, False), (32769, 11, False), (1025, 5, True),
                                                (2500, 999, True), (16385, 77, True)])
def test_meshed_regrouping_at_ragged_sizes(R, orc, c2, n, first, prefilter):
    """The sorted order (windows of 32,768 ids sorted by azimuth, 8192 with the pre-filter, whose
    rejects go last; fewer than eight blocks below 2048 photons) at sizes and offsets that leave
    partial windows, photon by photon against the oracle."""
    cfg, gs, os_ = c2
    src = I.with_prefilter(cfg["source"]) if prefilter else cfg["source"]
    out = R.propagate(gs, src, n, cfg["seed"], first_id=first)
    ref = orc.propagate(os_, src, n, cfg["seed"], first_id=first)
    compare(out, ref, min_agree=0.99, label=f"C2 regroup n={n} first={first} pf={prefilter}")
    counts = to_np(out["fate_counts"])
    assert counts.sum() == n and counts[R.PREFILTERED] == int((ref["fate"] == orc.PREFILTERED).sum())


def test_zero_photons_is_a_no_op(R, c1):
    import torch
    cfg, gs, _ = c1
    t, o = R.alloc_outputs(gs, 1)
    t["fate"].fill_(77)
    s, keep = R.make_source(cfg["source"])
    R.rich_propagate(gs.handle, s, 0, cfg["seed"], 0, o)
    torch.cuda.synchronize()
    assert int(t["fate"][0]) == 77 and int(t["fate_counts"].sum()) == 0


def test_split_ranges_are_bit_identical(R, c2):
    cfg, gs, _ = c2
    n = 300_000
    full = R.propagate(gs, cfg["source"], n, cfg["seed"])
    a = R.propagate(gs, cfg["source"], 123_457, cfg["seed"], first_id=0)
    b = R.propagate(gs, cfg["source"], n - 123_457, cfg["seed"], first_id=123_457)
    for k in ("fate", "pixel"):
        assert np.array_equal(to_np(full[k]), np.concatenate([to_np(a[k]), to_np(b[k])]))
    fx = to_np(full["hit_xyz"])
    ab = np.concatenate([to_np(a["hit_xyz"]), to_np(b["hit_xyz"])])
    assert np.array_equal(fx, ab, equal_nan=True)
    assert np.array_equal(to_np(full["histogram"]), to_np(a["histogram"]) + to_np(b["histogram"]))


def test_large_analytic_launch_claims_ids(R, orc, c1):
    """Analytic launches of 2^22 photons or more hand ids to waves through per-XCD claim counters
    instead of a grid-stride loop: one such call equals, bit for bit, the same ids traced by two
    smaller (grid-stride) calls, and its last photons match the oracle."""
    import torch
    cfg, gs, os_ = c1
    n = (1 << 22) + 777
    half = n // 2
    full = R.propagate(gs, cfg["source"], n, cfg["seed"])
    a = R.propagate(gs, cfg["source"], half, cfg["seed"], first_id=0)
    b = R.propagate(gs, cfg["source"], n - half, cfg["seed"], first_id=half)
    for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time"):
        fk = to_np(full[k])
        assert np.array_equal(fk, np.concatenate([to_np(a[k]), to_np(b[k])]), equal_nan=fk.dtype.kind == "f"), k
    assert np.array_equal(to_np(full["fate_counts"]), to_np(a["fate_counts"]) + to_np(b["fate_counts"]))
    assert np.array_equal(to_np(full["histogram"]), to_np(a["histogram"]) + to_np(b["histogram"]))
    m = 5000
    tail = {k: v[n - m:] for k, v in full.items() if k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time")}
    compare(tail, orc.propagate(os_, cfg["source"], m, cfg["seed"], first_id=n - m), min_agree=0.999,
            label="C1 claimed ids, tail")
    del full, a, b
    torch.cuda.empty_cache()
    assert gs.status() == 0


def test_sorted_launch_beyond_one_chunk(R, orc, c2):
    """A forward launch on a meshed scene traces its photons in an order sorted by cone azimuth, in
    chunks of 2^24 photons (the order buffer's size).  One call of 2^24 + 4321 photons (two chunks,
    the second a ragged window) equals, bit for bit, the same ids traced by two calls split elsewhere;
    the photons of the second chunk match the oracle."""
    import torch
    cfg, gs, os_ = c2
    chunk = 1 << 24
    n, cut = chunk + 4321, 10_000_000
    full = R.propagate(gs, cfg["source"], n, cfg["seed"])
    a = R.propagate(gs, cfg["source"], cut, cfg["seed"], first_id=0)
    b = R.propagate(gs, cfg["source"], n - cut, cfg["seed"], first_id=cut)
    for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time"):
        fk = to_np(full[k])
        assert np.array_equal(fk, np.concatenate([to_np(a[k]), to_np(b[k])]), equal_nan=fk.dtype.kind == "f"), k
    assert np.array_equal(to_np(full["fate_counts"]), to_np(a["fate_counts"]) + to_np(b["fate_counts"]))
    assert np.array_equal(to_np(full["histogram"]), to_np(a["histogram"]) + to_np(b["histogram"]))
    assert int(to_np(full["fate_counts"]).sum()) == n
    tail = {k: v[chunk:] for k, v in full.items() if k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time")}
    ref = orc.propagate(os_, cfg["source"], n - chunk, cfg["seed"], first_id=chunk)
    compare(tail, ref, min_agree=0.999, label="C2 second chunk")
    del full, a, b
    torch.cuda.empty_cache()
    assert gs.status() == 0


def test_sorted_launch_with_outputs_left_out(R, c2):
    """Every per-photon output is optional: a sorted launch that asks only for the arrival times
    (and the fate counts) writes the same times as one that asks for everything."""
    import torch
    cfg, gs, _ = c2
    n = 100_000
    ref = R.propagate(gs, cfg["source"], n, cfg["seed"])
    s, keep = R.make_source(cfg["source"])
    t, o = R.alloc_outputs(gs, n)
    for f in ("fate", "pixel", "hit_xyz", "hit_uv"):
        setattr(o, f, None)
    R.rich_propagate(gs.handle, s, n, cfg["seed"], 0, o)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(t["hit_time"]), to_np(ref["hit_time"]), equal_nan=True)
    assert np.array_equal(to_np(t["fate_counts"]), to_np(ref["fate_counts"]))
    assert gs.status() == 0


def test_c2_meshed_subset_at_full_size(R, orc, c2):
    """The 1e7-photon launch as the benchmark runs it; every 100th photon checked against the oracle."""
    cfg, gs, os_ = c2
    n = cfg["n_photons"]
    out = R.propagate(gs, cfg["source"], n, cfg["seed"])
    ids = np.arange(0, n, 100, dtype=np.uint64)
    ref = orc.propagate(os_, cfg["source"], 0, cfg["seed"], ids=ids)
    sub = {k: to_np(out[k])[ids.astype(np.int64)] for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time")}
    rep = compare(sub, ref, label="C2 subset")
    _hist_counts_consistent(out, gs.nx, gs.ny)
    assert gs.status() == 0
    print(rep)


def test_c2_brute_force_oracle_small(R, orc, c2):
    """First 1000 photons against the oracle's brute-force scan over all 210k triangles."""
    cfg, gs, os_ = c2
    out = R.propagate(gs, cfg["source"], 1000, cfg["seed"])
    ref = orc.propagate(os_, cfg["source"], 1000, cfg["seed"], use_bvh=False)
    compare(out, ref, min_agree=0.999, label="C2 brute force")


def test_explicit_photons(R, orc, c1):
    """Photons handed over one by one (origin, direction, wavelength)."""
    cfg, gs, os_ = c1
    rng = np.random.default_rng(17)
    m = 20000
    o = rng.uniform(-200, 200, size=(m, 3)) * [1, 1, 0.5]
    th = rng.uniform(0, 0.3, m)
    ph = rng.uniform(0, 2 * np.pi, m)
    d = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
    src = I.explicit_source(o, d, rng.uniform(200, 600, m))
    out = R.propagate(gs, src, m, cfg["seed"])
    ref = orc.propagate(os_, src, m, cfg["seed"])
    compare(out, ref, label="explicit")


def test_on_axis_ring_radius(R):
    """T0 scene on the GPU: every photon on the circle r = (R/2) theta_c."""
    sc = I.scene_t0()
    gs = R.Scene(sc)
    out = R.propagate(gs, I.point_source(), 20000, 7)
    fate = to_np(out["fate"])
    assert np.all(fate == 0)
    uv = to_np(out["hit_uv"]).astype(np.float64)
    r = np.hypot(uv[:, 0], uv[:, 1])
    want = 0.5 * I.R_MIRROR * np.arccos(1 / 1.0014)
    assert abs(r.mean() / want - 1) < 2e-4
    assert r.std() < 5e-3


def test_max_bounces_zero(R, orc):
    sc = I.scene_g1()
    sc["max_bounces"] = 0
    gs = R.Scene(sc)
    out = R.propagate(gs, I.point_source(), 1000, 1)
    assert np.all(to_np(out["fate"]) == R.MAX_BOUNCES)


def test_hit_list_and_overflow_flag(R, c1):
    import torch
    cfg, gs, _ = c1
    n = 50000
    out = R.propagate(gs, cfg["source"], n, cfg["seed"], hit_list_capacity=n)
    torch.cuda.synchronize()
    cnt = int(out["hit_count"][0])
    fate = to_np(out["fate"])
    assert cnt == int((fate == 0).sum())
    ids, pix, xyz = R.decode_hits(out["hit_list"], cnt)
    order = np.argsort(ids)
    det = np.where(fate == 0)[0]
    assert np.array_equal(ids[order], det.astype(np.uint64))
    assert np.array_equal(pix[order], to_np(out["pixel"])[det])
    assert np.array_equal(xyz[order], to_np(out["hit_xyz"])[det])
    assert gs.status() == 0
    small = R.propagate(gs, cfg["source"], n, cfg["seed"], hit_list_capacity=1)
    torch.cuda.synchronize()
    assert int(small["hit_count"][0]) == cnt              # the count keeps running past the capacity
    assert gs.status() & R.FLAG_HITLIST_OVERFLOW
    assert gs.status() == 0                                # reading the flags clears them


def test_null_outputs_are_skipped(R, c1):
    import torch
    cfg, gs, _ = c1
    s, keep = R.make_source(cfg["source"])
    t = {"fate_counts": torch.zeros(7, dtype=torch.int64, device="cuda")}
    o = R.outputs_struct(t)
    R.rich_propagate(gs.handle, s, 10000, cfg["seed"], 0, o)
    torch.cuda.synchronize()
    assert int(t["fate_counts"].sum()) == 10000


def test_invalid_source_is_rejected(R, c1):
    cfg, gs, _ = c1
    bad = I.point_source(beta=0.99)
    s, keep = R.make_source(bad)
    t, o = R.alloc_outputs(gs, 10)
    with pytest.raises(R.RichError) as e:
        R.rich_propagate(gs.handle, s, 10, 1, 0, o)
    assert e.value.code == R.RICH_EINVAL
    with pytest.raises(R.RichError) as e:
        R.rich_propagate(gs.handle, R.make_source(cfg["source"])[0], 10, 1, 2**64 - 5, o)
    assert e.value.code == R.RICH_ERANGE


def test_c3_batch_subset(R, orc):
    """Persistent batched launch over 4096 Poisson-sized tracks; every 41st photon checked, with a
    fixed launch shape and with the autotuned one the benchmark uses (identical results)."""
    cfg = I.config(3)
    gs = R.Scene(cfg["scene"])
    out = R.propagate_batch(gs, cfg["source"], cfg["seed"], tune=R.tuning(256, 256, 4))
    n = cfg["n_photons"]
    ids = np.arange(0, n, 41, dtype=np.uint64)
    ref = orc.propagate(cfg["scene"], cfg["source"], 0, cfg["seed"], ids=ids)
    sub = {k: to_np(out[k])[ids.astype(np.int64)] for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time")}
    compare(sub, ref, label="C3 subset")
    _hist_counts_consistent(out, gs.nx, gs.ny)
    auto = R.propagate_batch(gs, cfg["source"], cfg["seed"])
    for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time", "histogram", "fate_counts"):
        assert np.array_equal(to_np(auto[k]), to_np(out[k]), equal_nan=True), k
    assert gs.status() == 0


def test_sorted_forward_in_a_captured_graph(R, c2):
    """A meshed forward launch (sort kernel, then the trace whose waves claim positions from
    counters the sort zeroes) captured into a HIP graph after a warm-up call (which grows the
    stream's order buffer) replays to the eager per-photon outputs every time, with eager work
    between the replays; fate counts and the histogram accumulate once per replay."""
    import torch
    cfg, gs, _ = c2
    n = 300_001
    ref = R.propagate(gs, cfg["source"], n, cfg["seed"])
    s, keep = R.make_source(cfg["source"])
    t, o = R.alloc_outputs(gs, n)
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        R.rich_propagate(gs.handle, s, n, cfg["seed"], 0, o, cs)   # warm-up: the stream's buffers
    cs.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cs):
        R.rich_propagate(gs.handle, s, n, cfg["seed"], 0, o, cs)
    for rep in range(3):
        for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time"):
            t[k].zero_()
        g.replay()
        torch.cuda.synchronize()
        other = R.propagate(gs, cfg["source"], 1000, cfg["seed"] + rep)   # eager work between replays
        assert int(to_np(other["fate_counts"]).sum()) == 1000
        for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time"):
            a, b = to_np(t[k]), to_np(ref[k])
            assert np.array_equal(a, b, equal_nan=a.dtype.kind == "f"), (rep, k)
        assert np.array_equal(to_np(t["fate_counts"]), (rep + 2) * to_np(ref["fate_counts"]))
        assert np.array_equal(to_np(t["histogram"]), (rep + 2) * to_np(ref["histogram"]))
    assert gs.status() == 0


def test_batch_graph_replay_matches_eager_single_source(R):
    """The batch graph replays to the same result every time, and equals per-track single-source calls."""
    import torch
    cfg = I.config(3)
    gs = R.Scene(cfg["scene"])
    b, keep, n = R.make_batch(cfg["source"])
    t, o = R.alloc_outputs(gs, n)
    tune = R.tuning(128, 128, 4)
    first = None
    for rep in range(3):
        t["histogram"].zero_()
        t["fate_counts"].zero_()
        R.rich_propagate_batch(gs.handle, b, n, cfg["seed"], o, tune)
        torch.cuda.synchronize()
        snap = {k: to_np(t[k]).copy() for k in ("fate", "pixel", "hit_xyz", "histogram", "fate_counts")}
        if first is None:
            first = snap
        else:
            for k in snap:
                assert np.array_equal(snap[k], first[k], equal_nan=True), k
        x = torch.ones(1000, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        assert float(x) == 1000.0
    # a few tracks alone through rich_propagate (same global ids, same photons)
    offs = np.asarray(cfg["source"]["offsets"], np.int64)
    for k in (0, 1234, 4095):
        tr = cfg["source"]["tracks"][k]
        src = I.point_source(origin=tr[0:3], direction=tr[3:6], beta=tr[7], length=tr[6])
        cnt = int(offs[k + 1] - offs[k])
        one = R.propagate(gs, src, cnt, cfg["seed"], first_id=int(offs[k]))
        sl = slice(int(offs[k]), int(offs[k + 1]))
        agree = (to_np(one["fate"]) == first["fate"][sl]) & (to_np(one["pixel"]) == first["pixel"][sl])
        assert agree.mean() >= 0.999


def test_track_below_threshold_gives_no_light(R, orc):
    """Device tracks are not checked on the host: photons of a track with n beta <= 1 come out
    ESCAPED untraced; the photons of the tracks before it are the oracle's, those after it are traced."""
    cfg = I.config(3)
    rng = np.random.default_rng(8)
    tracks = I.sample_tracks(rng, 6)
    tracks[2, 7] = I.f32(0.99)                      # 1.0014 * 0.99 < 1
    src = I.batch_source(tracks, np.full(6, 500))
    gs = R.Scene(cfg["scene"])
    out = R.propagate_batch(gs, src, 99, tune=R.tuning(64, 64, 1))
    fate = to_np(out["fate"])
    assert np.all(fate[1000:1500] == R.ESCAPED)
    assert (fate[1500:] != R.ESCAPED).mean() > 0.5
    ref = orc.propagate(cfg["scene"], I.batch_source(tracks[:2], np.full(2, 500)), 1000, 99)
    sub = {k: to_np(out[k])[:1000] for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time")}
    compare(sub, ref, min_agree=0.99, label="tracks before the dead one")
    assert gs.status() == 0


@pytest.mark.parametrize("chunk", [64, 320, 768])
def test_batch_chunks_that_are_not_whole_regroup_slices(R, orc, chunk):
    """Chunks need only be multiples of 64; those that are not whole 256-photon regrouping slices
    must still trace every photon exactly once."""
    cfg = I.config(3)
    gs = R.Scene(cfg["scene"])
    out = R.propagate_batch(gs, cfg["source"], cfg["seed"], tune=R.tuning(128, chunk, 2))
    n = cfg["n_photons"]
    assert int(to_np(out["fate_counts"]).sum()) == n
    _hist_counts_consistent(out, gs.nx, gs.ny)
    ids = np.arange(5, n, 997, dtype=np.uint64)
    ref = orc.propagate(cfg["scene"], cfg["source"], 0, cfg["seed"], ids=ids)
    sub = {k: to_np(out[k])[ids.astype(np.int64)] for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time")}
    compare(sub, ref, label=f"C3 chunk {chunk}")


def test_batch_graph_follows_every_source_field(R):
    """The captured batch graph is reused only while all launch arguments match: switching the
    pre-filter or the dispersion on the same batch struct and outputs must change the photons."""
    import torch
    cfg = I.config(3)
    gs = R.Scene(cfg["scene"])
    b, keep, n = R.make_batch(cfg["source"])
    t, o = R.alloc_outputs(gs, n)
    tune = R.tuning(256, 256, 4)
    R.rich_propagate_batch(gs.handle, b, n, cfg["seed"], o, tune)
    plain = to_np(t["fate"]).copy()
    R._set_prefilter(b.prefilter, [I.MIRROR, I.MIRROR])
    R.rich_propagate_batch(gs.handle, b, n, cfg["seed"], o, tune)
    pre = to_np(t["fate"]).copy()
    assert (pre == R.PREFILTERED).mean() > 0.5 and not (plain == R.PREFILTERED).any()
    b.prefilter.enabled = 0
    R._set_dispersion(b.dispersion, I.gas_dispersion(), keep)
    R.rich_propagate_batch(gs.handle, b, n, cfg["seed"], o, tune)
    disp = to_np(t["hit_time"]).copy()
    b.dispersion.n_nodes = 0
    R.rich_propagate_batch(gs.handle, b, n, cfg["seed"], o, tune)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(t["fate"]), plain)
    again = to_np(t["hit_time"])
    on = np.isfinite(again) & np.isfinite(disp)
    assert on.sum() > 1000 and not np.array_equal(again[on], disp[on])


def test_prefilter_mode_parity(R, orc, c2):
    """The paper's accept-reject before propagation (Section 4.3), photon by photon against the oracle."""
    cfg, gs, os_ = c2
    src = I.with_prefilter(cfg["source"])
    n = 200_000
    out = R.propagate(gs, src, n, cfg["seed"])
    ref = orc.propagate(os_, src, n, cfg["seed"])
    compare(out, ref, label="prefilter")
    fate = to_np(out["fate"])
    assert set(np.unique(fate)) <= {R.DETECTED, R.PREFILTERED, R.ABSORBED}
    _hist_counts_consistent(out, gs.nx, gs.ny)


def test_prefilter_batch_and_validation(R, orc):
    cfg = I.config(3)
    gs = R.Scene(cfg["scene"])
    src = I.with_prefilter(cfg["source"])
    out = R.propagate_batch(gs, src, cfg["seed"], tune=R.tuning(128, 128, 4))
    ids = np.arange(0, cfg["n_photons"], 97, dtype=np.uint64)
    ref = orc.propagate(cfg["scene"], src, 0, cfg["seed"], ids=ids)
    sub = {k: to_np(out[k])[ids.astype(np.int64)] for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time")}
    compare(sub, ref, label="prefilter batch")
    bad = I.with_prefilter(I.point_source(), mirror_materials=(I.ABSORBER,))
    s, keep = R.make_source(bad)
    t, o = R.alloc_outputs(gs, 10)
    with pytest.raises(R.RichError) as e:
        R.rich_propagate(gs.handle, s, 10, 1, 0, o)
    assert e.value.code == R.RICH_EINVAL


def test_autotune_cache_file(R, orc, tmp_path, monkeypatch):
    """rich_propagate_batch with no tuning autotunes once and stores the shape under RICH_TUNE_CACHE;
    another scene of the same kind reads it back instead of tuning; an invalid stored shape is replaced."""
    import json
    path = tmp_path / "tune.json"
    monkeypatch.setenv("RICH_TUNE_CACHE", str(path))
    cfg = I.config(3)
    src = I.poisson_batch(3, 512, 1000.0, clip=(50, 5000))
    gs = R.Scene(cfg["scene"])
    first = R.propagate_batch(gs, src, cfg["seed"])
    stored = json.loads(path.read_text())
    assert len(stored) == 1
    key, (block, chunk, bpc) = next(iter(stored.items()))
    assert block in (64, 128, 256, 512) and chunk % 64 == 0 and bpc >= 1
    path.write_text(json.dumps({key: [64, 128, 1]}))
    text = path.read_text()
    again = R.propagate_batch(R.Scene(cfg["scene"]), src, cfg["seed"])
    assert path.read_text() == text                      # read, not re-tuned
    for k in ("fate", "pixel", "hit_xyz"):
        assert np.array_equal(to_np(first[k]), to_np(again[k]), equal_nan=True), k
    path.write_text(json.dumps({key: [63, 100, 0]}))      # not a valid shape: tuned and stored again
    R.propagate_batch(R.Scene(cfg["scene"]), src, cfg["seed"])
    block, chunk, bpc = json.loads(path.read_text())[key]
    assert block in (64, 128, 256, 512) and chunk % 64 == 0 and bpc >= 1


def test_batch_with_empty_tracks(R, orc):
    """Tracks with no photons (first, in runs in the middle, last) take no ids: every photon
    still belongs to the track its offset range names, on the meshed scene with regrouping."""
    cfg = I.config(3)
    rng = np.random.default_rng(31)
    tracks = I.sample_tracks(rng, 40)
    counts = rng.integers(1, 700, size=40)
    counts[[0, 7, 8, 9, 21, 39]] = 0
    src = I.batch_source(tracks, counts)
    n = int(counts.sum())
    gs = R.Scene(cfg["scene"])
    for tune in (R.tuning(256, 256, 4), R.tuning(64, 64, 2)):
        out = R.propagate_batch(gs, src, cfg["seed"], tune=tune)
        assert int(to_np(out["fate_counts"]).sum()) == n
        ids = np.arange(0, n, 7, dtype=np.uint64)
        ref = orc.propagate(cfg["scene"], src, 0, cfg["seed"], ids=ids)
        sub = {k: to_np(out[k])[ids.astype(np.int64)] for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time")}
        compare(sub, ref, label=f"empty tracks {tune.block}x{tune.chunk}")
    assert gs.status() == 0


def test_batch_without_photons_is_a_no_op(R):
    """Every track empty: n_photons = 0 returns at once and writes nothing."""
    import torch
    cfg = I.config(3)
    src = I.batch_source(I.sample_tracks(np.random.default_rng(5), 3), [0, 0, 0])
    gs = R.Scene(cfg["scene"])
    b, keep, n = R.make_batch(src)
    assert n == 0
    t, o = R.alloc_outputs(gs, 1)
    t["fate"].fill_(77)
    R.rich_propagate_batch(gs.handle, b, 0, cfg["seed"], o, None)
    torch.cuda.synchronize()
    assert int(t["fate"][0]) == 77 and int(t["histogram"].sum()) == 0 and int(t["fate_counts"].sum()) == 0


def test_coincident_triangles_and_closed_edges(R, orc):
    """Two coincident copies of a fan-triangulated square, a mirror and an absorber: the copy listed
    first (lower primitive index) decides every photon, also photons through the fan's centre, along
    its inner edges and on its outer boundary (edges are closed and shared edges leak nothing);
    zero-area triangles in the mesh are never hit."""
    src = I.coincident_photons()
    n = len(src["lambda"])
    for mirror_first, fate in ((True, R.DETECTED), (False, R.ABSORBED)):
        sc = I.scene_coincident(mirror_first)
        gs = R.Scene(sc)
        out = R.propagate(gs, src, n, 1)
        assert (to_np(out["fate"]) == fate).all(), sc["name"]
        compare(out, orc.propagate(sc, src, n, 1), label=sc["name"])


def test_closed_triangle_box_is_watertight(R, orc):
    """Photons from inside a closed tessellated box (10,092 triangles), aimed at its vertices and
    edge midpoints, never slip out between triangles."""
    import copy
    box = I.box_mesh(I.BOX_LO, I.BOX_HI, 29)
    sc = copy.deepcopy(I.scene_g2())
    sc["box"] = None
    sc["meshes"] = [{"vertices": box, "material": I.ABSORBER, "segment": -1}]
    rng = np.random.default_rng(9)
    m = 20000
    o = rng.uniform(I.BOX_LO + 10, I.BOX_HI - 10, size=(m, 3))
    verts = box.reshape(-1, 3)
    k = rng.integers(0, len(box), m // 2)
    tgt = np.concatenate([verts[rng.integers(0, len(verts), m // 2)], 0.5 * (box[k, 0] + box[k, 1])])
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    src = I.explicit_source(o, d, np.full(m, 400.0))
    gs = R.Scene(sc)
    out = R.propagate(gs, src, m, 3)
    assert not (to_np(out["fate"]) == R.ESCAPED).any()
    compare(out, orc.propagate(sc, src, m, 3), label="closed box")
    # grazing photons: within 1 mm of a wall, 1e-7..1e-2 rad off parallel to it, and photons aimed
    # at the lines where two walls meet
    lo, hi = np.asarray(I.BOX_LO, float), np.asarray(I.BOX_HI, float)
    ax, side = rng.integers(0, 3, m), rng.integers(0, 2, m)
    o = rng.uniform(lo + 10, hi - 10, size=(m, 3))
    o[np.arange(m), ax] = np.where(side == 1, hi[ax], lo[ax]) + np.where(side == 1, -1, 1) * rng.uniform(1e-3, 1, m)
    d = rng.normal(size=(m, 3))
    d[np.arange(m), ax] = 0
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d[np.arange(m), ax] = np.where(side == 1, 1, -1) * np.tan(10 ** rng.uniform(-7, -2, m))
    e = rng.integers(0, 3, m)
    corner = np.where(rng.integers(0, 2, (m, 3)) == 1, hi, lo).astype(float)
    corner[np.arange(m), e] = rng.uniform(lo[e], hi[e])
    o2 = rng.uniform(lo + 10, hi - 10, size=(m, 3))
    for oo, dd in ((o, d), (o2, corner - o2)):
        dd = dd / np.linalg.norm(dd, axis=1, keepdims=True)
        out = R.propagate(gs, I.explicit_source(oo, dd, np.full(m, 400.0)), m, 3)
        assert not (to_np(out["fate"]) == R.ESCAPED).any()


def test_batch_size_other_than_the_track_total_is_flagged(R, orc):
    """n_photons below offsets[n_tracks]: the first n photons are traced as usual and the device
    raises RICH_FLAG_BATCH_SIZE (read and cleared by rich_get_status); the whole batch raises nothing."""
    cfg = I.config(3)
    src = I.batch_source(cfg["source"]["tracks"][:50], np.full(50, 300))
    gs = R.Scene(cfg["scene"])
    b, keep, n = R.make_batch(src)
    t, o = R.alloc_outputs(gs, n - 5)
    R.rich_propagate_batch(gs.handle, b, n - 5, cfg["seed"], o, R.tuning(256, 256, 4))
    assert gs.status() == R.FLAG_BATCH_SIZE
    assert gs.status() == 0
    ids = np.arange(0, n - 5, 11, dtype=np.uint64)
    ref = orc.propagate(cfg["scene"], src, 0, cfg["seed"], ids=ids)
    sub = {k: to_np(t[k])[ids.astype(np.int64)] for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time")}
    compare(sub, ref, label="batch prefix")
    out = R.propagate_batch(gs, src, cfg["seed"], tune=R.tuning(256, 256, 4))
    assert gs.status() == 0 and int(to_np(out["fate_counts"]).sum()) == n


def test_batch_processing_order_with_empty_tracks(R, orc):
    """Large batches on meshed scenes are processed in an order of the tracks by direction dealt to
    the XCD partitions: with tracks of no photons among them (first, a run in the middle, last),
    every photon still gets its own id, random numbers and results (2.4e6 photons: the order is on).
    With n_photons one short of the total the order is off and the prefix is traced in id order."""
    cfg = I.config(3)
    rng = np.random.default_rng(33)
    tracks = I.sample_tracks(rng, 600)
    counts = rng.integers(1000, 7000, size=600)
    counts[[0, 100, 101, 102, 599]] = 0
    src = I.batch_source(tracks, counts)
    n = int(counts.sum())
    assert n >= 1 << 21
    gs = R.Scene(cfg["scene"])
    ids = np.arange(0, n, 97, dtype=np.uint64)
    ref = orc.propagate(cfg["scene"], src, 0, cfg["seed"], ids=ids)
    for tune in (R.tuning(256, 256, 4), R.tuning(512, 1024, 1)):
        print(f"ordered batch {tune.block}x{tune.chunk}x{tune.blocks_per_cu}: {n} photons", flush=True)
        out = R.propagate_batch(gs, src, cfg["seed"], tune=tune)
        sub = {k: to_np(out[k])[ids.astype(np.int64)] for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time")}
        compare(sub, ref, label=f"ordered batch {tune.block}x{tune.chunk}")
        _hist_counts_consistent(out, gs.nx, gs.ny)
        assert gs.status() == 0
    b, keep, nb = R.make_batch(src)
    t, o = R.alloc_outputs(gs, n - 1)
    R.rich_propagate_batch(gs.handle, b, n - 1, cfg["seed"], o, R.tuning(256, 256, 4))
    assert gs.status() == R.FLAG_BATCH_SIZE
    pre = ids[ids < n - 1]
    sub = {k: to_np(t[k])[pre.astype(np.int64)] for k in ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time")}
    refp = {k: v[: len(pre)] for k, v in ref.items()}
    compare(sub, refp, label="batch prefix, order off")


def test_hit_list_with_regrouped_photons(R, c2):
    """The compact hit list when photons are traced out of id order (regrouped by azimuth), from the
    forward kernel on the meshed scene and from the persistent batch kernel: exactly the DETECTED
    photons, each once, with their own pixel and position."""
    import torch
    cfg, gs, _ = c2
    n = 300_000
    runs = [R.propagate(gs, cfg["source"], n, cfg["seed"], hit_list_capacity=n)]
    c3 = I.config(3)
    src = I.batch_source(c3["source"]["tracks"][:300], np.full(300, 1000))
    runs.append(R.propagate_batch(gs, src, cfg["seed"], tune=R.tuning(256, 256, 4), hit_list_capacity=300_000))
    for out in runs:
        torch.cuda.synchronize()
        fate = to_np(out["fate"])
        cnt = int(out["hit_count"][0])
        det = np.flatnonzero(fate == 0)
        assert cnt == len(det) > 1000
        ids, pix, xyz = R.decode_hits(out["hit_list"], cnt)
        order = np.argsort(ids)
        assert np.array_equal(ids[order], det.astype(np.uint64))
        assert np.array_equal(pix[order], to_np(out["pixel"])[det])
        assert np.array_equal(xyz[order], to_np(out["hit_xyz"])[det])
    assert gs.status() == 0


def test_side_stream_launches(R, c2):
    """Forward, batch (graph replay) and adjoint launched on a non-default stream give the results of
    the same calls on the default stream (all three are enqueued on the stream they are given)."""
    import torch
    cfg, gs, _ = c2
    n = 200_000
    ref = R.propagate(gs, cfg["source"], n, cfg["seed"])
    c3 = I.config(3)
    src = I.batch_source(c3["source"]["tracks"][:100], np.full(100, 1000))
    tune = R.tuning(256, 256, 4)
    ref_b = R.propagate_batch(gs, src, cfg["seed"], tune=tune)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        out = R.propagate(gs, cfg["source"], n, cfg["seed"], stream=side)
        out_b = R.propagate_batch(gs, src, cfg["seed"], tune=tune, stream=side)
    side.synchronize()
    for a, b in ((out, ref), (out_b, ref_b)):
        for k in ("fate", "pixel", "hit_xyz", "hit_time", "histogram", "fate_counts"):
            assert np.array_equal(to_np(a[k]), to_np(b[k]), equal_nan=True), k
    c4 = I.config(4)
    g4 = R.Scene(c4["scene"])
    tgt = np.zeros((c4["n_photons"], 2), np.float32)
    g_ref, l_ref = R.adjoint(g4, c4["source"], c4["seed"], targets=tgt)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        g_s, l_s = R.adjoint(g4, c4["source"], c4["seed"], targets=tgt, stream=side)
    side.synchronize()
    assert np.array_equal(to_np(g_s), to_np(g_ref)) and float(l_s) == float(l_ref)


def test_stack_overflow_is_flagged_not_faulted(R, orc):
    """64 parallel 20 mm squares stacked along z make a planar mesh whose BVH chains one square per
    group, about 21 BVH4 levels deep.  Listed far to near, every level puts three farther squares on
    the stack before descending towards the nearest: rays along the stack overflow the 32 entries.
    The overflow raises RICH_FLAG_STACK_OVERFLOW, the farthest entries are the ones dropped, and
    every photon still ends on the nearest square as in the oracle.  Listed near to far, the same
    squares leave the flag clear."""
    import copy
    z = 100.0 + 10.0 * np.arange(64)
    c, n = np.zeros(3), np.array([0.0, 0.0, -1.0])
    u, v = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    squares = [I.rect_mesh(c + np.array([0.0, 0.0, zk]), n, u, v, 10.0, 10.0, 1, 1) for zk in z]
    rng = np.random.default_rng(17)
    m = 256
    o = np.column_stack([rng.uniform(-5, 5, m), rng.uniform(-5, 5, m), np.zeros(m)])
    d = np.tile([0.0, 0.0, 1.0], (m, 1))
    src = I.explicit_source(o, d, np.full(m, 400.0))
    for far_first, flagged in ((True, True), (False, False)):
        sc = copy.deepcopy(I.scene_g2())
        sc["box"] = None
        tris = np.concatenate(squares[::-1] if far_first else squares)
        sc["meshes"] = [{"vertices": tris, "material": I.ABSORBER, "segment": -1}]
        gs = R.Scene(sc)
        assert gs.info()["max_depth"] >= 16
        out = R.propagate(gs, src, m, 5)
        flags = gs.status()
        assert bool(flags & R.FLAG_STACK_OVERFLOW) == flagged, (far_first, flags)
        assert (to_np(out["fate"]) == R.ABSORBED).all()
        compare(out, orc.propagate(sc, src, m, 5), label=f"stacked squares, far first {far_first}")
