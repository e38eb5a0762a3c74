"""Launches on one scene from several streams: each stream has its own device workspace (batch work
counters, fate-count slots, adjoint and ordering buffers, captured batch graph), so launches that
overlap on different streams give, bit for bit, what the same launches give one after another."""

import numpy as np
import pytest

from paper_2309_12496_amd import inputs as I
from parity import to_np

pytestmark = pytest.mark.gpu

KEYS = ("fate", "pixel", "hit_xyz", "hit_uv", "hit_time")


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2309_12496_amd import rich
    return rich


def same(a, b):
    a, b = to_np(a), to_np(b)
    return np.array_equal(a, b, equal_nan=a.dtype.kind == "f")


def side_streams(k):
    import torch
    cur = torch.cuda.current_stream()
    out = [torch.cuda.Stream() for _ in range(k)]
    for s in out:
        s.wait_stream(cur)   # inputs and zeroed outputs were made on the current stream
    return out


def test_forward_on_two_streams(R):
    """The headline scene's photons split in two id ranges traced on two streams at once, three
    times over: per-photon outputs equal one launch over all ids, and the fate counts and the
    histogram accumulate to three times its."""
    import torch
    cfg = I.config(2)
    sc = R.Scene(cfg["scene"])
    n, half, seed = 2_000_000, 1_000_000, cfg["seed"]
    ref = R.propagate(sc, cfg["source"], n, seed)
    s, keep = R.make_source(cfg["source"])
    ta, oa = R.alloc_outputs(sc, half)
    tb, ob = R.alloc_outputs(sc, n - half)
    a, b = side_streams(2)
    for _ in range(3):
        R.rich_propagate(sc.handle, s, half, seed, 0, oa, a)
        R.rich_propagate(sc.handle, s, n - half, seed, half, ob, b)
    torch.cuda.synchronize()
    for k in KEYS:
        assert same(ta[k], ref[k][:half]) and same(tb[k], ref[k][half:]), k
    assert same(ta["fate_counts"] + tb["fate_counts"], 3 * ref["fate_counts"])
    assert same(ta["histogram"] + tb["histogram"], 3 * ref["histogram"])
    assert sc.status() == 0


def test_batches_on_two_streams(R):
    """Two halves of the batched workload's tracks traced as two batches on two streams at once
    (each stream captures and replays its own graph) equal the same batches one after another."""
    import torch
    cfg = I.config(3)
    sc = R.Scene(cfg["scene"])
    tracks, offsets = cfg["source"]["tracks"], cfg["source"]["offsets"]
    counts = np.diff(np.asarray(offsets, np.int64))
    h = len(counts) // 2
    halves = [I.batch_source(tracks[:h], counts[:h]), I.batch_source(tracks[h:], counts[h:])]
    tune = R.tuning(256, 256, 4)
    refs = [R.propagate_batch(sc, src, cfg["seed"], tune=tune) for src in halves]
    torch.cuda.synchronize()
    made = [R.make_batch(src) for src in halves]
    outs = [R.alloc_outputs(sc, nb) for _, _, nb in made]
    streams = side_streams(2)
    for _ in range(2):   # the first launch on each stream captures its graph, the second replays it
        for (b, _, nb), (t, o), st in zip(made, outs, streams):
            R.rich_propagate_batch(sc.handle, b, nb, cfg["seed"], o, tune, st)
    torch.cuda.synchronize()
    for (t, _), ref in zip(outs, refs):
        for k in KEYS:
            assert same(t[k], ref[k]), k
        assert same(t["fate_counts"], 2 * ref["fate_counts"])
        assert same(t["histogram"], 2 * ref["histogram"])
    assert sc.status() == 0


def test_adjoints_on_two_streams(R):
    """Two fused-loss adjoints of the segmented mirror on two streams at once give bit for bit the
    gradient and loss of the same call on the current stream (each stream its own partial sums)."""
    import torch
    cfg = I.config(4)
    sc = R.Scene(cfg["scene"])
    n, seed = 200_000, cfg["seed"]
    src = I.batch_source(cfg["source"]["tracks"][:200], np.full(200, 1000))
    fwd = R.propagate_batch(sc, src, seed, tune=R.tuning(256, 256, 4))
    mask = ((fwd["fate"] == R.DETECTED) | (fwd["fate"] == R.QE_REJECTED)).to(torch.uint8)
    targets = torch.nan_to_num(fwd["hit_uv"]) + 0.5
    g0, l0 = R.adjoint(sc, src, seed, targets=targets, mask=mask)
    assert int(mask.sum()) > 1000 and float(l0) > 0
    b, keep, nb = R.make_batch(src)
    assert nb == n
    grads = [torch.zeros_like(g0) for _ in range(2)]
    losses = [torch.zeros_like(l0) for _ in range(2)]
    streams = side_streams(2)
    for _ in range(2):
        for g, l, st in zip(grads, losses, streams):
            R.rich_propagate_adjoint(sc.handle, None, b, nb, seed, 0, None, targets, mask, None, g, l, st)
    torch.cuda.synchronize()
    for g, l in zip(grads, losses):
        assert same(g, g0) and same(l, l0)
    assert sc.status() == 0


def test_stream_slots_run_out_with_an_error(R):
    """A scene serves 64 launch streams; a launch from a 65th is refused with RICH_ESTATE, and the
    streams that hold slots keep working.  (torch hands out streams from a pool of 32, so the 65
    distinct streams are made with the HIP runtime.)"""
    import ctypes
    import torch
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipStreamCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    hip.hipStreamDestroy.argtypes = [ctypes.c_void_p]
    hip.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
    cfg = I.config(1)
    sc = R.Scene(cfg["scene"])
    s, keep = R.make_source(cfg["source"])
    t, o = R.alloc_outputs(sc, 64)
    torch.cuda.synchronize()
    streams = []
    try:
        for _ in range(65):
            h = ctypes.c_void_p()
            assert hip.hipStreamCreate(ctypes.byref(h)) == 0
            streams.append(h.value)
        assert len(set(streams)) == 65
        for st in streams[:64]:
            R.rich_propagate(sc.handle, s, 64, cfg["seed"], 0, o, st)
        with pytest.raises(R.RichError) as e:
            R.rich_propagate(sc.handle, s, 64, cfg["seed"], 0, o, streams[64])
        assert e.value.code == R.RICH_ESTATE
        R.rich_propagate(sc.handle, s, 64, cfg["seed"], 0, o, streams[0])
        for st in streams:
            assert hip.hipStreamSynchronize(st) == 0
    finally:
        for st in streams:
            hip.hipStreamDestroy(st)
    assert int(t["fate_counts"].sum()) == 65 * 64
    assert sc.status() == 0
