"""rich_propagate_adjoint_noalloc (partial sums in the library's static device array) gives what
rich_propagate_adjoint gives, call after call, and refuses work whose partial sums do not fit."""

import numpy as np
import pytest

from paper_2309_12496_amd import inputs as I
from parity import to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2309_12496_amd import rich
    return rich


def _both(R, scene, src, n, seed, **kw):
    """The same adjoint through both entry points, the no-allocation one first."""
    import torch
    b, keep, nb = R.make_batch(src)
    assert n <= nb
    dev = lambda x, dt: None if x is None else torch.as_tensor(x, device="cuda", dtype=dt).contiguous()
    gu, tg = dev(kw.get("grad_uv"), torch.float32), dev(kw.get("targets"), torch.float32)
    mk = dev(kw.get("mask"), torch.uint8)
    rc = None if kw.get("cut") is None else torch.tensor([kw["cut"]], device="cuda", dtype=torch.float32)
    out = []
    for fn in (R.rich_propagate_adjoint_noalloc, R.rich_propagate_adjoint):
        grad = torch.full((scene.n_segments, 6), 7.0, device="cuda")
        loss = torch.full((1,), 7.0, device="cuda")
        print(f"{fn.__name__}: {n} photons, {scene.n_segments} segments", flush=True)
        fn(scene.handle, None, b, n, seed, 0, gu, tg, mk, rc, grad, loss)
        torch.cuda.synchronize()
        out.append((to_np(grad), to_np(loss)))
    assert scene.status() == 0
    return out


def test_noalloc_adjoint_matches_the_allocating_one(R):
    """Two calls in a row, the second on fewer photons (fewer blocks, so the array still holds
    rows of the first call beyond them): both equal rich_propagate_adjoint bit for bit."""
    cfg = I.config(4)
    gs = R.Scene(cfg["scene"])
    gs.set_params(cfg["target_params"])
    src, seed = cfg["source"], cfg["seed"]
    n1 = cfg["n_photons"]
    rng = np.random.default_rng(4242)
    targets = rng.normal(0.0, 200.0, size=(n1, 2)).astype(np.float32)
    mask = (rng.uniform(size=n1) < 0.9).astype(np.uint8)
    (g_na, l_na), (g_a, l_a) = _both(R, gs, src, n1, seed, targets=targets, mask=mask, cut=400.0)
    assert np.array_equal(g_na, g_a) and np.array_equal(l_na, l_a)
    assert np.count_nonzero(np.abs(g_a).sum(1)) >= 4 and l_a[0] > 0

    n2 = 60_000
    grad_uv = rng.normal(size=(n2, 2)).astype(np.float32)
    (g_na, l_na), (g_a, l_a) = _both(R, gs, src, n2, seed, grad_uv=grad_uv)
    assert np.array_equal(g_na, g_a)
    assert np.abs(g_a).sum() > 0


def test_noalloc_adjoint_refuses_what_does_not_fit(R):
    """2.5e9 photons with a mask need 7.3 MB of mask counts and offsets besides the partial sums of
    256 segments: beyond the 8 MiB array, so RICH_ERANGE and nothing launched (outputs untouched).
    The mask is all zeros and grad_uv one row: had anything run, it would read no photon's data.
    1e5 photons fit and match rich_propagate_adjoint."""
    import torch
    cells = I.grid_cells(16, 16)
    scene = I.scene_g1()
    scene["segments"] = I._segments_for_cells(cells)
    scene["params"] = I._nominal_params(len(cells))
    scene["caps"] = I._caps_for_cells(cells, list(range(len(cells))))
    gs = R.Scene(scene)
    s, keep = R.make_source(I.point_source())
    n = 2_500_000_000
    mask = torch.zeros(n, dtype=torch.uint8, device="cuda")
    gu = torch.zeros((1, 2), device="cuda")
    grad = torch.full((gs.n_segments, 6), 7.0, device="cuda")
    loss = torch.full((1,), 7.0, device="cuda")
    print(f"no-alloc refusal: {n} photons, {gs.n_segments} segments", flush=True)
    with pytest.raises(R.RichError) as e:
        R.rich_propagate_adjoint_noalloc(gs.handle, s, None, n, 1, 0, gu, None, mask, None, grad, loss)
    assert e.value.code == R.RICH_ERANGE
    torch.cuda.synchronize()
    assert bool((grad == 7.0).all()) and float(loss[0]) == 7.0
    del mask
    n = 100_000
    tg = torch.zeros((n, 2), device="cuda")
    for fn in (R.rich_propagate_adjoint_noalloc, R.rich_propagate_adjoint):
        fn(gs.handle, s, None, n, 1, 0, None, tg, None, None, grad, loss)
        torch.cuda.synchronize()
        if fn is R.rich_propagate_adjoint_noalloc:
            g0, l0 = to_np(grad).copy(), to_np(loss).copy()
    assert np.array_equal(g0, to_np(grad)) and np.array_equal(l0, to_np(loss))
    assert gs.status() == 0
