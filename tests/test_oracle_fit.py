"""Pins of the oracle's FP64 Adam (the alignment fit's optimiser) against closed forms."""

import numpy as np


def _run(orc, grads, losses, n_steps=40, lr=0.3, lr_final=1e-4, free=(True, True, True, False, False, False),
         scale=(1e-3, 1e-3, 10.0, 1.0, 1.0, 1.0), eps=1e-12, **kw):
    p0 = np.arange(12, dtype=np.float64).reshape(2, 6)
    return p0, orc.adam_fit_steps(p0, grads, losses, n_steps, lr, lr_final, scale, free, eps=eps, **kw)


def test_constant_gradient_moves_by_the_summed_step_sizes(orc):
    """With a constant gradient the bias-corrected moments are exactly g and g^2, so every step
    moves z by size_t * g / (|g| + eps); over the whole cosine schedule the sizes sum to
    n lr_final + (lr - lr_final)(n + 1)/2 (the cosines sum to 1)."""
    rng = np.random.default_rng(3)
    G = rng.normal(size=(2, 6)) * 10.0 ** rng.uniform(-3, 3, size=(2, 6))
    n, lr, lrf = 40, 0.3, 1e-4
    sc = np.array([1e-3, 1e-3, 10.0, 1.0, 1.0, 1.0])
    p0, r = _run(orc, [G] * n, [1.0] * n, n_steps=n, lr=lr, lr_final=lrf)
    g = G * sc
    total = n * lrf + (lr - lrf) * (n + 1) / 2
    want = -total * g / (np.abs(g) + 1e-12)
    free = np.array([True, True, True, False, False, False])
    np.testing.assert_allclose(r["z"][-1][:, free], want[:, free], rtol=1e-12)
    assert not r["z"][:, :, ~free].any()                                   # fixed columns never move
    np.testing.assert_array_equal(r["params"][-1][:, ~free], p0[:, ~free])
    np.testing.assert_allclose(r["params"][-1], p0 + r["z"][-1] * sc, rtol=1e-15)
    # first step: exactly lr against the gradient's sign
    np.testing.assert_allclose(r["z"][0][:, free], -lr * np.sign(g[:, free]) * np.abs(g[:, free])
                               / (np.abs(g[:, free]) + 1e-12), rtol=1e-12)


def test_second_step_uses_bias_corrected_weighted_averages(orc):
    """After gradients g1, g2 the corrected moments are the weighted averages
    (beta g1 + g2) / (1 + beta) and (beta2 g1^2 + g2^2) / (1 + beta2)."""
    b1, b2, n, lr, lrf = 0.9, 0.999, 10, 0.2, 0.01
    g1 = np.full((2, 6), 2.0)
    g2 = np.full((2, 6), -0.5)
    _, r = _run(orc, [g1, g2], [1.0, 1.0], n_steps=n, lr=lr, lr_final=lrf, free=(True,) * 6,
                scale=(1.0,) * 6, eps=1e-9)
    size2 = lrf + 0.5 * (lr - lrf) * (1 + np.cos(np.pi / n))
    mh = (b1 * g1 + g2) / (1 + b1)
    vh = (b2 * g1 ** 2 + g2 ** 2) / (1 + b2)
    want = -lr * g1 / (np.abs(g1) + 1e-9) - size2 * mh / (np.sqrt(vh) + 1e-9)
    np.testing.assert_allclose(r["z"][1], want, rtol=1e-12)


def test_residual_cut_follows_the_loss(orc):
    """cut = k sqrt(L) + floor after a step with loss L; +inf after a step that counted no photon."""
    G = np.ones((2, 6))
    _, r = _run(orc, [G, G, G], [4.0, 0.0, 0.25], outlier_cut=5.0, cut_floor=1e-3)
    assert r["cut"][0] == 5.0 * 2.0 + 1e-3
    assert np.isinf(r["cut"][1])
    assert r["cut"][2] == 5.0 * 0.5 + 1e-3
