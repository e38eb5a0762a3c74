"""Pins of the oracle's film read-out emulation (Section 4.4: camera, film, intensity threshold).

A detected photon is projected by a pinhole camera onto the film and splatted
with a Gaussian reconstruction filter; pixels at or above the threshold are
hits.  The pins place single photons at known film positions and check the
closed-form Gaussian weights, the leak of one photon into several hit pixels,
the field-of-view scale, and that undetected photons leave no trace.
"""

import math

import numpy as np
import pytest

FILM = {"width": 64, "height": 48, "distance": 478.69, "fov": math.radians(116.38), "sigma": 0.5, "threshold": 45.0}


def _uv_of(film, x, y):
    """Detector (u, v) whose image falls at film coordinates (x, y) (pinhole camera on the normal)."""
    f = 0.5 * film["width"] / math.tan(0.5 * film["fov"])
    return ((x - 0.5 * film["width"]) * film["distance"] / f, (y - 0.5 * film["height"]) * film["distance"] / f)


def test_photon_at_a_pixel_centre(orc):
    u, v = _uv_of(FILM, 20.5, 10.5)
    img, hits = orc.film_readout(FILM, [0], [[u, v]])
    assert img[10, 20] == pytest.approx(255.0, abs=1e-9)
    for dj, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        assert img[10 + dj, 20 + di] == pytest.approx(255.0 * math.exp(-2.0), abs=1e-9)
    assert img[11, 21] == pytest.approx(255.0 * math.exp(-4.0), abs=1e-9)
    assert img[10, 22] == pytest.approx(255.0 * math.exp(-8.0), abs=1e-9)     # window edge: 4 sigma = 2 px
    assert img[10, 23] == 0.0
    # the discrete Gaussian over the 5 x 5 window
    g = sum(math.exp(-k * k / 0.5) for k in range(-2, 3))
    assert img.sum() == pytest.approx(255.0 * g * g, rel=1e-12)
    assert hits.sum() == 1 and hits[10, 20] == 1


def test_photon_at_a_pixel_corner_leaks_into_four_hits(orc):
    u, v = _uv_of(FILM, 30.0, 20.0)
    img, hits = orc.film_readout(FILM, [0], [[u, v]])
    for j in (19, 20):
        for i in (29, 30):
            assert img[j, i] == pytest.approx(255.0 * math.exp(-1.0), abs=1e-9)
            assert hits[j, i] == 1
    assert hits.sum() == 4


def test_field_of_view_scale_and_undetected_photons(orc):
    """A hit at u = distance tan(fov/2) lands on the film's right edge; other fates are ignored."""
    u = FILM["distance"] * math.tan(0.5 * FILM["fov"])
    img, _ = orc.film_readout(FILM, [0, 1, 3], [[u, 0.0], [0.0, 0.0], [0.0, 0.0]])
    assert img[23, 63] == pytest.approx(255.0 * math.exp(-1.0), abs=1e-9)    # x = 64, y = 24: centres 0.5 away
    assert img[:, :60].sum() == 0.0
    # accumulation over calls
    img2, _ = orc.film_readout(FILM, [0], [[u, 0.0]], image=img)
    assert img2[23, 63] == pytest.approx(2 * 255.0 * math.exp(-1.0), abs=1e-9)
