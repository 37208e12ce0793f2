"""Pins of the oracle's quadratic background removal (Methods, "Reconstruction
procedure": a two-dimensional quadratic fitted to the background area of each
slice after tomography).  A surface built from known coefficients must come
back exactly, whatever sits inside the sample cylinder; the fit must ignore
everything inside it; and too small a background must be refused."""

import math

import numpy as np
import pytest

import oracle as O


def _surface(coef_re, coef_im, n):
    c = (np.arange(n) + 0.5 - n / 2.0) / (n / 2.0)
    x, z = c[None, :], c[:, None]
    mono = [np.ones((n, n)), x + 0 * z, z + 0 * x, x * x + 0 * z, x * z, z * z + 0 * x]
    return sum(a * m for a, m in zip(coef_re, mono)) + 1j * sum(b * m for b, m in zip(coef_im, mono))


def test_known_surface_is_recovered():
    rng = np.random.default_rng(5)
    n, r_bg = 48, 18.0
    coefs = rng.standard_normal((3, 2, 6))
    vol = np.stack([_surface(c[0], c[1], n) for c in coefs])
    out, coef = O.background_quadratic(vol, r_bg)
    assert np.max(np.abs(coef - coefs)) < 1e-10
    assert np.max(np.abs(out)) < 1e-10


def test_sample_inside_the_cylinder_is_untouched():
    """Disks inside r_bg on top of a quadratic background: the result is the disks alone."""
    rng = np.random.default_rng(6)
    n, r_bg = 64, 24.0
    c = np.arange(n) + 0.5 - n / 2.0
    rr = np.hypot(c[None, :] - 3.0, c[:, None] + 2.0)
    sample = np.where(rr < 14.0, 0.3 - 0.1j, 0.0) + np.where(np.hypot(c[None, :] + 6, c[:, None] - 5) < 6, 1.0j, 0.0)
    assert np.all(sample[O.background_mask(n, r_bg)] == 0)   # the fixture's sample is inside the cylinder
    bg = _surface(rng.standard_normal(6), rng.standard_normal(6), n)
    out, _ = O.background_quadratic((sample + bg)[None], r_bg)
    assert np.max(np.abs(out[0] - sample)) < 1e-10


def test_background_area_is_the_outside_of_the_cylinder():
    n, r = 32, 10.0
    m = O.background_mask(n, r)
    c = np.arange(n) + 0.5 - n / 2.0
    for iz in range(n):
        for ix in range(n):
            assert m[iz, ix] == (math.hypot(c[ix], c[iz]) >= r)


def test_fit_uses_only_the_background():
    """Changing voxels inside r_bg changes nothing of the fitted coefficients."""
    rng = np.random.default_rng(7)
    n, r_bg = 40, 15.0
    vol = rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))
    _, c1 = O.background_quadratic(vol, r_bg)
    inside = ~O.background_mask(n, r_bg)
    vol2 = vol.copy()
    vol2[0][inside] += 5.0 + 2.0j
    _, c2 = O.background_quadratic(vol2, r_bg)
    assert np.max(np.abs(c1 - c2)) < 1e-12
    # and the residual over the background is orthogonal to every monomial
    out, _ = O.background_quadratic(vol, r_bg)
    basis = O.background_basis(n)[:, ~inside]
    assert np.max(np.abs(basis @ out[0][~inside])) < 1e-9


def test_too_small_background_is_refused():
    with pytest.raises(ValueError):
        O.background_quadratic(np.zeros((1, 16, 16)), 16.0 * math.sqrt(2.0))
