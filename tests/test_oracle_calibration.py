"""Pins of the oracle's calibration front end (Methods, Eq. 3 and the IPSF /
IOTF of Eqs. 4-5; Results, "Diffuser transmission function"):

* fully developed speckle of a complex Gaussian field with a known Gaussian
  correlation obeys the Siegert relation, so the fit returns that field's
  coherence length (statistical error only);
* the autocorrelation against a brute-force double loop on a tiny image;
* exact Wiener inversion (eps = 0, IOTF without zeros) and its limits;
* a zero-phase diffuser is recovered exactly from its noise-free, unblurred
  reference speckle.
"""

import dataclasses
import math

import numpy as np

import oracle as O
import synthetic as S


def _gaussian_speckle(n, x_c, y_c, seed=0):
    """|E|^2 for E complex Gaussian with correlation exp(-pi d^2 / (2 c^2)) per axis (px)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    u = np.fft.fftfreq(n)[None, :]
    v = np.fft.fftfreq(n)[:, None]
    # amplitude filter whose power spectrum is the transform of exp(-pi d^2 / (2 c^2))
    h = np.exp(-math.pi * (u * x_c) ** 2) * np.exp(-math.pi * (v * y_c) ** 2)
    return np.abs(np.fft.ifft2(np.fft.fft2(w) * h)) ** 2


def test_siegert_fit_recovers_the_coherence_length():
    for x_c, y_c in ((3.0, 5.0), (4.5, 2.5)):
        I = _gaussian_speckle(1024, x_c, y_c)
        gx, gy = O.speckle_g2(I, 24)
        assert abs(gx[0] - 2.0) < 0.06 and abs(gy[0] - 2.0) < 0.06   # contrast 1: <I^2> = 2 <I>^2 (sampling error ~2%)
        xc, cx = O.fit_coherence_length(gx, 1.0)
        yc, cy = O.fit_coherence_length(gy, 1.0)
        assert abs(xc / x_c - 1) < 0.05 and abs(yc / y_c - 1) < 0.05, (xc, yc)   # sampling error ~2%
        assert abs(cx - 1) < 0.07 and abs(cy - 1) < 0.07


def test_g2_matches_brute_force():
    rng = np.random.default_rng(1)
    I = rng.random((6, 7)) + 0.5
    gx, gy = O.speckle_g2(I, 3)
    m2 = I.mean() ** 2
    for d in range(4):
        sx = sum(I[y, x] * I[y, (x + d) % 7] for y in range(6) for x in range(7)) / 42 / m2
        sy = sum(I[y, x] * I[(y + d) % 6, x] for y in range(6) for x in range(7)) / 42 / m2
        assert abs(gx[d] - sx) < 1e-12 and abs(gy[d] - sy) < 1e-12


def test_fit_is_exact_on_a_model_curve_with_contrast():
    d = np.arange(40, dtype=np.float64)
    g2 = 1.0 + 0.37 * np.exp(-math.pi * (d * 0.65e-6) ** 2 / (4.1e-6) ** 2)
    g2[0] += 0.8   # the noise spike at zero shift is not fitted
    xc, c = O.fit_coherence_length(g2, 0.65e-6)
    assert abs(xc / 4.1e-6 - 1) < 1e-12 and abs(c - 0.37) < 1e-12


def test_wiener_exact_inverse_and_limits():
    inp = S.instance_inputs(0)
    prob = O.make_problem(inp["t"], inp["geometry"])
    rng = np.random.default_rng(2)
    I = rng.random(prob.shape) + 1.0
    blurred = np.real(O.filter_(I, prob.iotf))
    assert np.max(np.abs(O.wiener_deconvolve(blurred, prob.iotf, 0.0) - I)) < 1e-9 * np.max(I)
    ones = np.ones_like(prob.iotf)
    assert np.max(np.abs(O.wiener_deconvolve(I, ones, 0.0) - I)) < 1e-12 * np.max(I)
    # large eps: the filter tends to IOTF / eps
    big = O.wiener_deconvolve(I, prob.iotf, 1e6)
    assert np.max(np.abs(big * 1e6 - np.real(O.filter_(I, prob.iotf)))) < 1e-5 * np.max(I)


def test_zero_phase_diffuser_recovered_from_its_reference():
    inp = S.instance_inputs(0)
    geo = dataclasses.replace(inp["geometry"], sigma_x_px=0.0, sigma_y_px=0.0)
    prob = O.make_problem(inp["t"], geo)
    rng = np.random.default_rng(4)
    a = 1.0 + 0.2 * np.real(O.filter_(rng.standard_normal(prob.shape), np.exp(-(prob.u ** 2 + prob.v ** 2) * 1e-9)))
    assert a.min() > 0
    t_true = O.free_propagation(a, prob, -prob.z2_m)
    ref = np.abs(O.free_propagation(t_true, prob, prob.z2_m)) ** 2
    t = O.diffuser_from_reference(ref, dataclasses.replace(prob, t=t_true), 0.0)
    assert np.max(np.abs(t - t_true)) < 1e-10
