"""Pins of the oracle's diagnostics (Methods): the RMSE image at the truth
equals the Poisson noise level, and the shell correlation of Eq. 16 obeys its
closed forms: 1 for identical volumes, -1 for opposite ones, about 0 for
independent noise, and SNR / (1 + SNR) for signal plus independent noise of
known power (Eq. 18, which gives the paper's 1/4 criterion)."""

import math

import numpy as np

import oracle as O
import synthetic as S


def test_rmse_image_at_truth_is_the_noise_level():
    inp = S.instance_inputs(0)
    prob = O.make_problem(inp["t"], inp["geometry"])
    f, _, _ = O.physical_model(inp["psi_true"], prob)
    y = S.poisson_intensity(f, inp["seed_key"])
    img = O.rmse_image(y, inp["psi_true"], prob, 1.0)
    # E|y - f| = sqrt(2 / pi) sqrt(f / N) for Poisson counts at N = 1e4 photons per unit intensity
    expect = 100.0 * math.sqrt(2.0 / math.pi) * np.mean(np.sqrt(f / 1e4))
    assert abs(img.mean() / expect - 1.0) < 0.03
    assert np.max(O.rmse_image(f, inp["psi_true"], prob, 1.0)) < 1e-9


def test_shell_correlation_closed_forms():
    rng = np.random.default_rng(0)
    g = rng.standard_normal((32, 32, 32))
    assert np.allclose(O.shell_correlation(g, g)[1:], 1.0)
    assert np.allclose(O.shell_correlation(g, -g)[1:], -1.0)
    h = rng.standard_normal((32, 32, 32))
    fsc = O.shell_correlation(g, h)
    counts = np.bincount(np.rint(np.sqrt(sum(a * a for a in np.meshgrid(*([np.fft.fftfreq(32) * 32] * 3),
                                                                          indexing="ij")))).astype(int).ravel())
    assert np.all(np.abs(fsc[2:]) < 5.0 / np.sqrt(counts[2:17]))


def test_shell_correlation_of_signal_plus_noise():
    rng = np.random.default_rng(1)
    n = 48
    s = rng.standard_normal((n, n, n))
    for snr in (3.0, 1.0 / 3.0):
        sig = math.sqrt(1.0 / snr)
        g1 = s + sig * rng.standard_normal((n, n, n))
        g2 = s + sig * rng.standard_normal((n, n, n))
        fsc = O.shell_correlation(g1, g2)
        assert abs(np.mean(fsc[8:24]) - snr / (1.0 + snr)) < 0.02, snr
    # FSC = 1/4 at SNR = 1/3: the 1/4 criterion is the shell where the signal
    # still correlates 1/2 with the data (Eq. 17)
    assert abs((1 / 3) / (1 + 1 / 3) - 0.25) < 1e-15


def test_frc_2d_and_resolution():
    rng = np.random.default_rng(2)
    n = 128
    # signal whose power falls off so that the FRC crosses 1/4 inside the band
    k = np.fft.fftfreq(n) * n
    r = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    s = np.real(np.fft.ifft2(np.fft.fft2(rng.standard_normal((n, n))) * np.exp(-r / 10.0)))
    noise = 0.05
    frc = O.shell_correlation(s + noise * rng.standard_normal((n, n)), s + noise * rng.standard_normal((n, n)))
    res = O.resolution_from_fsc(frc, n, 1e-6)
    kappa = n * 1e-6 / res
    assert frc[int(kappa)] < 0.25 <= frc[int(kappa) - 1]


def test_resolution_without_crossing_is_nyquist():
    assert O.resolution_from_fsc(np.ones(65), 128, 1e-6) == 2e-6
