"""The half-form x-spectra of the intensity path, modelled in numpy.

The sweeps keep the x-spectra of real rows (intensity, residual, measured
speckle) in half form: kx = 1 .. nx/2 - 1 at position kx, and the two real
values at kx = 0 and nx/2 packed into position 0, the latter scaled by the
IOTF's x factor at nx/2 (Eq. 5's Gaussian window is separable and even).  The
column transform then carries the two real columns as real and imaginary
parts; the residual path applies the IOTF twice, so the back-blur rebuild
multiplies the kx = nx/2 value by the x factor once more, and the loss counts
columns s > 0 twice (they stand for kx and -kx).  This model follows those
steps and must reproduce the plain 2-D definitions: Filter(I, IOTF), the
residual's Parseval sum and Filter(-e, IOTF) of the residual (Eq. 2).
"""

import numpy as np
import pytest


def _windows(ny, nx, sigma, rng):
    fx, fy = np.fft.fftfreq(nx), np.fft.fftfreq(ny)
    ix = np.exp(-2.0 * np.pi ** 2 * sigma ** 2 * fx ** 2)
    iy = np.exp(-2.0 * np.pi ** 2 * sigma ** 2 * fy ** 2)
    intensity = rng.uniform(0.5, 1.5, (ny, nx))
    y = intensity + 0.05 * rng.standard_normal((ny, nx))
    return ix, iy, intensity, y


def _half_rows(a, scale_nyq):
    """Half form of the x-spectra of the real rows of ``a``."""
    nx = a.shape[1]
    x = np.fft.fft(a, axis=1)
    h = x[:, : nx // 2].copy()
    h[:, 0] = x[:, 0].real + 1j * scale_nyq * x[:, nx // 2].real
    return h


def _full_rows(h, scale_nyq):
    """Full x-spectra rebuilt from the half form (Hermitian rows)."""
    ny, half = h.shape
    nx = 2 * half
    x = np.zeros((ny, nx), complex)
    x[:, 1:half] = h[:, 1:]
    x[:, half + 1:] = np.conj(h[:, 1:][:, ::-1])
    x[:, 0] = h[:, 0].real
    x[:, half] = scale_nyq * h[:, 0].imag
    return x


@pytest.mark.parametrize("ny,nx,sigma", [(16, 32, 1.5), (32, 8, 0.7), (64, 64, 2.0)])
def test_residual_path_matches_2d_definitions(ny, nx, sigma):
    rng = np.random.default_rng(ny * 1000 + nx)
    ix, iy, intensity, y = _windows(ny, nx, sigma, rng)
    iotf = iy[:, None] * ix[None, :]
    # plain definitions
    r_full = iotf * np.fft.fft2(intensity) - np.fft.fft2(y)        # = -F{e}, e = y - f
    loss_ref = np.sum(np.abs(r_full) ** 2)
    back_ref = np.real(np.fft.ifft2(iotf * r_full))
    # half form: S4 / setup rows, S5 columns, S6 rebuild
    hx = np.where(np.arange(nx // 2) == 0, 1.0, ix[: nx // 2])    # x factor per column (packed: 1)
    w = np.where(np.arange(nx // 2) == 0, 1.0, 2.0)
    z = np.fft.fft(_half_rows(intensity, ix[nx // 2]), axis=0)
    zy = np.fft.fft(_half_rows(y, 1.0), axis=0)
    h = iy[:, None] * hx[None, :]
    rr = h * z - zy
    loss = np.sum(w[None, :] * np.abs(rr) ** 2)
    back = np.real(np.fft.ifft(_full_rows(np.fft.ifft(h * rr, axis=0), ix[nx // 2]), axis=1))
    assert abs(loss - loss_ref) <= 1e-12 * loss_ref
    assert np.max(np.abs(back - back_ref)) <= 1e-12 * np.max(np.abs(back_ref))


def test_forward_blur_matches_2d_filter():
    rng = np.random.default_rng(7)
    ny, nx = 32, 64
    ix, iy, intensity, _ = _windows(ny, nx, 1.2, rng)
    f_ref = np.real(np.fft.ifft2(iy[:, None] * ix[None, :] * np.fft.fft2(intensity)))
    hx = np.where(np.arange(nx // 2) == 0, 1.0, ix[: nx // 2])
    z = np.fft.fft(_half_rows(intensity, ix[nx // 2]), axis=0) * iy[:, None] * hx[None, :]
    f = np.real(np.fft.ifft(_full_rows(np.fft.ifft(z, axis=0), 1.0), axis=1))
    assert np.max(np.abs(f - f_ref)) <= 1e-12 * np.max(np.abs(f_ref))


def test_packed_column_keeps_the_two_residuals_apart():
    """|R_A + i R_B|^2 summed over ky is |R_A|^2 + |R_B|^2 for Hermitian R_A, R_B;
    dropping the Hermitian structure (complex rows) breaks it, so the model
    above depends on real rows."""
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal(32), rng.standard_normal(32)
    ra, rb = np.fft.fft(a), np.fft.fft(b)
    assert np.isclose(np.sum(np.abs(ra + 1j * rb) ** 2), np.sum(np.abs(ra) ** 2) + np.sum(np.abs(rb) ** 2))
    c = a + 1j * rng.standard_normal(32)
    rc = np.fft.fft(c)
    assert not np.isclose(np.sum(np.abs(rc + 1j * rb) ** 2), np.sum(np.abs(rc) ** 2) + np.sum(np.abs(rb) ** 2))
