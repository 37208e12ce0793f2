"""Pins of the oracle's filtered back-projection (Methods, "Reconstruction
procedure"): the ramp kernel against the inverse transform of |f| by
quadrature, its frequency response, analytic disk projections (centred and
off centre, which fixes the sign conventions of the geometry), and a slice of
the ellipsoid phantom against its voxelised refractive index."""

import math

import numpy as np
from scipy import integrate

import oracle as O
import synthetic as S


def test_ramp_kernel_is_the_band_limited_ramp():
    h = O.ramp_kernel(256)
    for n in range(6):
        ref, _ = integrate.quad(lambda f: 2.0 * f * math.cos(2.0 * math.pi * f * n), 0.0, 0.5, limit=200)
        assert abs(h[n] - ref) < 1e-10, n
        assert h[-n] == h[n]


def test_ramp_frequency_response():
    n_pad = 256
    H = np.real(np.fft.fft(O.ramp_kernel(n_pad)))
    f = np.abs(np.fft.fftfreq(n_pad))
    assert np.max(np.abs(H - f)) < 2.0 / (math.pi ** 2 * n_pad / 2)   # truncation of the odd tail


def _disk_sinogram(nx, angles, radius, cx, cz):
    u = np.arange(nx) + 0.5 - nx / 2.0
    rows = []
    for th in angles:
        uc = cx * math.cos(th) - cz * math.sin(th)
        d2 = radius ** 2 - (u - uc) ** 2
        rows.append(2.0 * np.sqrt(np.maximum(d2, 0.0)))
    return np.array(rows)


def test_disk_reconstruction_centred_and_off_centre():
    nx, n_out, P = 96, 96, 360
    angles = np.pi * np.arange(P) / P
    c = np.arange(n_out) + 0.5 - n_out / 2.0
    X, Z = c[None, :], c[:, None]
    for cx, cz in ((0.0, 0.0), (14.0, -9.0)):
        img = np.real(O.fbp_slice(_disk_sinogram(nx, angles, 18.0, cx, cz), angles, n_out))
        r = np.sqrt((X - cx) ** 2 + (Z - cz) ** 2)
        assert abs(img[r < 14].mean() - 1.0) < 0.01, (cx, cz, img[r < 14].mean())
        assert abs(img[(r > 22) & (np.abs(X) < 40) & (np.abs(Z) < 40)].mean()) < 0.01
        mirror = np.sqrt((X + cx) ** 2 + (Z - cz) ** 2) < 14
        if cx != 0.0:
            assert img[mirror & (r > 22)].mean() < 0.05     # not reconstructed at the mirrored place


def test_ellipsoid_slice_matches_voxelised_index():
    n, P = 64, 180
    geo = S.Geometry(ny=n, nx=n)
    phantom = S.ellipsoid_phantom(n, 12)
    angles = np.pi * np.arange(P) / P
    row = n // 2
    sino = np.stack([S.project_ellipsoids(phantom, th, n, n, geo.pixel_m, geo.wavelength_m)[row] for th in angles])
    vol = O.fbp_slice(sino, angles, n)
    delta, beta = O.refractive_index(vol, geo.wavelength_m, geo.pixel_m)
    # voxelised phantom at voxel centres of the slice (y = row centre)
    c = np.arange(n) + 0.5 - n / 2.0
    y = row + 0.5 - n / 2.0
    ref = np.zeros((n, n))
    for e in phantom:
        a_mat = e["rot"] @ np.diag(1.0 / e["axes"] ** 2) @ e["rot"].T
        r = np.stack(np.broadcast_arrays(c[None, :], y, c[:, None]), axis=-1) - e["centre"]
        inside = np.einsum("...i,ij,...j->...", r, a_mat, r) <= 1.0
        ref += inside * e["delta"]
    assert ref.max() > 0
    corr = np.corrcoef(delta.ravel(), ref.ravel())[0, 1]
    assert corr > 0.9, corr
    assert abs(np.sum(delta) / np.sum(ref) - 1.0) < 0.05
    assert np.allclose(beta * 100.0, delta, atol=0.05 * ref.max())    # beta = delta / 100 in the phantom
