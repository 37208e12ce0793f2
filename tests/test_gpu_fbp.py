"""Filtered back-projection on the GPU (pwf_fbp) against the oracle.

FP32 ramp filtering (radix FFTs) and FP32 sums over the angles against FP64:
relative L2 1e-5 per slice.  Cases: the 64^3 ellipsoid phantom from its
analytic projections at 180 angles (every slice), an off-centre disk, and the
180 x 1024^2 workload's projections at full size (sampled slices).
"""

import math

import numpy as np
import pytest

import oracle as O
import synthetic as S
from gpu_helpers import device, rel, say, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5


def test_fbp_small_phantom_every_slice():
    from paper_2503_20146_amd import fbp
    dev = device()
    n, P = 64, 180
    geo = S.Geometry(ny=n, nx=n)
    phantom = S.ellipsoid_phantom(n, 12)
    angles = np.pi * np.arange(P) / P
    psis = [S.project_ellipsoids(phantom, th, n, n, geo.pixel_m, geo.wavelength_m) for th in angles]
    say("fbp 180 x 64^2")
    scale = geo.wavelength_m / (2 * math.pi * geo.pixel_m)
    vol = fbp([to_dev(p.astype(np.complex64), dev) for p in psis], angles, n, scale).cpu().numpy()
    ref = O.fbp_volume(psis, angles, n) * scale
    assert rel(vol, ref) <= TOL
    delta, beta = O.refractive_index(ref / scale, geo.wavelength_m, geo.pixel_m)
    assert np.allclose(vol.imag, delta, rtol=0, atol=TOL * np.abs(delta).max() * 10)


@pytest.mark.parametrize("nx,ny,P,n_out", [(128, 32, 90, 128), (64, 32, 37, 48)])
def test_fbp_off_centre_disk(nx, ny, P, n_out):
    """The second case: a partial chunk of angles and a side that is not a multiple of 32."""
    from paper_2503_20146_amd import fbp
    dev = device()
    angles = np.pi * np.arange(P) / P
    u = np.arange(nx) + 0.5 - nx / 2.0
    sino = np.array([2.0 * np.sqrt(np.maximum(20.0 ** 2 - (u - (25 * math.cos(th) + 10 * math.sin(th))) ** 2, 0))
                     for th in angles])
    psis = [np.repeat(sino[j][None, :], ny, axis=0).astype(np.complex64) * (1 + 0.5j) for j in range(P)]
    say(f"fbp off-centre disk {P} x {ny} x {nx} -> {n_out}^2")
    vol = fbp([to_dev(p, dev) for p in psis], angles, n_out).cpu().numpy()
    ref = O.fbp_slice(np.stack([p[0] for p in psis]).astype(np.complex128), angles, n_out)
    for y in sorted({0, ny // 2 + 1, ny - 1}):
        assert rel(vol[y], ref) <= TOL


def test_fbp_workload_180x1024_sampled_slices():
    from paper_2503_20146_amd import fbp
    import torch
    dev = device()
    say("fbp 180 x 1024^2: projections")
    d = S.tomo_projection_inputs(2, range(180))
    geo = d["geometry"]
    angles = np.pi * np.arange(180) / 180
    psis = [to_dev(p.astype(np.complex64), dev) for p in d["psi_true"]]
    say("fbp 180 x 1024^2: GPU")
    vol = fbp(psis, angles, 1024)
    torch.cuda.synchronize()
    for y in (100, 512, 900):
        say(f"fbp 180 x 1024^2: oracle slice {y}")
        ref = O.fbp_slice(np.stack([p[y] for p in d["psi_true"]]), angles, 1024)
        assert rel(vol[y].cpu().numpy(), ref) <= TOL, y
