"""Seeded generators for the five PWF workloads.

Recipe (shared by tests, bench and the oracle leg of the bench):

* Single-projection workloads (128^2 and 1024^2): a phase object made from
  N(0,1) white noise, low-passed with a periodic Gaussian of ``sigma_phi`` px,
  min-max scaled to ``[0, phi_max]`` rad; absorption ``mu = 0.05 * phi``;
  complex phase ``psi_true = -mu + i*phi``.  The diffuser has a per-pixel
  phase drawn from U[0, pi], smoothed by a periodic Gaussian of 1 px (no
  rescaling afterwards), and an i.i.d. amplitude drawn from U[0.9, 1].
* Tomographic workloads: 40 random ellipsoids in an ``n^3`` voxel frame
  (voxel = pixel), semi-axes U[n/32, n/8] voxels, uniformly random
  orientation, bounding sphere inside the cylinder of radius 0.45 n about the
  vertical axis and inside rows [0.05 n, 0.95 n]; decrement delta ~
  U[1e-7, 5e-7] and beta = delta / 100.  Projections at equally spaced
  angles over [0, 180) deg use closed-form chord lengths at pixel centres:
  ``phi = (2 pi / lambda) sum delta * chord``, ``mu`` likewise with beta.
* Poisson noise: ``y = Poisson(n_ph * f) / n_ph`` with ``n_ph = 1e4``
  photons per pixel of unit flat field.

Every draw comes from NumPy's PCG64 seeded from ``BASE_SEED + workload`` (and
an instance index where a workload has several independent instances), in a
fixed order: white noise, diffuser phase, diffuser amplitude, phantom.
Poisson noise uses its own stream so that the noise-free speckle can be made
by either side before it is drawn.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 20250326
PHOTONS_PER_PIXEL = 1.0e4


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Imaging geometry of one projection (SI units)."""

    ny: int
    nx: int
    pixel_m: float = 1.0e-6
    wavelength_m: float = 0.05e-9
    z1_m: float = 5.0e-3      # sample -> diffuser
    z2_m: float = 200.0e-3    # diffuser -> detector
    sigma_x_px: float = 1.0   # Gaussian source blur at the detector, in px
    sigma_y_px: float = 1.0


def config_geometry(workload: int, n: int | None = None, sigma_px: float | None = None) -> Geometry:
    """Geometry of workload 0..4 (grid side ``n`` overrides the default)."""
    default_n = {0: 128, 1: 1024, 2: 1024, 3: 512, 4: 2048}[workload]
    default_sigma = 1.0 if workload in (0, 3) else 1.5
    n = default_n if n is None else n
    s = default_sigma if sigma_px is None else sigma_px
    return Geometry(ny=n, nx=n, sigma_x_px=s, sigma_y_px=s)


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _periodic_gaussian_lowpass(a: np.ndarray, sigma_px: float) -> np.ndarray:
    """Circular convolution with a unit-sum Gaussian of ``sigma_px`` pixels."""
    ny, nx = a.shape
    fy = np.fft.fftfreq(ny)[:, None]
    fx = np.fft.fftfreq(nx)[None, :]
    w = np.exp(-2.0 * math.pi ** 2 * sigma_px ** 2 * (fx ** 2 + fy ** 2))
    return np.real(np.fft.ifft2(np.fft.fft2(a) * w))


def phase_object(rng: np.random.Generator, ny: int, nx: int, sigma_px: float,
                 phi_max: float, mu_over_phi: float = 0.05) -> np.ndarray:
    """Complex phase ``psi = -mu + i phi`` of a smooth random sample (complex128)."""
    noise = rng.standard_normal((ny, nx))
    s = _periodic_gaussian_lowpass(noise, sigma_px)
    phi = phi_max * (s - s.min()) / (s.max() - s.min())
    mu = mu_over_phi * phi
    return -mu + 1j * phi


def diffuser(rng: np.random.Generator, ny: int, nx: int, smooth_px: float = 1.0,
             amp_lo: float = 0.9, amp_hi: float = 1.0) -> np.ndarray:
    """Diffuser transmission ``t`` (complex64)."""
    theta = rng.uniform(0.0, math.pi, size=(ny, nx))
    theta = _periodic_gaussian_lowpass(theta, smooth_px)
    amp = rng.uniform(amp_lo, amp_hi, size=(ny, nx))
    return (amp * np.exp(1j * theta)).astype(np.complex64)


def poisson_intensity(f: np.ndarray, seed_key: tuple[int, ...],
                      photons: float = PHOTONS_PER_PIXEL) -> np.ndarray:
    """Flat-field-normalised Poisson counts ``Poisson(photons * f) / photons`` (float32)."""
    rng = _rng(*seed_key, 0xB015)
    lam = np.clip(np.asarray(f, dtype=np.float64), 0.0, None) * photons
    return (rng.poisson(lam) / photons).astype(np.float32)


def instance_inputs(workload: int, n: int | None = None, instance: int | None = None,
                    sigma_px: float | None = None) -> dict:
    """Inputs of one single-projection instance (workloads 0, 1 and the ROIs of 3).

    Returns ``psi_true`` (complex128), ``t`` (complex64), the ``geometry`` and
    the ``seed_key`` to pass to :func:`poisson_intensity`.
    """
    key = (BASE_SEED + workload,) if instance is None else (BASE_SEED + workload, instance)
    geo = config_geometry(workload, n, sigma_px)
    rng = _rng(*key)
    if workload == 1:
        sigma_phi, phi_max = 16.0, 4.0
    else:
        sigma_phi, phi_max = 4.0, 2.0
    psi = phase_object(rng, geo.ny, geo.nx, sigma_phi, phi_max)
    t = diffuser(rng, geo.ny, geo.nx)
    return {"psi_true": psi, "t": t, "geometry": geo, "seed_key": key}


def roi_batch_specs() -> list[tuple[int, float]]:
    """(side, source sigma px) of the 64 uneven ROI instances: 24x512, 32x1024, 8x2048."""
    master = _rng(BASE_SEED + 3, 0xA11)
    sides = [512] * 24 + [1024] * 32 + [2048] * 8
    sigmas = master.uniform(0.5, 2.0, size=len(sides))
    return [(s, float(g)) for s, g in zip(sides, sigmas)]


# --------------------------------------------------------------------------- phantom

def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly random rotation matrix (unit quaternion from 4 normals)."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoid_phantom(n_vox: int, n_ellipsoids: int = 40, seed_key: tuple[int, ...] = (BASE_SEED + 2,),
                      scale: float = 1.0) -> list[dict]:
    """Random ellipsoids in an ``n_vox^3`` frame centred on the rotation axis.

    Coordinates are in voxels relative to the frame centre, x horizontal,
    y vertical (the rotation axis), z along the beam at angle 0.  ``scale``
    multiplies every length (the 2048^3 phantom is the 1024^3 one with
    ``scale = 2``).
    """
    rng = _rng(*seed_key, 0xE111)
    n = n_vox / scale
    out = []
    for _ in range(n_ellipsoids):
        axes = rng.uniform(n / 32.0, n / 8.0, size=3)
        rot = _random_rotation(rng)
        amax = axes.max()
        r_lim = 0.45 * n - amax
        rad = r_lim * math.sqrt(rng.uniform())
        ang = rng.uniform(0.0, 2.0 * math.pi)
        cy = rng.uniform(0.05 * n + amax, 0.95 * n - amax) - n / 2.0
        centre = np.array([rad * math.cos(ang), cy, rad * math.sin(ang)])
        delta = rng.uniform(1e-7, 5e-7)
        out.append({
            "centre": centre * scale,
            "axes": axes * scale,
            "rot": rot,
            "delta": delta,
            "beta": delta / 100.0,
        })
    return out


def project_ellipsoids(ellipsoids: list[dict], angle_rad: float, ny: int, nx: int,
                       pixel_m: float, wavelength_m: float) -> np.ndarray:
    """Complex phase ``-mu + i phi`` of the phantom rotated by ``angle_rad`` about y.

    Chord lengths through each ellipsoid are the closed-form line/quadric
    intersection along the beam direction at every pixel centre.
    """
    k0 = 2.0 * math.pi / wavelength_m
    ca, sa = math.cos(angle_rad), math.sin(angle_rad)
    ex = np.array([ca, 0.0, -sa])      # detector x direction in the sample frame
    ey = np.array([0.0, 1.0, 0.0])
    d = np.array([sa, 0.0, ca])        # beam direction in the sample frame
    phi = np.zeros((ny, nx))
    mu = np.zeros((ny, nx))
    for e in ellipsoids:
        c, axes, rot = e["centre"], e["axes"], e["rot"]
        a_mat = rot @ np.diag(1.0 / axes ** 2) @ rot.T
        amax = axes.max()
        # bounding box of the projected ellipsoid on the detector (pixel indices)
        u_c, v_c = c @ ex, c @ ey
        i0 = max(int(math.floor(u_c - amax + nx / 2.0 - 1)), 0)
        i1 = min(int(math.ceil(u_c + amax + nx / 2.0 + 1)), nx)
        j0 = max(int(math.floor(v_c - amax + ny / 2.0 - 1)), 0)
        j1 = min(int(math.ceil(v_c + amax + ny / 2.0 + 1)), ny)
        if i1 <= i0 or j1 <= j0:
            continue
        u = (np.arange(i0, i1) + 0.5 - nx / 2.0)[None, :]
        v = (np.arange(j0, j1) + 0.5 - ny / 2.0)[:, None]
        # ray r(s) = u ex + v ey + s d; with w = r(0) - c the chord solves
        # qa s^2 + 2 qb s + qc = 0, expanded as polynomials in (u, v)
        ad, ac = a_mat @ d, a_mat @ c
        qa = d @ ad
        qb = u * (ex @ ad) + v * (ey @ ad) - c @ ad
        qc = (u * u * (ex @ a_mat @ ex) + 2.0 * u * v * (ex @ a_mat @ ey) + v * v * (ey @ a_mat @ ey)
              - 2.0 * u * (ex @ ac) - 2.0 * v * (ey @ ac) + c @ ac - 1.0)
        disc = qb * qb - qa * qc
        chord = 2.0 * np.sqrt(np.maximum(disc, 0.0)) / qa
        chord_m = chord * pixel_m
        phi[j0:j1, i0:i1] += k0 * e["delta"] * chord_m
        mu[j0:j1, i0:i1] += k0 * e["beta"] * chord_m
    return -mu + 1j * phi


def tomo_projection_inputs(workload: int, indices, n_angles: int | None = None) -> dict:
    """Projections ``indices`` of the tomographic workloads (2: 180 x 1024^2, 4: 720 x 2048^2).

    Returns ``psi_true`` (list of complex128 arrays), the shared diffuser ``t``
    (drawn by the 1024^2 single-projection recipe at the workload's size),
    the ``geometry`` and per-projection Poisson ``seed_keys``.
    """
    if workload == 2:
        n, scale, default_angles = 1024, 1.0, 180
    elif workload == 4:
        n, scale, default_angles = 2048, 2.0, 720
    else:
        raise ValueError("tomographic workloads are 2 and 4")
    n_angles = default_angles if n_angles is None else n_angles
    geo = config_geometry(workload, n)
    rng = _rng(BASE_SEED + workload)
    _ = rng.standard_normal((n, n))          # keeps the draw order of the recipe
    t = diffuser(rng, n, n)
    phantom = ellipsoid_phantom(n, 40, (BASE_SEED + 2,), scale)
    psis, keys = [], []
    for j in indices:
        ang = math.pi * j / n_angles
        psis.append(project_ellipsoids(phantom, ang, n, n, geo.pixel_m, geo.wavelength_m))
        keys.append((BASE_SEED + workload, int(j)))
    return {"psi_true": psis, "t": t, "geometry": geo, "seed_keys": keys}
