"""The ellipsoid phantom's projections computed on a torch device.

The same closed-form chords as :func:`synthetic.generators.project_ellipsoids`
(pixel centres, rotation about the vertical axis), evaluated in float64 on the
device so that the 720 x 2048^2 workload is generated in seconds instead of
the CPU's tens of minutes.  Input generation only: no step of the method.
"""

from __future__ import annotations

import math

import numpy as np


def project_ellipsoids_device(ellipsoids: list[dict], angles_rad, ny: int, nx: int, pixel_m: float,
                              wavelength_m: float, out, chunk: int = 16) -> None:
    """Write ``-mu + i phi`` of each angle into ``out[j]`` (complex64 [n_angles, ny, nx] on the device)."""
    import torch
    dev = out.device
    angles = [float(a) for a in angles_rad]
    k0 = 2.0 * math.pi / wavelength_m
    out.zero_()
    ucol = (torch.arange(nx, device=dev, dtype=torch.float64) + 0.5 - nx / 2.0)[None, None, :]
    for e in ellipsoids:
        c, axes, rot = np.asarray(e["centre"]), np.asarray(e["axes"]), np.asarray(e["rot"])
        a_mat = rot @ np.diag(1.0 / axes ** 2) @ rot.T
        amax = float(axes.max())
        v_c = float(c[1])
        j0 = max(int(math.floor(v_c - amax + ny / 2.0 - 1)), 0)
        j1 = min(int(math.ceil(v_c + amax + ny / 2.0 + 1)), ny)
        if j1 <= j0:
            continue
        v = (torch.arange(j0, j1, device=dev, dtype=torch.float64) + 0.5 - ny / 2.0)[None, :, None]
        ey = np.array([0.0, 1.0, 0.0])
        for a0 in range(0, len(angles), chunk):
            ang = angles[a0:a0 + chunk]
            coef = []
            for th in ang:
                ca, sa = math.cos(th), math.sin(th)
                ex = np.array([ca, 0.0, -sa])
                d = np.array([sa, 0.0, ca])
                ad, ac = a_mat @ d, a_mat @ c
                coef.append([d @ ad, ex @ ad, ey @ ad, c @ ad, ex @ a_mat @ ex, ex @ a_mat @ ey, ey @ a_mat @ ey,
                             ex @ ac, ey @ ac, c @ ac])
            q = torch.tensor(coef, device=dev, dtype=torch.float64)[:, :, None, None]   # [A, 10, 1, 1]
            qa, bx, by, bc, axx, axy, ayy, cx, cy, cc = (q[:, i] for i in range(10))
            qb = ucol * bx + v * by - bc
            qc = (ucol * ucol * axx + 2.0 * ucol * v * axy + v * v * ayy - 2.0 * ucol * cx - 2.0 * v * cy + cc - 1.0)
            disc = qb * qb - qa * qc
            chord_m = 2.0 * torch.sqrt(torch.clamp(disc, min=0.0)) / qa * pixel_m
            phase = (k0 * e["delta"]) * chord_m
            atten = (k0 * e["beta"]) * chord_m
            block = out[a0:a0 + len(ang), j0:j1, :]
            block += torch.complex(-atten, phase).to(torch.complex64)
