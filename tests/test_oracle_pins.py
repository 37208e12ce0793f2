"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a textbook closed form, a
brute-force sum, the DFT definition, an invariant of the method, a finite
difference, or a constant printed in the paper (``tests/golden``).
"""

import json
import math
import os

import numpy as np
import pytest

import oracle as O
import synthetic as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _geo(n=32, **kw):
    base = dict(ny=n, nx=n)
    base.update(kw)
    return S.Geometry(**base)


def _rand_c(rng, shape, scale=1.0):
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def _small_problem(n=32, seed=0, **kw):
    rng = np.random.default_rng(seed)
    t = S.diffuser(rng, n, n)
    geo = _geo(n, **{k: v for k, v in kw.items() if k in ("z1_m", "z2_m", "sigma_x_px", "sigma_y_px", "wavelength_m", "pixel_m")})
    rest = {k: v for k, v in kw.items() if k not in ("z1_m", "z2_m", "sigma_x_px", "sigma_y_px", "wavelength_m", "pixel_m")}
    return O.make_problem(t, geo, **rest), rng


# --------------------------------------------------------------------------- Fourier primitive

@pytest.mark.parametrize("ny,nx", [(16, 16), (8, 32), (12, 10)])
def test_fft_matches_direct_dft(ny, nx):
    """The transform used by Filter is the DFT with the exp(-2 pi i k r / n) kernel."""
    rng = np.random.default_rng(1)
    a = _rand_c(rng, (ny, nx))
    ky, kx = np.arange(ny), np.arange(nx)
    ey = np.exp(-2j * math.pi * np.outer(ky, ky) / ny)
    ex = np.exp(-2j * math.pi * np.outer(kx, kx) / nx)
    direct = np.zeros((ny, nx), complex)
    for p in range(ny):
        for q in range(nx):
            direct[p, q] = np.sum(a * ey[p][:, None] * ex[q][None, :])
    assert np.max(np.abs(O.fft2(a) - direct)) <= 1e-12 * np.max(np.abs(direct))
    assert np.max(np.abs(O.ifft2(direct) - a)) <= 1e-13 * np.max(np.abs(a)) * 10


# --------------------------------------------------------------------------- propagation

def test_propagation_is_unitary():
    """|Q| = 1 on propagating bins, so Parseval keeps the field's energy."""
    prob, rng = _small_problem(64)
    a = _rand_c(rng, (64, 64))
    for dist in (5e-3, 0.2, -0.2, 3.0):
        b = O.free_propagation(a, prob, dist)
        assert abs(np.linalg.norm(b) / np.linalg.norm(a) - 1.0) <= 1e-14


def test_zero_distance_is_identity():
    prob, rng = _small_problem(32)
    a = _rand_c(rng, (32, 32))
    assert np.max(np.abs(O.free_propagation(a, prob, 0.0) - a)) <= 1e-15 * 10


def test_propagations_compose():
    """Q is exponential in L: two propagations equal one over the summed distance."""
    prob, rng = _small_problem(32)
    a = _rand_c(rng, (32, 32))
    b = O.free_propagation(O.free_propagation(a, prob, 5e-3), prob, 0.2)
    c = O.free_propagation(a, prob, 0.205)
    assert np.max(np.abs(b - c)) <= 1e-14 * np.max(np.abs(a)) * 10


def test_backward_propagation_is_adjoint():
    """<P_L a, b> = <a, P_{-L} b>: FreePropagation(-L) is the adjoint used by the gradient."""
    prob, rng = _small_problem(32)
    a, b = _rand_c(rng, (32, 32)), _rand_c(rng, (32, 32))
    lhs = np.vdot(O.free_propagation(a, prob, 0.2), b)
    rhs = np.vdot(a, O.free_propagation(b, prob, -0.2))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_gaussian_beam_closed_form():
    """Paraxial Gaussian beam: u(z) = exp(-r^2/(w0^2 q)) / q with q = 1 + i z / z_R."""
    n, p, lam, w0_px, z = 128, 1e-6, 0.05e-9, 4.0, 2.0
    geo = _geo(n, pixel_m=p, wavelength_m=lam)
    prob = O.make_problem(np.ones((n, n)), geo)
    c = (np.arange(n) - n // 2) * p
    xx, yy = np.meshgrid(c, c)
    r2 = xx ** 2 + yy ** 2
    w0 = w0_px * p
    u0 = np.exp(-r2 / w0 ** 2)
    z_r = math.pi * w0 ** 2 / lam
    q = 1.0 + 1j * z / z_r
    expect = np.exp(-r2 / (w0 ** 2 * q)) / q
    got = O.free_propagation(u0, prob, z)
    assert np.max(np.abs(got - expect)) <= 1e-10
    # the opposite sign convention would be far off
    wrong = np.exp(-r2 / (w0 ** 2 * np.conj(q))) / np.conj(q)
    assert np.max(np.abs(got - wrong)) > 1e-2


def test_brute_force_fresnel_integral_32():
    """Direct Fresnel sum on a 32x32 support against the transfer-function result.

    u(x) = (i lambda z)^-1 sum_x' u0(x') exp(i pi |x - x'|^2 / (lambda z)) p^2,
    the impulse response paired with the paraxial form of the propagator.  The
    TF result is taken on a zero-padded 256^2 grid so that nothing wraps.
    """
    n, npad, p, lam, z = 32, 256, 1e-6, 0.05e-9, 2.0
    rng = np.random.default_rng(7)
    c = (np.arange(n) - n // 2) * p
    xx, yy = np.meshgrid(c, c)
    # Gaussian envelope (w0 = 4 px) times a smooth random phase of at most 1 rad:
    # the integrand of the direct sum stays well inside the sampling band.
    w0 = 4.0 * p
    smooth = np.real(np.fft.ifft2(np.fft.fft2(rng.standard_normal((n, n))) *
                                  np.exp(-2 * math.pi ** 2 * 3.0 ** 2 *
                                         (np.fft.fftfreq(n)[:, None] ** 2 + np.fft.fftfreq(n)[None, :] ** 2))))
    u0 = np.exp(-(xx ** 2 + yy ** 2) / w0 ** 2) * np.exp(1j * smooth / np.abs(smooth).max())
    # brute force on the 32x32 output window
    dx = xx.ravel()[:, None] - xx.ravel()[None, :]
    dy = yy.ravel()[:, None] - yy.ravel()[None, :]
    kern = np.exp(1j * math.pi * (dx ** 2 + dy ** 2) / (lam * z)) / (1j * lam * z) * p * p
    brute = (kern @ u0.ravel()).reshape(n, n)
    # transfer function on a padded grid
    geo = _geo(npad, pixel_m=p, wavelength_m=lam)
    prob = O.make_problem(np.ones((npad, npad)), geo)
    big = np.zeros((npad, npad), complex)
    o = npad // 2 - n // 2
    big[o:o + n, o:o + n] = u0
    tf = O.free_propagation(big, prob, z)[o:o + n, o:o + n]
    err = np.max(np.abs(tf - brute)) / np.max(np.abs(brute))
    assert err <= 1e-6, err
    tf_wrong = O.free_propagation(big, prob, -z)[o:o + n, o:o + n]
    assert np.max(np.abs(tf_wrong - brute)) / np.max(np.abs(brute)) >= 1e-3


def test_evanescent_bins_are_zero():
    """Bins with lambda^2 rho^2 >= 1 do not propagate."""
    u, v = O.spatial_frequencies(16, 16, 1e-9)
    q = O.transfer_function(u, v, 1.5e-9, 1e-6)
    rho2 = u * u + v * v
    assert np.all(q[(1.5e-9) ** 2 * rho2 >= 1.0] == 0)
    assert np.allclose(np.abs(q[(1.5e-9) ** 2 * rho2 < 1.0]), 1.0, atol=1e-15)


# --------------------------------------------------------------------------- coherence windows

def test_iotf_is_transform_of_unit_ipsf():
    """Eq. 5 is the Fourier transform of Eq. 4 (unit integral, std sigma px)."""
    n, p, sig = 64, 1e-6, 2.0
    x_coh, y_coh = O.coherence_lengths(sig, sig, p)
    k = O.ipsf_kernel(n, n, p, x_coh, y_coh)
    assert abs(np.sum(k) * p * p - 1.0) <= 1e-12
    xs = np.where(np.arange(n) < n // 2, np.arange(n), np.arange(n) - n)
    assert abs(np.sum(k * (xs[None, :] * 1.0) ** 2) * p * p - sig ** 2) <= 1e-9
    u, v = O.spatial_frequencies(n, n, p)
    win = O.iotf_window(u, v, x_coh, y_coh)
    dft = np.real(O.fft2(k)) * p * p
    assert np.max(np.abs(dft - win)) <= 1e-7


def test_stf_relation_to_iotf():
    """Eqs. 5 and 14 at the same coherence lengths: STF = IOTF^(2 gamma); Gamma^2(0) = 0."""
    u, v = O.spatial_frequencies(32, 48, 1e-6)
    x_coh, y_coh = 3.47e-6, 4.31e-6
    for gamma in (0.5, 1.0, 4.0):
        stf = O.stf_window(u, v, x_coh, y_coh, gamma)
        assert np.allclose(stf, O.iotf_window(u, v, x_coh, y_coh) ** (2 * gamma), rtol=1e-13)
        g2 = O.regularization_window(u, v, x_coh, y_coh, gamma)
        assert g2[0, 0] == 0.0 and np.all(g2 >= 0) and np.all(g2 <= 1)


def test_source_forms_agree():
    """The three ways to give the source describe the same windows for a Gaussian IPSF:
    sigma px (Eq. 4 with x_coh = 2 sqrt(pi) sigma p), the coherence lengths (Eq. 5), and
    the sampled IOTF with STF = IOTF^(2 gamma) (Eqs. 5, 14)."""
    n, p = 48, 1e-6
    rng = np.random.default_rng(21)
    t = S.diffuser(rng, n, n)
    sx, sy = 1.3, 0.7
    geo = _geo(n, pixel_m=p, sigma_x_px=sx, sigma_y_px=sy)
    for gamma in (1.0, 0.6):
        a = O.make_problem(t, geo, gamma=gamma)
        b = O.make_problem(t, _geo(n, pixel_m=p, sigma_x_px=0.0, sigma_y_px=0.0), gamma=gamma,
                           coherence=(2 * math.sqrt(math.pi) * sx * p, 2 * math.sqrt(math.pi) * sy * p))
        c = O.make_problem(t, _geo(n, pixel_m=p), gamma=gamma, iotf=a.iotf)
        fy = np.fft.fftfreq(n)[:, None]
        fx = np.fft.fftfreq(n)[None, :]
        gauss = np.exp(-2 * math.pi ** 2 * (sx * sx * fx * fx + sy * sy * fy * fy))   # OTF of the IPSF
        for prob in (a, b, c):
            assert np.max(np.abs(prob.iotf - gauss)) <= 1e-15
            assert np.max(np.abs(prob.gamma2 - (1 - gauss ** (2 * gamma)))) <= 1e-14


# --------------------------------------------------------------------------- forward model

def test_no_propagation_forward_and_gradient():
    """L1 = L2 = 0, t = 1, no blur: f = exp(2 Re psi) and g = -e exp(2 Re psi) (real)."""
    n = 16
    geo = _geo(n, z1_m=0.0, z2_m=0.0, sigma_x_px=0.0, sigma_y_px=0.0)
    prob = O.make_problem(np.ones((n, n), np.complex64), geo)
    rng = np.random.default_rng(3)
    psi = _rand_c(rng, (n, n), 0.3)
    y = rng.uniform(0.5, 1.5, (n, n))
    f, _, _ = O.physical_model(psi, prob)
    assert np.max(np.abs(f - np.exp(2 * psi.real))) <= 1e-14 * 10
    _, g, _ = O.gradient(psi, y, prob)
    e = y - f
    assert np.max(np.abs(g - (-e * np.exp(2 * psi.real)))) <= 1e-14 * 10


def test_weak_object_contrast_transfer():
    """Weak object, t = 1, no blur: I^ = delta + 2 eps [sin(pi lam L rho^2) Phi - cos(pi lam L rho^2) M] + O(eps^2)."""
    n, p, lam, l1, l2 = 64, 1e-6, 0.05e-9, 5e-3, 0.2
    geo = _geo(n, pixel_m=p, wavelength_m=lam, z1_m=l1, z2_m=l2, sigma_x_px=0.0, sigma_y_px=0.0)
    prob = O.make_problem(np.ones((n, n)), geo)
    rng = np.random.default_rng(4)
    mu1, phi1 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    u, v = O.spatial_frequencies(n, n, p)
    arg = math.pi * lam * (l1 + l2) * (u * u + v * v)
    errs = []
    for eps in (1e-3, 2e-3):
        f, _, _ = O.physical_model(eps * (-mu1 + 1j * phi1), prob)
        spec = O.fft2(f)
        spec[0, 0] -= n * n
        pred = 2 * eps * (np.sin(arg) * O.fft2(phi1) - np.cos(arg) * O.fft2(mu1))
        errs.append(np.max(np.abs(spec - pred)))
        assert np.max(np.abs(spec - pred)) <= 0.05 * np.max(np.abs(pred))
    assert 3.0 <= errs[1] / errs[0] <= 5.0   # residual is second order in eps


def _gaussian_otf(ny, nx, sx, sy):
    """Fourier transform of a unit-integral Gaussian of std (sx, sy) px: exp(-2 pi^2 (sx^2 fx^2 + sy^2 fy^2))."""
    fy = np.fft.fftfreq(ny)[:, None]
    fx = np.fft.fftfreq(nx)[None, :]
    return np.exp(-2.0 * math.pi ** 2 * (sx * sx * fx * fx + sy * sy * fy * fy))


@pytest.mark.parametrize("sx,sy", [(1.5, 1.5), (1.0, 2.0)])
def test_weak_object_contrast_transfer_with_source_blur(sx, sy):
    """Weak object, t = 1, Gaussian IPSF of std (sx, sy) px (Eqs. 1, 4-5): the intensity
    spectrum is the weak-object CTF times the Gaussian's transform,
    F{f} = OTF [delta + 2 eps (sin(pi lam L rho^2) Phi - cos(pi lam L rho^2) M)] + O(eps^2).
    Fails if the blur is left out, applied twice, or with the wrong width."""
    n, p, lam, l1, l2 = 64, 1e-6, 0.05e-9, 5e-3, 0.2
    geo = _geo(n, pixel_m=p, wavelength_m=lam, z1_m=l1, z2_m=l2, sigma_x_px=sx, sigma_y_px=sy)
    prob = O.make_problem(np.ones((n, n)), geo)
    rng = np.random.default_rng(14)
    mu1, phi1 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    u, v = O.spatial_frequencies(n, n, p)
    arg = math.pi * lam * (l1 + l2) * (u * u + v * v)
    otf = _gaussian_otf(n, n, sx, sy)
    errs = []
    for eps in (1e-3, 2e-3):
        f, _, _ = O.physical_model(eps * (-mu1 + 1j * phi1), prob)
        spec = O.fft2(f)
        spec[0, 0] -= n * n
        pred = otf * 2 * eps * (np.sin(arg) * O.fft2(phi1) - np.cos(arg) * O.fft2(mu1))
        # the DC bin holds the O(eps^2) change of the mean intensity: compare the others
        spec[0, 0] = pred[0, 0] = 0.0
        errs.append(np.max(np.abs(spec - pred)))
        assert np.max(np.abs(spec - pred)) <= 0.05 * np.max(np.abs(pred))
        # without the blur the same comparison is far off
        assert np.max(np.abs(spec - pred / otf)) >= 0.2 * np.max(np.abs(pred))
    assert 3.0 <= errs[1] / errs[0] <= 5.0


def test_source_blur_is_convolution_with_sampled_ipsf():
    """Eq. 1's blur: f at sigma = 2 px equals the circular convolution of the coherent
    intensity (sigma = 0) with the unit-sum Gaussian exp(-r^2 / 2 sigma^2) (Eq. 4 in
    pixels), summed shift by shift on 32 x 32 (aliasing of a 2 px Gaussian < 1e-12)."""
    n, sig = 32, 2.0
    rng = np.random.default_rng(15)
    t = S.diffuser(rng, n, n)
    psi = S.phase_object(rng, n, n, 3.0, 2.0)
    coh = O.make_problem(t, _geo(n, sigma_x_px=0.0, sigma_y_px=0.0))
    blur = O.make_problem(t, _geo(n, sigma_x_px=sig, sigma_y_px=sig))
    i0, _, _ = O.physical_model(psi, coh)
    f, _, _ = O.physical_model(psi, blur)
    d = np.where(np.arange(n) <= n // 2, np.arange(n), np.arange(n) - n).astype(np.float64)
    ker = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2 * sig * sig))
    ker /= ker.sum()
    conv = np.zeros((n, n))
    for dy in range(n):
        for dx in range(n):
            conv += ker[dy, dx] * np.roll(np.roll(i0, dy, axis=0), dx, axis=1)
    assert np.max(np.abs(f - conv)) <= 1e-10 * np.max(np.abs(conv))
    assert np.max(np.abs(i0 - conv)) >= 1e-3 * np.max(np.abs(conv))   # the blur is not vacuous


def test_truth_point_has_zero_loss_and_gradient():
    """Noise-free y made at psi_true: L = 0 and g = 0 there."""
    prob, rng = _small_problem(32, z1_m=5e-3, z2_m=0.2, sigma_x_px=1.0, sigma_y_px=1.0)
    psi = S.phase_object(rng, 32, 32, 4.0, 2.0)
    f, _, _ = O.physical_model(psi, prob)
    l, g, _ = O.gradient(psi, f, prob)
    assert l <= 1e-26 * f.size
    assert np.max(np.abs(g)) <= 1e-13


def test_linearised_model_adjoint():
    """Dot-product test of the Jacobian: <J dpsi, w> = Re<J^T w, dpsi>, and J^T w = -2 max|t|^2 g(e = w).

    The JVP is checked against central differences of the forward model, so
    both sides of the adjoint identity are tied to f itself."""
    prob, rng = _small_problem(32, z1_m=5e-3, z2_m=0.2, sigma_x_px=1.5, sigma_y_px=1.0)
    psi = _rand_c(rng, (32, 32), 0.2)
    dpsi = _rand_c(rng, (32, 32))
    w = rng.standard_normal((32, 32))
    jv = O.model_jvp(psi, dpsi, prob)
    h = 1e-6
    fd = (O.physical_model(psi + h * dpsi, prob)[0] - O.physical_model(psi - h * dpsi, prob)[0]) / (2 * h)
    assert np.max(np.abs(jv - fd)) <= 1e-7 * np.max(np.abs(jv))
    lhs = np.sum(jv * w)
    _, x, v = O.physical_model(psi, prob)
    jt_w = O.model_vjp(x, v, w, prob)
    assert abs(lhs - np.real(np.vdot(jt_w, dpsi))) <= 1e-12 * abs(lhs)
    g_w = O.wirtinger_derivative(w, x, v, prob)
    assert np.max(np.abs(jt_w + 2.0 * np.max(np.abs(prob.t) ** 2) * g_w)) <= 1e-13 * np.max(np.abs(jt_w))


def test_gradient_matches_central_differences():
    """grad_real L = dL/dRe psi + i dL/dIm psi = 4 max|t|^2 g (central differences, h = 1e-4)."""
    n = 32
    prob, rng = _small_problem(n, z1_m=5e-3, z2_m=0.2, sigma_x_px=1.0, sigma_y_px=1.0)
    psi = S.phase_object(rng, n, n, 4.0, 2.0)
    f, _, _ = O.physical_model(psi, prob)
    y = f + 0.05 * rng.standard_normal((n, n))
    _, g, _ = O.gradient(psi, y, prob)
    scale = 4.0 * np.max(np.abs(prob.t) ** 2)
    h = 1e-4
    for idx in rng.choice(n * n, 8, replace=False):
        r, c = divmod(int(idx), n)
        for unit in (1.0, 1j):
            dp = np.zeros((n, n), complex)
            dp[r, c] = h * unit
            lp = O.loss(y, O.physical_model(psi + dp, prob)[0])
            lm = O.loss(y, O.physical_model(psi - dp, prob)[0])
            fd = (lp - lm) / (2 * h)
            an = scale * (g[r, c].real if unit == 1.0 else g[r, c].imag)
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (r, c, unit, fd, an)


# --------------------------------------------------------------------------- update direction

def test_regularizer_is_gradient_of_tikhonov_energy():
    """Regularizer = grad_real of R = Re(a)/2 ||Gamma Re psi||^2 + Im(a)/2 ||Gamma Im psi||^2."""
    n = 24
    prob, rng = _small_problem(n, sigma_x_px=1.0, sigma_y_px=1.5, alpha=complex(0.3, 0.07))
    psi = _rand_c(rng, (n, n))

    def energy(p):
        a, b = O.fft2(p.real), O.fft2(p.imag)
        return (prob.alpha.real / 2 * np.sum(prob.gamma2 * np.abs(a) ** 2) +
                prob.alpha.imag / 2 * np.sum(prob.gamma2 * np.abs(b) ** 2)) / p.size

    rho = O.regularizer(psi, prob)
    h = 1e-5
    for idx in rng.choice(n * n, 6, replace=False):
        r, c = divmod(int(idx), n)
        for unit in (1.0, 1j):
            dp = np.zeros((n, n), complex)
            dp[r, c] = h * unit
            fd = (energy(psi + dp) - energy(psi - dp)) / (2 * h)
            an = rho[r, c].real if unit == 1.0 else rho[r, c].imag
            assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))


def test_preconditioner_single_fourier_mode():
    """A cosine of bin (ky, kx) in Im g is scaled by s_P / ((kx/nx)^2 + (ky/ny)^2); Re g passes; DC -> 0."""
    ny, nx = 32, 48
    prob = O.make_problem(np.ones((ny, nx)), _geo(ny, nx=nx))
    yy, xx = np.mgrid[0:ny, 0:nx]
    s_p = 1.0 / (4 * math.pi ** 2)
    for ky, kx in ((1, 0), (3, 5), (16, 24), (5, 47)):
        mode = np.cos(2 * math.pi * (ky * yy / ny + kx * xx / nx))
        out = O.preconditioner(0.7 * mode + 1j * mode, prob)
        fy = ky if ky <= ny // 2 else ky - ny
        fx = kx if kx <= nx // 2 else kx - nx
        assert np.allclose(out.real, 0.7 * mode, atol=1e-14)
        assert np.allclose(out.imag, mode * s_p / ((fx / nx) ** 2 + (fy / ny) ** 2), atol=1e-11)
    out = O.preconditioner(1j * np.ones((ny, nx)), prob)
    assert np.max(np.abs(out.imag)) <= 1e-15


def test_nesterov_scalars():
    """tau_1 = golden ratio, tau_2 = 2.193527; momentum (tau_prev - 1)/tau = 0, 0.281754, 0.434043."""
    taus = [1.0]
    for _ in range(3):
        taus.append(O.nesterov_tau(taus[-1]))
    assert abs(taus[1] - (1 + math.sqrt(5)) / 2) <= 1e-15
    assert abs(taus[2] - 2.193527) <= 5e-7
    betas = [(taus[k] - 1) / taus[k + 1] for k in range(3)]
    assert betas[0] == 0.0
    assert abs(betas[1] - 0.281754) <= 5e-7 and abs(betas[2] - 0.434043) <= 5e-7


def test_nesterov_meets_accelerated_rate_where_plain_descent_does_not():
    """FISTA bound f(z_k) - f* <= 2 L ||x0 - x*||^2 / (k+1)^2 on an ill-conditioned quadratic.

    Plain gradient descent with the same step exceeds the bound, so the test
    fails if the momentum term is lost or mis-signed.
    """
    h = np.logspace(-5, 0, 400)
    lip = h.max()
    x0 = np.ones_like(h)
    fval = lambda x: 0.5 * np.sum(h * x * x)
    bound = lambda k: 2 * lip * np.sum(x0 * x0) / (k + 1) ** 2
    psi, z, tau = x0.copy(), np.zeros_like(x0), 1.0
    gd = x0.copy()
    ok_gd = True
    for k in range(1, 201):
        z, tau, psi = O.nesterov_update(psi, z if k > 1 else np.zeros_like(x0), tau, h * psi, 1.0 / lip)
        gd = gd - (h * gd) / lip
        assert fval(z) <= bound(k)
        ok_gd = ok_gd and fval(gd) <= bound(k)
    assert not ok_gd


def test_phase_mean_is_invariant():
    """P^-1(0) = 0 and Gamma^2(0) = 0: the mean of Im psi never moves from 0."""
    inp = S.instance_inputs(0)
    prob = O.make_problem(inp["t"], inp["geometry"])
    f, _, _ = O.physical_model(inp["psi_true"], prob)
    y = S.poisson_intensity(f, inp["seed_key"])
    st = O.initial_state(prob.shape)
    for _ in range(6):
        st, _ = O.pwf_step(st, y, prob)
        assert abs(np.mean(st.psi.imag)) <= 1e-13
        assert abs(np.mean(st.psi.real)) > 1e-6   # the attenuation DC does move


def test_loss_decreases_on_small_workload():
    """With the default step size the 128^2 workload's loss falls monotonically over 50 iterations."""
    inp = S.instance_inputs(0)
    prob = O.make_problem(inp["t"], inp["geometry"])
    f, _, _ = O.physical_model(inp["psi_true"], prob)
    y = S.poisson_intensity(f, inp["seed_key"])
    _, hist, _ = O.pwf(y, prob, 50)
    assert np.all(np.diff(hist) < 0)
    assert hist[-1] < O.loss(y, f)   # below the noise floor of the truth


# --------------------------------------------------------------------------- stopping correlation
#
# The stopping rule (Methods, "Reconstruction procedure") correlates the
# retrieved fields exp(psi) of consecutive iterations.  The pins below fix the
# normalisation, the modulus and the use of exp(psi) rather than psi.

def _corr_field(n=16, seed=11):
    rng = np.random.default_rng(seed)
    # varying amplitude (so a missing normalisation shows) and phase
    return -0.3 * rng.uniform(0.0, 1.0, (n, n)) + 1j * rng.uniform(-3.0, 3.0, (n, n))


def test_field_correlation_of_global_phase_shift_is_one():
    """x_b = exp(i theta) x_a is the same field: the correlation is exactly 1."""
    psi = _corr_field()
    for theta in (0.0, 0.4, -2.5, 3.0):
        assert abs(O.field_correlation(psi, psi + 1j * theta) - 1.0) <= 1e-14


def test_field_correlation_of_orthogonal_fields_is_zero():
    """Plane waves of two different DFT bins are orthogonal fields: correlation 0.

    As phases (psi itself) the two are far from orthogonal, so correlating psi
    instead of exp(psi) fails here."""
    n = 16
    yy, xx = np.mgrid[0:n, 0:n]
    amp = -0.7   # a constant attenuation leaves the fields orthogonal
    for (a, b) in (((1, 0), (0, 1)), ((2, 3), (5, 3)), ((0, 0), (4, 7))):
        pa = amp + 2j * math.pi * (a[0] * yy + a[1] * xx) / n
        pb = 2j * math.pi * (b[0] * yy + b[1] * xx) / n
        assert O.field_correlation(pa, pb) <= 1e-13
        assert abs(np.vdot(pa, pb)) / (np.linalg.norm(pa) * np.linalg.norm(pb)) > 0.1


def test_field_correlation_second_order_closed_form():
    """psi_b = psi_a + eps xi: 1 - corr = (eps^2 / 2) Var_w(xi) + O(eps^3), w = |x_a|^2.

    For a phase perturbation (xi = i eta) the correlation is the modulus of
    the w-weighted characteristic function of eta, for an amplitude one the
    ratio of moment generating functions; both expand to the weighted
    variance at second order."""
    psi = _corr_field(24, 5)
    rng = np.random.default_rng(6)
    w = np.exp(2.0 * psi.real)
    w = w / w.sum()
    for kind in ("phase", "amplitude"):
        xi = rng.standard_normal(psi.shape)
        var = float(np.sum(w * xi * xi) - np.sum(w * xi) ** 2)
        ratios = []
        for eps in (1e-3, 2e-3):
            d = 1j * eps * xi if kind == "phase" else eps * xi
            got = 1.0 - O.field_correlation(psi, psi + d)
            ratios.append(got / (0.5 * eps * eps * var))
        assert abs(ratios[0] - 1.0) <= 1e-2, (kind, ratios)
        # the deviation from the closed form shrinks with eps
        assert abs(ratios[1] - 1.0) >= abs(ratios[0] - 1.0) - 1e-6


def test_field_correlation_brute_force_8x8():
    """Explicit double loop over the 8 x 8 pixels of |sum conj(x_a) x_b| / (|x_a| |x_b|)."""
    rng = np.random.default_rng(8)
    pa = rng.uniform(-0.5, 0.2, (8, 8)) + 1j * rng.uniform(-3, 3, (8, 8))
    pb = rng.uniform(-0.5, 0.2, (8, 8)) + 1j * rng.uniform(-3, 3, (8, 8))
    num_re = num_im = na = nb = 0.0
    for r in range(8):
        for c in range(8):
            ar = math.exp(pa[r, c].real) * math.cos(pa[r, c].imag)
            ai = math.exp(pa[r, c].real) * math.sin(pa[r, c].imag)
            br = math.exp(pb[r, c].real) * math.cos(pb[r, c].imag)
            bi = math.exp(pb[r, c].real) * math.sin(pb[r, c].imag)
            num_re += ar * br + ai * bi
            num_im += ar * bi - ai * br
            na += ar * ar + ai * ai
            nb += br * br + bi * bi
    expect = math.hypot(num_re, num_im) / math.sqrt(na * nb)
    assert abs(O.field_correlation(pa, pb) - expect) <= 1e-14
    assert 0.0 < expect < 1.0


def test_correlation_stop():
    inp = S.instance_inputs(0)
    prob = O.make_problem(inp["t"], inp["geometry"])
    f, _, _ = O.physical_model(inp["psi_true"], prob)
    y = S.poisson_intensity(f, inp["seed_key"])
    _, hist, st = O.pwf(y, prob, 400, corr_tol=O.PAPER_STOP_CORR)
    assert 1 <= len(hist) < 400 and st.k == len(hist)
    assert abs((1 - O.PAPER_STOP_CORR) - 2.3026e-5) <= 1e-9


def test_nonfinite_loss_raises():
    prob, rng = _small_problem(16)
    y = np.full((16, 16), np.nan)
    with pytest.raises(FloatingPointError):
        O.pwf_step(O.initial_state((16, 16)), y, prob)


def test_paper_constants():
    """Defaults that the paper prints match the cited values."""
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        c = json.load(fh)
    assert O.PAPER_ALPHA == complex(c["alpha_re"]["value"], c["alpha_im"]["value"])
    assert O.PAPER_GAMMA == c["gamma"]["value"]
    assert O.PAPER_ETA == c["eta"]["value"]
    assert O.PAPER_STOP_CORR == 10.0 ** c["stop_exponent"]["value"]
    # coherence lengths of the beamline data correspond to an IPSF std of about 1 px at 1 um
    sig = c["x_coh_m"]["value"] / (2 * math.sqrt(math.pi) * 1e-6)
    assert 0.9 < sig < 1.1
