"""Plain FP64 oracle of preconditioned Wirtinger flow (PWF).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP path.

The oracle follows the paper "Speckle-based X-ray microtomography via
preconditioned Wirtinger flow" (Lee, Hugonnet, Lim, Park; arXiv 2503.20146).
The forward model is Eq. 1 written as a composition of operators
(propagation, diffuser, squared modulus, source blur); the gradient of the
loss of Eq. 2 is the transpose of that model's Jacobian applied to the
misfit, scaled as the paper's Wirtinger gradient; the direction adds the
inverse-Laplacian preconditioner of Eqs. 6-11 and the gradient of the
Tikhonov term with the window of Eqs. 14-15; the loop is the Nesterov
iteration of Algorithm S1.  Every operation is complex128/float64 and uses
``scipy.fft`` as the Fourier transform primitive; nothing is blocked or
fused.

Notation.  ``psi = log x = -mu + i phi`` is the complex phase (Results,
"Preconditioned Wirtinger flow").  Algorithm S1 reuses the letters phi and mu
for the Nesterov gradient-step iterate and the momentum scalar; here they are
``z`` and ``tau`` so that phi and mu keep their physical meaning.

Readings where the paper is silent or ambiguous (each one is listed in the
design notes of the repository):

* Propagator: angular spectrum with the constant carrier ``exp(i 2 pi L /
  lambda)`` dropped (a global phase that cancels in ``|v|^2`` and in the
  gradient), in the cancellation-free form
  ``theta = -2 pi L lambda rho^2 / (1 + sqrt(1 - lambda^2 rho^2))``; bins with
  ``lambda^2 rho^2 >= 1`` are evanescent and set to 0.
* Preconditioner: Eqs. 9-11 derive the inverse Laplacian and then drop its
  constants (the 4 pi^2 of the Laplacian's Fourier symbol, its sign and a
  factor 2).  Here ``P^-1_k = s_P / (u^2 + v^2)`` with frequencies in cycles
  per pixel and ``s_P = 1 / (4 pi^2)``, i.e. the magnitude of the inverse
  Laplacian symbol on the pixel grid; its DC value is 0 (text after Eq. 11).
* Step size: the paper fixes ``eta = 1`` for its beamline normalisation.  With
  unit flat field, ``max|t|^2 ~ 1`` and the geometry of the synthetic
  workloads, the unpreconditioned absorption channel of the Gauss-Newton
  operator has ``eta * lambda_max ~ 1.7 > 4/3`` at ``eta = 1``, beyond the
  stability limit of Nesterov momentum, so the default is ``eta = 1/2``: the
  largest of {1, 1/2, 1/4, 1/8} for which the 128^2 workload's loss falls
  monotonically over 50 iterations.
* Filters of real images by real even windows keep the real part
  (IOTF, preconditioner): the imaginary residue is rounding only.
* The IPSF is Gaussian with standard deviation ``sigma`` px at the detector,
  i.e. ``x_coh = 2 sqrt(pi) sigma p`` in Eqs. 4-5; the IOTF is applied as a
  Fourier window (Results: "equivalently ... as a window function").
* The loss is the plain sum of Eq. 2; the loss history holds the loss at the
  iterate that enters each iteration.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.fft as _sfft

PAPER_ALPHA = complex(0.1, 0.01)   # regularisation parameter (Results, PWF subsection)
PAPER_GAMMA = 1.0                  # oversampling ratio (Results, PWF subsection)
PAPER_ETA = 1.0                    # step size (Results, PWF subsection)
PAPER_STOP_CORR = 10.0 ** (-0.00001)  # stopping correlation (Methods, Reconstruction procedure)
DEFAULT_ETA = 0.5                     # step size used for the synthetic workloads (see header)
DEFAULT_PRECOND_SCALE = 1.0 / (4.0 * math.pi ** 2)  # s_P of the preconditioner (see header)


# --------------------------------------------------------------------------- grids & windows

def spatial_frequencies(ny: int, nx: int, pixel_m: float):
    """Spatial frequencies ``u`` (along x) and ``v`` (along y) in cycles/m.

    DFT bin ``k`` of an ``n``-point axis has frequency ``k/(n p)`` for
    ``k < n/2`` and ``(k - n)/(n p)`` otherwise (the usual FFT ordering).
    """
    def axis(n):
        k = np.arange(n, dtype=np.float64)
        k = np.where(k < (n + 1) // 2, k, k - n)
        return k / (n * pixel_m)
    return axis(nx)[None, :], axis(ny)[:, None]


def coherence_lengths(sigma_x_px: float, sigma_y_px: float, pixel_m: float):
    """``x_coh, y_coh`` of a Gaussian IPSF of std ``sigma`` px (Eq. 4 rewritten)."""
    c = 2.0 * math.sqrt(math.pi) * pixel_m
    return c * sigma_x_px, c * sigma_y_px


def iotf_window(u, v, x_coh: float, y_coh: float):
    """Eq. 5: ``IOTF_k = exp[-(pi/2)(u^2 x_coh^2 + v^2 y_coh^2)]``."""
    return np.exp(-0.5 * math.pi * (u * u * x_coh * x_coh + v * v * y_coh * y_coh))


def ipsf_kernel(ny: int, nx: int, pixel_m: float, x_coh: float, y_coh: float):
    """Eq. 4 sampled at pixel centres of a periodic grid (origin at index 0), in 1/m^2."""
    def axis(n):
        k = np.arange(n, dtype=np.float64)
        return np.where(k < (n + 1) // 2, k, k - n) * pixel_m
    x = axis(nx)[None, :]
    y = axis(ny)[:, None]
    return 2.0 / (x_coh * y_coh) * np.exp(-2.0 * math.pi * (x * x / x_coh ** 2 + y * y / y_coh ** 2))


def stf_window(u, v, x_coh: float, y_coh: float, gamma: float):
    """Eq. 14: ``STF_k = exp[-pi gamma (u^2 x_coh^2 + v^2 y_coh^2)]``."""
    return np.exp(-math.pi * gamma * (u * u * x_coh * x_coh + v * v * y_coh * y_coh))


def regularization_window(u, v, x_coh: float, y_coh: float, gamma: float):
    """Eq. 15: ``Gamma^2_k = 1 - STF_k``."""
    return 1.0 - stf_window(u, v, x_coh, y_coh, gamma)


def preconditioning_filter(u, v, pixel_m: float, scale: float = DEFAULT_PRECOND_SCALE):
    """Eq. 11: ``P^-1_k = scale/(u^2 + v^2)`` with frequencies in cycles/pixel; 0 at DC."""
    rho2 = (u * u + v * v) * pixel_m * pixel_m
    out = np.zeros(np.broadcast(u, v).shape)
    nz = rho2 > 0
    out[nz] = scale / rho2[nz]
    return out


def transfer_function(u, v, wavelength_m: float, distance_m: float):
    """FreePropagation window ``Q_k = exp(i 2 pi w L)``, ``w = sqrt(lambda^-2 - u^2 - v^2)``.

    The constant ``exp(i 2 pi L / lambda)`` is dropped.  The remaining phase
    ``2 pi L (w - 1/lambda)`` is evaluated without cancellation; evanescent
    bins (``lambda^2 rho^2 >= 1``) are 0.
    """
    rho2 = u * u + v * v
    s = wavelength_m * wavelength_m * rho2
    prop = s < 1.0
    root = np.sqrt(np.where(prop, 1.0 - s, 0.0))
    theta = -2.0 * math.pi * distance_m * wavelength_m * rho2 / (1.0 + root)
    return np.where(prop, np.exp(1j * theta), 0.0)


# --------------------------------------------------------------------------- problem

@dataclasses.dataclass
class Problem:
    """Everything Algorithm S1 takes besides ``y`` (windows precomputed in FP64)."""

    t: np.ndarray            # diffuser transmission, complex128
    wavelength_m: float
    z1_m: float
    z2_m: float
    pixel_m: float
    iotf: np.ndarray         # IOTF_k
    p_inv: np.ndarray        # P^-1_k
    gamma2: np.ndarray       # Gamma^2_k
    alpha: complex
    eta: float
    u: np.ndarray
    v: np.ndarray
    precondition: bool = True

    @property
    def shape(self):
        return self.t.shape


def make_problem(t, geometry, *, alpha: complex = PAPER_ALPHA, gamma: float = PAPER_GAMMA,
                 eta: float = DEFAULT_ETA, precond_scale: float = DEFAULT_PRECOND_SCALE,
                 precondition: bool = True, coherence: tuple[float, float] | None = None,
                 iotf: np.ndarray | None = None) -> Problem:
    """Build the FP64 windows of one projection from a ``synthetic.Geometry``-like object.

    The source is the geometry's Gaussian IPSF (``sigma_*_px``), or the coherence
    lengths ``coherence = (x_coh, y_coh)`` in metres (Eqs. 4-5), or a given IOTF
    window ``iotf`` on the DFT grid.  For a given window the sample transfer
    function is ``STF = IOTF^(2 gamma)`` (negative samples count as 0), the
    relation that Eqs. 5 and 14 give for the Gaussian model."""
    g = geometry
    u, v = spatial_frequencies(g.ny, g.nx, g.pixel_m)
    if coherence is None:
        x_coh, y_coh = coherence_lengths(g.sigma_x_px, g.sigma_y_px, g.pixel_m)
    else:
        x_coh, y_coh = float(coherence[0]), float(coherence[1])
    if iotf is None:
        win = iotf_window(u, v, x_coh, y_coh)
        gamma2 = regularization_window(u, v, x_coh, y_coh, gamma)
    else:
        win = np.asarray(iotf, np.float64)
        gamma2 = 1.0 - np.maximum(win, 0.0) ** (2.0 * gamma)
    return Problem(
        t=np.asarray(t, dtype=np.complex128),
        wavelength_m=g.wavelength_m, z1_m=g.z1_m, z2_m=g.z2_m, pixel_m=g.pixel_m,
        iotf=win,
        p_inv=preconditioning_filter(u, v, g.pixel_m, precond_scale),
        gamma2=gamma2,
        alpha=complex(alpha), eta=float(eta), u=u, v=v, precondition=precondition,
    )


# --------------------------------------------------------------------------- Eq. 1 as an operator
#
# Eq. 1 composes three stages.  The sample's transmission x = exp(psi) passes a
# linear map A (free-space propagation over L1, multiplication by the diffuser
# t, free-space propagation over L2); the squared modulus of the detector field
# is taken; the partially coherent source blurs it with the IPSF, a linear,
# real and self-adjoint operator B:
#     f(psi) = B |A exp(psi)|^2.
# The gradient of the loss of Eq. 2 is the chain rule through these stages:
# with J the Jacobian of f, the real gradient dL/dRe psi + i dL/dIm psi equals
# -2 J^T (y - f), and J^T is written out below from the adjoints of A and B.
# Algorithm S2 evaluates the same expression with the constant factors folded
# into its normalisation by max|t|^2.

FFT_WORKERS = -1  # scipy.fft threads (-1: all cores); the transform itself is unchanged


def fft2(a):
    """2-D DFT ``A_k = sum_r a_r exp(-2 pi i k.r / n)`` (library primitive)."""
    return _sfft.fft2(np.asarray(a, np.complex128), workers=FFT_WORKERS)


def ifft2(a):
    """Inverse 2-D DFT with the ``1/m`` normalisation (library primitive)."""
    return _sfft.ifft2(np.asarray(a, np.complex128), workers=FFT_WORKERS)


def filter_(x, w):
    """Fourier multiplier ``F^-1{ W_k F{x} }`` (the Filter primitive of Algorithm S2)."""
    return ifft2(fft2(x) * w)


def free_propagation(x, prob: Problem, distance_m: float):
    """Angular-spectrum propagation over ``distance_m`` (FreePropagation).

    The transfer function has unit modulus on propagating bins, so propagation
    over ``-L`` is the adjoint (and inverse) of propagation over ``L``."""
    return filter_(x, transfer_function(prob.u, prob.v, prob.wavelength_m, distance_m))


def detector_field(x, prob: Problem):
    """``A x = P_L2(t P_L1(x))``: the field at the detector for the sample transmission x."""
    return free_propagation(prob.t * free_propagation(x, prob, prob.z1_m), prob, prob.z2_m)


def detector_field_adjoint(w, prob: Problem):
    """``A^H w = P_L1^H(conj(t) P_L2^H(w))``, the adjoint of :func:`detector_field`."""
    return free_propagation(np.conj(prob.t) * free_propagation(w, prob, -prob.z2_m), prob, -prob.z1_m)


def source_blur(image, prob: Problem):
    """``B``: convolution of a real image with the IPSF of Eq. 4, applied as the IOTF window of Eq. 5.

    The window is real and even, so ``B`` maps real images to real images and is self-adjoint."""
    return np.real(filter_(image, prob.iotf))


def physical_model(psi, prob: Problem):
    """Eq. 1: ``f = B |A exp(psi)|^2``.  Returns ``f``, ``x = exp(psi)`` and ``v = A x``."""
    x = np.exp(psi)
    v = detector_field(x, prob)
    return source_blur(np.abs(v) ** 2, prob), x, v


def model_jvp(psi, dpsi, prob: Problem):
    """Directional derivative ``J dpsi`` of f at psi along a complex ``dpsi``.

    ``d exp(psi) = x dpsi``, ``dv = A(x dpsi)``, ``d|v|^2 = 2 Re(conj(v) dv)``, then ``B``."""
    _, x, v = physical_model(psi, prob)
    dv = detector_field(x * dpsi, prob)
    return source_blur(2.0 * np.real(np.conj(v) * dv), prob)


def model_vjp(x, v, w, prob: Problem):
    """``J^T w`` for a real image w: the complex image with ``Re<J^T w, dpsi> = sum_r w_r (J dpsi)_r``.

    Transposing the three stages of :func:`model_jvp` in reverse order gives
    ``J^T w = 2 conj(x) A^H(v B w)``."""
    return 2.0 * np.conj(x) * detector_field_adjoint(v * source_blur(w, prob), prob)


def loss(y, f) -> float:
    """Eq. 2: ``sum_r (y_r - f_r)^2``."""
    return float(np.sum((np.asarray(y, np.float64) - f) ** 2))


def wirtinger_derivative(e, x, v, prob: Problem):
    """The gradient ``g`` of Algorithm S2 for the misfit ``e = y - f``.

    The real gradient of Eq. 2 is ``-2 J^T e``; the paper's ``g`` leaves out
    the factor 4 (2 of the Wirtinger convention, 2 of the squared modulus) and
    divides by ``max|t|^2``, so ``g = -J^T e / (2 max|t|^2)``."""
    return -model_vjp(x, v, e, prob) / (2.0 * np.max(np.abs(prob.t) ** 2))


def preconditioner(g, prob: Problem):
    """Eqs. 6-11: the phase part ``Im g`` is smoothed by the inverse Laplacian ``P^-1``
    (a Fourier multiplier, 0 at DC); the attenuation part ``Re g`` is kept."""
    phase = np.imag(g)
    if prob.precondition:
        phase = np.real(filter_(phase, prob.p_inv))
    return np.real(g) + 1j * phase


def regularizer(psi, prob: Problem):
    """Real gradient of the Tikhonov term (Results, PWF subsection; Eqs. 14-15).

    ``R = Re(alpha)/2 ||Gamma Re psi||^2 + Im(alpha)/2 ||Gamma Im psi||^2`` with
    the real, even window ``Gamma^2 = 1 - STF`` has the gradient
    ``Re(alpha) Gamma^2 * Re psi + i Im(alpha) Gamma^2 * Im psi``."""
    attenuation = np.real(filter_(np.real(psi), prob.gamma2))
    phase = np.real(filter_(np.imag(psi), prob.gamma2))
    return prob.alpha.real * attenuation + 1j * prob.alpha.imag * phase


def gradient(psi, y, prob: Problem):
    """Loss, Wirtinger gradient ``g`` and update direction ``d`` at ``psi``."""
    f, x, v = physical_model(psi, prob)
    e = np.asarray(y, np.float64) - f
    g = wirtinger_derivative(e, x, v, prob)
    d = preconditioner(g, prob) + regularizer(psi, prob)
    return float(np.sum(e * e)), g, d


def nesterov_tau(tau: float) -> float:
    """Momentum scalar update of Algorithm S1: ``(1 + sqrt(1 + 4 tau^2)) / 2``."""
    return 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * tau * tau))


def field_correlation(psi_a, psi_b) -> float:
    """Normalised correlation ``|<x_a, x_b>| / (|x_a| |x_b|)`` of the fields ``x = exp(psi)``."""
    xa, xb = np.exp(psi_a), np.exp(psi_b)
    num = abs(np.vdot(xa, xb))
    return float(num / math.sqrt(np.vdot(xa, xa).real * np.vdot(xb, xb).real))


@dataclasses.dataclass
class PWFState:
    """Iterate of Algorithm S1: extrapolated ``psi``, gradient-step ``z``, momentum ``tau``."""

    psi: np.ndarray
    z: np.ndarray
    tau: float = 1.0
    k: int = 0


def initial_state(shape, psi0=None) -> PWFState:
    psi = np.zeros(shape, np.complex128) if psi0 is None else np.array(psi0, np.complex128)
    return PWFState(psi=psi, z=np.zeros(shape, np.complex128), tau=1.0, k=0)


def nesterov_update(psi, z_prev, tau_prev: float, d, eta: float):
    """Gradient step and Nesterov extrapolation of Algorithm S1.

    ``z = psi - eta d``; ``tau = (1 + sqrt(1 + 4 tau_prev^2)) / 2``;
    ``psi_new = z + ((tau_prev - 1) / tau) (z - z_prev)``.
    """
    z = psi - eta * d
    tau = nesterov_tau(tau_prev)
    return z, tau, z + ((tau_prev - 1.0) / tau) * (z - z_prev)


def pwf_step(state: PWFState, y, prob: Problem):
    """One iteration of Algorithm S1.  Returns (new state, loss at the entering ``psi``)."""
    l, g, d = gradient(state.psi, y, prob)
    if not math.isfinite(l):
        raise FloatingPointError("PWF loss is not finite")
    z, tau, psi = nesterov_update(state.psi, state.z, state.tau, d, prob.eta)
    return PWFState(psi=psi, z=z, tau=tau, k=state.k + 1), l


def pwf(y, prob: Problem, iters: int, corr_tol: float = 0.0, psi0=None, state: PWFState | None = None):
    """Algorithm S1: ``iters`` iterations (or fewer when the correlation stop is met).

    Returns ``(psi, loss_history, state)``.  With ``corr_tol > 0`` the loop stops
    after the first iteration whose new ``exp(psi)`` correlates with the
    previous one above ``corr_tol`` (the paper uses ``10^-0.00001``).
    """
    st = initial_state(prob.shape, psi0) if state is None else state
    hist = []
    for _ in range(iters):
        prev = st.psi
        st, l = pwf_step(st, y, prob)
        hist.append(l)
        if corr_tol > 0 and field_correlation(st.psi, prev) > corr_tol:
            break
    return st.psi, np.array(hist), st


# --------------------------------------------------------------------------- joint diffuser refinement
#
# Results ("Diffuser transmission function") and Fig. S12: the diffuser t can
# be retrieved together with the sample, as in ptychographic iterations, and
# since every projection angle shares it, t is updated continuously from all
# projections.  The paper states no update rule; the reading here:
#
# * the diffuser enters as u2 = t u1 with u1 = FreePropagation(x, L1), so the
#   Wirtinger derivative of the loss is dL/dt* = conj(u1) a2, where a2 is the
#   misfit back-propagated to the diffuser plane (the field that
#   WirtingerDerivative multiplies by conj(t));  the real gradient is 4 times
#   it, the same factor as for psi;
# * each iteration first takes the PWF step of every projection at the
#   current t, then a gradient step on t with the sum over projections,
#   normalised by sum_j max|u1_j|^2 (the analogue of the 1/max|t|^2 of the
#   sample gradient):  t <- t - eta_t sum_j conj(u1_j) a2_j / sum_j max|u1_j|^2;
# * eta_t = 1/2 (DEFAULT_ETA_T): on three 64^2 projections of the 128^2
#   generator with a 5%-perturbed diffuser, eta_t = 1 diverges within 30
#   iterations and 1/2 lowers the loss furthest.

DEFAULT_ETA_T = 0.5


def diffuser_gradient(e, x, v, prob: Problem):
    """``(conj(u1) a2, max|u1|^2)`` of one projection: the derivative of the loss
    with respect to ``t*`` and the normalisation of its step.

    t enters Eq. 1 through ``v = P_L2(t u1)``; the chain rule as in
    :func:`model_vjp` gives the real gradient ``-4 conj(u1) P_L2^H(v B e)``,
    i.e. 4 conj(u1) a2 with ``a2 = P_L2^H(v B(-e))``."""
    u1 = free_propagation(x, prob, prob.z1_m)
    a2 = -free_propagation(v * source_blur(e, prob), prob, -prob.z2_m)
    return np.conj(u1) * a2, float(np.max(np.abs(u1) ** 2))


def pwf_joint(ys, prob: Problem, iters: int, eta_t: float, psi0s=None):
    """Algorithm S1 on every projection in ``ys`` (shared geometry and diffuser
    ``prob.t``), with the diffuser step above after each iteration.

    Returns ``(psis, t, loss_history[j, k])``; the loss of projection j at
    iteration k is taken at its entering psi and the t of that iteration.
    """
    n = len(ys)
    states = [initial_state(prob.shape, None if psi0s is None else psi0s[j]) for j in range(n)]
    t = np.array(prob.t, np.complex128)
    hist = np.zeros((n, iters))
    for k in range(iters):
        pk = dataclasses.replace(prob, t=t)
        g_t = np.zeros_like(t)
        norm = 0.0
        for j in range(n):
            st = states[j]
            f, x, v = physical_model(st.psi, pk)
            e = np.asarray(ys[j], np.float64) - f
            hist[j, k] = float(np.sum(e * e))
            if not math.isfinite(hist[j, k]):
                raise FloatingPointError("PWF loss is not finite")
            g = wirtinger_derivative(e, x, v, pk)
            d = preconditioner(g, pk) + regularizer(st.psi, pk)
            z, tau, psi = nesterov_update(st.psi, st.z, st.tau, d, pk.eta)
            states[j] = PWFState(psi=psi, z=z, tau=tau, k=st.k + 1)
            gj, mj = diffuser_gradient(e, x, v, pk)
            g_t += gj
            norm += mj
        t = t - eta_t * g_t / norm
    return [s.psi for s in states], t, hist


# --------------------------------------------------------------------------- calibration front end
#
# Methods ("Intensity optical transfer function (IOTF)", Eq. 3) and Results
# ("Diffuser transmission function"): the coherence lengths come from the
# normalised autocorrelation of the reference speckle through the Siegert
# relation g2 = 1 + |g1|^2 and the Gaussian model g2 = 1 + exp(-pi dx^2 /
# x_coh^2), one axis at a time, averaged along the other axis; the diffuser
# is the reference speckle deconvolved by the IOTF (Wiener), square-rooted
# with zero phase and propagated back over L2.  Readings:
#
# * g2 is taken circularly (periodic images), g2(d) = <I(r) I(r + d)> / <I>^2;
# * the fit allows a contrast c (blurred or noisy speckle is not fully
#   developed): ln(g2(d) - 1) = ln c - pi d^2 p^2 / x_coh^2, least squares
#   over d = 1 .. K (K >= 2), K the last shift before g2 - 1 first drops
#   below FIT_FLOOR (g2(1) - 1); d = 0 carries the noise variance and is
#   left out;
# * Wiener filter IOTF / (IOTF^2 + eps) with eps given by the caller
#   (relative to IOTF(0) = 1); negative deconvolved intensities are clipped
#   to 0 before the square root.

FIT_FLOOR = 0.02


def speckle_g2(I, max_shift: int):
    """Normalised circular autocorrelations ``(g2_x[d], g2_y[d])``, d = 0 .. max_shift."""
    I = np.asarray(I, np.float64)
    m2 = np.mean(I) ** 2
    gx = np.array([np.mean(I * np.roll(I, -d, axis=1)) / m2 for d in range(max_shift + 1)])
    gy = np.array([np.mean(I * np.roll(I, -d, axis=0)) / m2 for d in range(max_shift + 1)])
    return gx, gy


def fit_coherence_length(g2, pixel_m: float):
    """``(x_coh, c)`` of the Gaussian model fitted to ``g2`` (see the readings above)."""
    s = np.asarray(g2, np.float64) - 1.0
    k = 1
    while k + 1 < len(s) and s[k + 1] >= FIT_FLOOR * s[1]:
        k += 1
    if k < 2:
        raise ValueError("autocorrelation too narrow to fit")
    d = np.arange(1, k + 1, dtype=np.float64)
    A = np.stack([np.ones_like(d), (d * pixel_m) ** 2], axis=1)
    coef, *_ = np.linalg.lstsq(A, np.log(s[1:k + 1]), rcond=None)
    return math.sqrt(-math.pi / coef[1]), math.exp(coef[0])


def wiener_deconvolve(I, iotf, eps: float):
    """``Re F^-1{ F{I} IOTF / (IOTF^2 + eps) }``."""
    return np.real(filter_(I, iotf / (iotf * iotf + eps)))


def diffuser_from_reference(I_ref, prob: Problem, eps: float):
    """Diffuser estimate: back-propagation over L2 of the zero-phase field
    ``sqrt(max(Wiener(I_ref), 0))``."""
    a = np.sqrt(np.maximum(wiener_deconvolve(I_ref, prob.iotf, eps), 0.0))
    return free_propagation(a, prob, -prob.z2_m)


# --------------------------------------------------------------------------- tomography
#
# Methods ("Reconstruction procedure"): filtered back-projection with the
# Ram-Lak filter applied slice by slice (every detector row is one parallel-
# beam sinogram over the angles in [0, pi)), then the constant lambda / (2 pi p)
# turns the reconstructed phase and attenuation into delta and beta.
# Readings:
#
# * the Ram-Lak filter is the band-limited ramp in the sample domain (unit
#   detector spacing): h(0) = 1/4, h(n odd) = -1/(pi^2 n^2), h(n even) = 0,
#   i.e. the inverse transform of |f| on |f| <= 1/2, applied by circular
#   convolution of rows zero-padded to n_pad = max(64, next power of two of
#   2 nx) (the padding of MATLAB's iradon);
# * geometry of the synthetic phantom: detector pixel i sees u = i + 1/2 -
#   nx/2 (voxel units); a sample point (X, Z) of a slice projects at
#   u = X cos(theta) - Z sin(theta); reconstruction voxel centres X, Z =
#   k + 1/2 - N/2; back-projection interpolates linearly in u and treats
#   samples outside the detector as 0;
# * f(X, Z) = (pi / P) sum_j q_j(u_j(X, Z)) for P equally spaced angles;
# * psi = -mu + i phi is reconstructed as one complex sinogram (the filter is
#   real): delta = Im(f) lambda / (2 pi p), beta = -Re(f) lambda / (2 pi p);
# * the quadratic background fit is a separate step (background_quadratic).


def fbp_pad_length(nx: int) -> int:
    return max(64, 1 << int(math.ceil(math.log2(2 * nx))))


def ramp_kernel(n_pad: int) -> np.ndarray:
    """Band-limited ramp h(n) on a circular grid of ``n_pad`` samples."""
    n = np.arange(n_pad)
    n = np.where(n <= n_pad // 2, n, n - n_pad)
    h = np.zeros(n_pad)
    h[n == 0] = 0.25
    odd = (n % 2) != 0
    h[odd] = -1.0 / (math.pi ** 2 * n[odd].astype(np.float64) ** 2)
    return h


def fbp_filter(sino, n_pad: int | None = None) -> np.ndarray:
    """Rows of ``sino`` [P, nx] convolved with the ramp (zero-padded, circular)."""
    sino = np.asarray(sino)
    p, nx = sino.shape
    n_pad = fbp_pad_length(nx) if n_pad is None else n_pad
    pad = np.zeros((p, n_pad), np.complex128)
    pad[:, :nx] = sino
    H = np.real(np.fft.fft(ramp_kernel(n_pad)))
    return np.fft.ifft(np.fft.fft(pad, axis=1) * H[None, :], axis=1)[:, :nx]


def backproject(q, angles, n_out: int) -> np.ndarray:
    """``(pi / P) sum_j q_j(X cos theta_j - Z sin theta_j)`` on the n_out x n_out grid [Z, X]."""
    q = np.asarray(q)
    p, nx = q.shape
    c = np.arange(n_out) + 0.5 - n_out / 2.0
    X = c[None, :]
    Z = c[:, None]
    out = np.zeros((n_out, n_out), np.complex128)
    for j, th in enumerate(angles):
        idx = X * math.cos(th) - Z * math.sin(th) + nx / 2.0 - 0.5
        i0 = np.floor(idx).astype(np.int64)
        w = idx - i0
        lo = np.where((i0 >= 0) & (i0 < nx), q[j][np.clip(i0, 0, nx - 1)], 0.0)
        hi = np.where((i0 + 1 >= 0) & (i0 + 1 < nx), q[j][np.clip(i0 + 1, 0, nx - 1)], 0.0)
        out += (1.0 - w) * lo + w * hi
    return out * (math.pi / p)


def fbp_slice(sino, angles, n_out: int) -> np.ndarray:
    return backproject(fbp_filter(sino), angles, n_out)


def fbp_volume(psis, angles, n_out: int, rows=None) -> np.ndarray:
    """Slices ``rows`` (default all) of the tomogram of the projections ``psis``: [row, Z, X]."""
    psis = [np.asarray(p) for p in psis]
    ny = psis[0].shape[0]
    rows = range(ny) if rows is None else rows
    return np.stack([fbp_slice(np.stack([p[y] for p in psis]), angles, n_out) for y in rows])


def refractive_index(vol, wavelength_m: float, pixel_m: float):
    """``(delta, beta)`` of a tomogram of psi = -mu + i phi."""
    c = wavelength_m / (2.0 * math.pi * pixel_m)
    return np.imag(vol) * c, -np.real(vol) * c


# --------------------------------------------------------------------------- background removal
#
# Methods ("Reconstruction procedure"): phase-gradient sensing recovers slow
# phase variations poorly, so each reconstructed slice carries a smooth
# background, removed after tomography by a quadratic surface fit.  Readings:
# the fit is per slice, by least squares over the voxels whose centre lies at
# a distance >= r_bg (voxels) from the rotation axis, the sample being inside
# that radius; the surface is b = c0 + c1 x + c2 z + c3 x^2 + c4 x z + c5 z^2
# in the voxel-centre coordinates divided by N/2; real and imaginary parts are
# fitted separately and the surface is subtracted from the whole slice.


def background_basis(n: int) -> np.ndarray:
    """The six quadratic monomials on the n x n voxel-centre grid, [6, Z, X]."""
    c = (np.arange(n) + 0.5 - n / 2.0) / (n / 2.0)
    x = np.broadcast_to(c[None, :], (n, n))
    z = np.broadcast_to(c[:, None], (n, n))
    return np.stack([np.ones((n, n)), x, z, x * x, x * z, z * z])


def background_mask(n: int, r_bg: float) -> np.ndarray:
    c = np.arange(n) + 0.5 - n / 2.0
    return np.hypot(c[None, :], c[:, None]) >= r_bg


def background_quadratic(vol, r_bg: float):
    """Slices of ``vol`` [slice, Z, X] minus their fitted quadratic backgrounds,
    and the coefficients [slice, part (re, im), 6]."""
    vol = np.asarray(vol)
    n = vol.shape[-1]
    basis = background_basis(n)
    mask = background_mask(n, r_bg)
    a = basis[:, mask].T
    if a.shape[0] < 6 or np.linalg.matrix_rank(a) < 6:
        raise ValueError("too few background voxels for a quadratic fit")
    out = np.empty(vol.shape, np.complex128)
    coef = np.empty((vol.shape[0], 2, 6))
    for s, sl in enumerate(vol):
        coef[s, 0] = np.linalg.lstsq(a, sl.real[mask], rcond=None)[0]
        coef[s, 1] = np.linalg.lstsq(a, sl.imag[mask], rcond=None)[0]
        bg = np.tensordot(coef[s, 0], basis, 1) + 1j * np.tensordot(coef[s, 1], basis, 1)
        out[s] = sl - bg
    return out, coef


# --------------------------------------------------------------------------- diagnostics
#
# Methods ("Reconstruction procedure"): the RMSE image of one measurement is
# |y - f(x)| normalised by the mean intensity of the reference speckle, in
# percent.  Methods ("Fourier shell correlation", Eq. 16): the normalised
# cross-correlation of two tomograms' transforms over shells |k| = kappa; the
# paper's resolution criterion is FSC = 1/4 (its Eqs. 17-18).  Readings: the
# shells are integer bins of |k| in frequency-index units, kappa =
# round(sqrt(kx^2 + ky^2 + kz^2)) with signed indices of a cubic grid, up to
# n/2; the numerator is the real part of the shell sum (exact for real
# volumes); FRC is the same on square images.


def rmse_image(y, psi, prob: Problem, ref_mean: float):
    f, _, _ = physical_model(psi, prob)
    return 100.0 * np.abs(np.asarray(y, np.float64) - f) / ref_mean


def shell_correlation(g1, g2):
    """FSC (3-D) or FRC (2-D) of two real arrays on a cubic / square grid, shells 0..n/2."""
    g1 = np.asarray(g1, np.float64)
    g2 = np.asarray(g2, np.float64)
    n = g1.shape[0]
    G1 = np.fft.fftn(g1)
    G2 = np.fft.fftn(g2)
    k = np.fft.fftfreq(n) * n
    grids = np.meshgrid(*([k] * g1.ndim), indexing="ij")
    shell = np.rint(np.sqrt(sum(g * g for g in grids))).astype(np.int64)
    nsh = n // 2 + 1
    keep = shell < nsh
    num = np.bincount(shell[keep], np.real(np.conj(G1) * G2)[keep], nsh)
    a = np.bincount(shell[keep], (np.abs(G1) ** 2)[keep], nsh)
    b = np.bincount(shell[keep], (np.abs(G2) ** 2)[keep], nsh)
    return num / np.sqrt(a * b)


def resolution_from_fsc(fsc, n: int, pixel_m: float, criterion: float = 0.25):
    """Length ``n p / kappa`` at the first shell (from 1) where the FSC falls below ``criterion``."""
    for kappa in range(1, len(fsc)):
        if fsc[kappa] < criterion:
            return n * pixel_m / kappa
    return 2.0 * pixel_m
