"""Shared helpers of the GPU parity tests (inputs from ``synthetic``, expected values from ``oracle``)."""

import sys

import numpy as np
import pytest

import oracle as O
import synthetic as S


def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_20146_amd import _lib
    _lib.load()  # fails loudly when the HIP library is missing
    return torch.device("cuda:0")


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def instance(workload=0, n=None, instance=None, sigma=None, geometry=None):
    """(inputs, oracle problem, noisy y float32) for a single-projection instance."""
    inp = S.instance_inputs(workload, n, instance, sigma)
    geo = inp["geometry"] if geometry is None else geometry
    prob = O.make_problem(inp["t"], geo)
    f, _, _ = O.physical_model(inp["psi_true"], prob)
    y = S.poisson_intensity(f, inp["seed_key"])
    return inp, geo, prob, y


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def gpu_problem(geo, t, dev, **kw):
    from paper_2503_20146_amd import problem_from_geometry
    return problem_from_geometry(geo, to_dev(np.asarray(t, np.complex64), dev), **kw)


def loss_tolerance(y, f_ref, fwd_tol=1e-5):
    """Relative tolerance of L = sum (y - f)^2 implied by the forward tolerance on f:
    |dL| <= 2 ||y - f|| ||df||, so |dL|/L <= 2 fwd_tol ||f|| / ||y - f||."""
    y = np.asarray(y, np.float64)
    return 2.0 * fwd_tol * float(np.linalg.norm(f_ref) / np.linalg.norm(y - f_ref))


def loss_history_tolerance(y, hist_ref, fwd_tol=1e-5):
    """Per-iteration relative tolerance of a loss history: ||y - f_k|| = sqrt(L_k), so the
    forward tolerance gives |dL_k| / L_k <= 2 fwd_tol ||y|| / sqrt(L_k) (||f_k|| ~ ||y||)."""
    y = np.asarray(y, np.float64)
    return 2.0 * fwd_tol * float(np.linalg.norm(y)) / np.sqrt(np.asarray(hist_ref, np.float64))


def fd_check(psi, y, prob, grad, pixels, h=1e-4, rtol=1e-3, grad_tol=1e-4):
    """Central differences of the FP64 oracle loss against a GPU gradient at the listed pixels.

    Allowed deviation: rtol of the difference quotient (its O(h^2) truncation and FP64
    cancellation) plus a floor of 5 grad_tol RMS(grad), five times the per-pixel RMS error
    that the relative-L2 budget of the gradient allows: FP32 rounding of the GPU gradient
    is spread evenly over pixels, so small entries carry errors of that absolute size.
    """
    psi = np.asarray(psi).astype(np.complex128)
    floor = 5 * grad_tol * float(np.sqrt(np.mean(np.abs(grad) ** 2)))
    for (r, c) in pixels:
        for unit in (1.0, 1j):
            dp = np.zeros(psi.shape, complex)
            dp[r, c] = h * unit
            lp = O.loss(y, O.physical_model(psi + dp, prob)[0])
            lm = O.loss(y, O.physical_model(psi - dp, prob)[0])
            fd = (lp - lm) / (2 * h)
            an = grad[r, c].real if unit == 1.0 else grad[r, c].imag
            assert abs(fd - an) <= rtol * abs(fd) + floor, (r, c, unit, fd, an)
