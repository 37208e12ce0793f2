"""Pins of the oracle's joint diffuser refinement (Results, "Diffuser
transmission function"; Fig. S12), independent of its own formulas:
central differences of the FP64 loss in t, the invariance of the loss under a
constant phase on t, descent of the t step, the noise-free truth point, and
the reduction to independent PWF when the diffuser step is zero."""

import dataclasses

import numpy as np
import pytest

import oracle as O
import synthetic as S


def _shared_batch(n=3, size=64):
    """``n`` projections of the 128^2 generator (cropped to ``size``) sharing one diffuser."""
    base = S.instance_inputs(0, size)
    prob = O.make_problem(base["t"], base["geometry"])
    ys, psis = [], []
    for i in range(n):
        d = S.instance_inputs(0, size, instance=i)
        f, _, _ = O.physical_model(d["psi_true"], prob)
        ys.append(S.poisson_intensity(f, d["seed_key"]))
        psis.append(d["psi_true"])
    return prob, ys, psis


def _loss_at(psi, y, prob, t):
    f, _, _ = O.physical_model(psi, dataclasses.replace(prob, t=t))
    return O.loss(y, f)


def test_diffuser_gradient_matches_central_differences():
    prob, ys, psis = _shared_batch(1)
    psi = 0.7 * psis[0]
    f, x, v = O.physical_model(psi, prob)
    g, _ = O.diffuser_gradient(np.asarray(ys[0], np.float64) - f, x, v, prob)
    rng = np.random.default_rng(7)
    h = 1e-5
    scale = np.max(np.abs(g))
    for k in rng.choice(prob.t.size, 6, replace=False):
        r, c = divmod(int(k), prob.t.shape[1])
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            dt = np.zeros_like(prob.t)
            dt[r, c] = h * unit
            fd = (_loss_at(psi, ys[0], prob, prob.t + dt) - _loss_at(psi, ys[0], prob, prob.t - dt)) / (2 * h)
            assert abs(fd - 4.0 * part(g[r, c])) <= 1e-6 * max(abs(fd), scale), (r, c, unit, fd, g[r, c])


def test_diffuser_gradient_orthogonal_to_constant_phase():
    """L(t e^{i theta}) = L(t), so sum_r Im(t_r conj(G_r)) = 0."""
    prob, ys, psis = _shared_batch(1)
    f, x, v = O.physical_model(0.5 * psis[0], prob)
    g, _ = O.diffuser_gradient(np.asarray(ys[0], np.float64) - f, x, v, prob)
    s = np.sum(prob.t * np.conj(g))
    assert abs(s.imag) <= 1e-12 * np.sum(np.abs(prob.t) * np.abs(g))
    assert abs(s.real) > 1e-6 * np.sum(np.abs(prob.t) * np.abs(g))   # the pin is not vacuous


def test_diffuser_gradient_zero_at_noise_free_truth():
    prob, _, psis = _shared_batch(1)
    f, x, v = O.physical_model(psis[0], prob)
    g, m = O.diffuser_gradient(np.zeros_like(f), x, v, prob)
    assert np.max(np.abs(g)) == 0.0 and m > 0.5


def test_diffuser_step_descends():
    prob, ys, psis = _shared_batch(3)
    psi = [0.8 * p for p in psis]
    g_t = np.zeros_like(prob.t)
    norm = 0.0
    for j in range(3):
        f, x, v = O.physical_model(psi[j], prob)
        g, m = O.diffuser_gradient(np.asarray(ys[j], np.float64) - f, x, v, prob)
        g_t += g
        norm += m
    before = sum(_loss_at(psi[j], ys[j], prob, prob.t) for j in range(3))
    after = sum(_loss_at(psi[j], ys[j], prob, prob.t - 0.05 * g_t / norm) for j in range(3))
    assert after < before


def test_joint_with_zero_step_is_independent_pwf():
    prob, ys, _ = _shared_batch(2)
    psis, t, hist = O.pwf_joint(ys, prob, 5, 0.0)
    assert np.array_equal(t, prob.t)
    for j in range(2):
        psi_ref, hist_ref, _ = O.pwf(ys[j], prob, 5)
        assert np.array_equal(psis[j], psi_ref)
        assert np.array_equal(hist[j], hist_ref)


def test_joint_refinement_lowers_the_loss_of_a_perturbed_diffuser():
    """Starting from a diffuser with a 5% amplitude error, 30 joint iterations
    at the default diffuser step end below the total loss of PWF with the wrong
    diffuser held fixed (and above that with the true diffuser)."""
    prob, ys, _ = _shared_batch(3)
    rng = np.random.default_rng(3)
    t_bad = prob.t * (1.0 + 0.05 * rng.standard_normal(prob.t.shape))
    bad = dataclasses.replace(prob, t=t_bad)
    _, _, hist = O.pwf_joint(ys, bad, 30, O.DEFAULT_ETA_T)
    fixed = sum(O.pwf(y, bad, 30)[1][-1] for y in ys)
    true = sum(O.pwf(y, prob, 30)[1][-1] for y in ys)
    assert true < hist[:, -1].sum() < fixed
