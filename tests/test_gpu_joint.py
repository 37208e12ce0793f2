"""Joint diffuser refinement on the GPU (pwf_solve_joint) against the oracle.

The diffuser step sums conj(u1_j) a2_j over every instance in FP64; the
instances then run the ordinary PWF sweeps.  Parity: each psi within the
phase tolerance, the diffuser change t - t0 within relative L2 1e-3 (FP32
gradients carry ~1e-4 and the step compounds over the iterations), and the
loss history within the derived loss tolerance.  A zero step reproduces
pwf_solve bit for bit.
"""

import dataclasses

import numpy as np
import pytest

import oracle as O
import synthetic as S
from gpu_helpers import device, loss_history_tolerance, rel, say, to_dev

pytestmark = pytest.mark.gpu

PHASE_TOL = 1e-3
DT_TOL = 1e-3


def _perturbed_batch(n, size=None, workload=0):
    base = S.instance_inputs(workload, size)
    geo = base["geometry"]
    prob = O.make_problem(base["t"], geo)
    ys = []
    for i in range(n):
        d = S.instance_inputs(workload, size, instance=i)
        f, _, _ = O.physical_model(d["psi_true"], prob)
        ys.append(S.poisson_intensity(f, d["seed_key"]))
    rng = np.random.default_rng(3)
    t0 = (prob.t * (1.0 + 0.05 * rng.standard_normal(prob.t.shape))).astype(np.complex64)
    return geo, prob, ys, t0


def _gpu_batch(geo, t_dev, n):
    from paper_2503_20146_amd import PWF, problem_from_geometry
    return PWF([problem_from_geometry(geo, t_dev) for _ in range(n)])


def _check(out, hist, t_gpu, t0, psis_ref, t_ref, hist_ref, ys):
    for j, psi_ref in enumerate(psis_ref):
        psi = out[j].cpu().numpy()
        assert np.sqrt(np.mean(np.abs(psi - psi_ref) ** 2)) <= PHASE_TOL, j
        assert np.all(np.abs(hist[j].cpu().numpy() - hist_ref[j]) / hist_ref[j]
                      <= loss_history_tolerance(ys[j], hist_ref[j])), j
    dt_ref = t_ref - t0.astype(np.complex128)
    dt = t_gpu.astype(np.complex128) - t0.astype(np.complex128)
    assert rel(dt, dt_ref) <= DT_TOL


def test_joint_matches_oracle_128():
    dev = device()
    geo, prob, ys, t0 = _perturbed_batch(4)
    say("joint refinement 4 x 128^2, 20 iterations")
    t_dev = to_dev(t0, dev)
    batch = _gpu_batch(geo, t_dev, 4)
    out, hist = batch.solve_joint([to_dev(y, dev) for y in ys], 20, eta_t=O.DEFAULT_ETA_T)
    t_gpu = t_dev.cpu().numpy()
    psis_ref, t_ref, hist_ref = O.pwf_joint(ys, dataclasses.replace(prob, t=t0.astype(np.complex128)), 20,
                                            O.DEFAULT_ETA_T)
    _check(out, hist, t_gpu, t0, psis_ref, t_ref, hist_ref, ys)


def test_joint_zero_step_equals_solve():
    import torch
    dev = device()
    geo, prob, ys, t0 = _perturbed_batch(3)
    say("joint refinement with eta_t = 0")
    t_dev = to_dev(t0, dev)
    batch = _gpu_batch(geo, t_dev, 3)
    yd = [to_dev(y, dev) for y in ys]
    out_j, hist_j = batch.solve_joint(yd, 10, eta_t=0.0)
    out_s, hist_s = batch.solve(yd, 10)
    assert np.array_equal(t_dev.cpu().numpy(), t0)
    for j in range(3):
        assert torch.equal(out_j[j], out_s[j])
    assert torch.equal(hist_j, hist_s)


def test_joint_rejects_distinct_diffusers():
    from paper_2503_20146_amd import PWF, problem_from_geometry
    dev = device()
    geo, prob, ys, t0 = _perturbed_batch(2)
    batch = PWF([problem_from_geometry(geo, to_dev(t0, dev)), problem_from_geometry(geo, to_dev(t0, dev))])
    with pytest.raises(ValueError):
        batch.solve_joint([to_dev(y, dev) for y in ys], 2)


def test_joint_16_projections_1024():
    """16 projections of the 180 x 1024^2 workload's phantom with a perturbed
    shared diffuser, 3 joint iterations, in the bench's launch configuration."""
    dev = device()
    say("joint refinement 16 x 1024^2: generating projections")
    d = S.tomo_projection_inputs(2, [11 * j for j in range(16)])
    geo = d["geometry"]
    prob = O.make_problem(d["t"], geo)
    ys = []
    for j in range(16):
        f, _, _ = O.physical_model(d["psi_true"][j], prob)
        ys.append(S.poisson_intensity(f, d["seed_keys"][j]))
    rng = np.random.default_rng(5)
    t0 = (prob.t * (1.0 + 0.05 * rng.standard_normal(prob.t.shape))).astype(np.complex64)
    t_dev = to_dev(t0, dev)
    batch = _gpu_batch(geo, t_dev, 16)
    say("joint refinement 16 x 1024^2: GPU")
    out, hist = batch.solve_joint([to_dev(y, dev) for y in ys], 3)
    t_gpu = t_dev.cpu().numpy()
    say("joint refinement 16 x 1024^2: oracle")
    psis_ref, t_ref, hist_ref = O.pwf_joint(ys, dataclasses.replace(prob, t=t0.astype(np.complex128)), 3,
                                            O.DEFAULT_ETA_T)
    _check(out, hist, t_gpu, t0, psis_ref, t_ref, hist_ref, ys)
