"""Parity at the workloads' full sizes and launch configurations, on sampled outputs.

* 180 projections x 1024^2 in one batched, graph-captured solve of 100 iterations (the
  configuration bench.py times): projections 0 and 90 against the oracle, projection 0
  bit for bit against its unbatched solve.
* 64 uneven ROIs (24 x 512^2, 32 x 1024^2, 8 x 2048^2) in one batch of 100 iterations:
  one instance per size class against the oracle and bit for bit against its unbatched
  solve.
* The correlation stop of the Methods section against the oracle's.
"""

import numpy as np
import pytest

import oracle as O
import synthetic as S
from gpu_helpers import (device, fd_check, gpu_problem, instance, loss_history_tolerance, loss_tolerance, rel,
                         say, to_dev)

pytestmark = pytest.mark.gpu

PHASE_TOL = 1e-3


def _rms(a, b):
    return float(np.sqrt(np.mean(np.abs(np.asarray(a) - np.asarray(b)) ** 2)))


def test_tomographic_batch_180x1024_in_bench_configuration():
    import torch
    from paper_2503_20146_amd import PWF, problem_from_geometry
    dev = device()
    n_proj, iters, checked = 180, 100, (0, 90)
    say("workload 180 x 1024^2: generating projections")
    d = S.tomo_projection_inputs(2, range(n_proj))
    geo = d["geometry"]
    t = torch.from_numpy(d["t"]).to(dev)
    probs = [problem_from_geometry(geo, t) for _ in range(n_proj)]
    batch = PWF(probs)
    # measured speckle: oracle forward for the checked projections, GPU forward elsewhere
    psi_true = [torch.from_numpy(p.astype(np.complex64)).to(dev) for p in d["psi_true"]]
    f = batch.forward(psi_true)
    oprob = O.make_problem(d["t"], geo)
    ys = []
    for j in range(n_proj):
        if j in checked:
            fj, _, _ = O.physical_model(d["psi_true"][j], oprob)
        else:
            fj = f[j].cpu().numpy()
        ys.append(to_dev(S.poisson_intensity(fj, d["seed_keys"][j]), dev))
    del f, psi_true
    say("workload 180 x 1024^2: batched solve, 100 iterations")
    out, hist = batch.solve(ys, iters)
    torch.cuda.synchronize()
    psi90 = out[90].cpu().numpy()
    psi0 = out[0].clone()
    h90 = hist[90].cpu().numpy()
    h0 = hist[0].cpu().numpy()
    del out
    say("workload 180 x 1024^2: projection 0 unbatched")
    one, _ = PWF([probs[0]]).solve([ys[0]], iters)
    assert torch.equal(one[0], psi0)
    for j, psi_j, h_j in ((90, psi90, h90), (0, psi0.cpu().numpy(), h0)):
        say(f"workload 180 x 1024^2: oracle on projection {j}")
        yj = ys[j].cpu().numpy()
        psi_ref, hist_ref, _ = O.pwf(yj, oprob, iters)
        assert _rms(psi_j.imag, psi_ref.imag) <= PHASE_TOL, j
        assert _rms(psi_j.real, psi_ref.real) <= PHASE_TOL, j
        assert np.all(np.abs(h_j - hist_ref) / hist_ref <= loss_history_tolerance(yj, hist_ref)), j


def test_uneven_roi_batch_64_instances():
    """The 64 distinct ROI instances in one batch, 100 iterations: the first 512^2 and
    1024^2 instances against the oracle, the first of every class bit for bit against
    its unbatched solve (the 2048^2 one is checked against the oracle below)."""
    import torch
    from paper_2503_20146_amd import PWF
    dev = device()
    iters = 100
    specs = S.roi_batch_specs()
    say("uneven ROI batch: generating 64 instances")
    probs, psis, keep = [], [], {}
    oracle_checked, first = (0, 24), (0, 24, 56)
    for i, (side, sigma) in enumerate(specs):
        inp = S.instance_inputs(3, side, instance=i, sigma_px=sigma)
        probs.append(gpu_problem(inp["geometry"], inp["t"], dev))
        psis.append(inp)
    # noise-free speckle: the oracle's for the instances checked against it, the GPU's elsewhere
    f_gpu = PWF(probs).forward([to_dev(inp["psi_true"].astype(np.complex64), dev) for inp in psis])
    ys = []
    for i, inp in enumerate(psis):
        if i in oracle_checked:
            prob = O.make_problem(inp["t"], inp["geometry"])
            f, _, _ = O.physical_model(inp["psi_true"], prob)
        else:
            f = f_gpu[i].cpu().numpy()
        y = S.poisson_intensity(f, inp["seed_key"])
        ys.append(to_dev(y, dev))
        if i in oracle_checked:
            keep[i] = (prob, y)
    del f_gpu
    say("uneven ROI batch: batched solve, 100 iterations")
    out, hist = PWF(probs).solve(ys, iters)
    torch.cuda.synchronize()
    for i in first:
        say(f"uneven ROI batch: instance {i} ({specs[i][0]}^2) unbatched")
        one, h1 = PWF([probs[i]]).solve([ys[i]], iters)
        assert torch.equal(one[0], out[i]), i
        assert torch.equal(h1[0], hist[i]), i
    for i, (prob, y) in keep.items():
        say(f"uneven ROI batch: instance {i} ({specs[i][0]}^2) against the oracle")
        psi_ref, hist_ref, _ = O.pwf(y, prob, iters)
        psi = out[i].cpu().numpy()
        assert _rms(psi.imag, psi_ref.imag) <= PHASE_TOL, i
        assert _rms(psi.real, psi_ref.real) <= PHASE_TOL, i
        assert np.all(np.abs(hist[i].cpu().numpy() - hist_ref) / hist_ref <= loss_history_tolerance(y, hist_ref)), i


def test_uneven_merged_launch_equals_per_class():
    """One launch per sweep over the 512^2, 1024^2 and 2048^2 classes equals the classes
    launched separately on parallel streams, bit for bit, eagerly and in graph replays
    (with eager work and synchronisations between the replays)."""
    import torch
    from paper_2503_20146_amd import PWF, set_graph_mode, set_merged_launch
    dev = device()
    say("merged vs per-class launches: 2 x 512^2 + 2 x 1024^2 + 1 x 2048^2")
    specs = S.roi_batch_specs()
    pick = [0, 1, 24, 25, 56]
    probs, ys = [], []
    for i in pick:
        side, sigma = specs[i]
        inp = S.instance_inputs(3, side, instance=i, sigma_px=sigma)
        probs.append(gpu_problem(inp["geometry"], inp["t"], dev))
        ys.append(to_dev(S.poisson_intensity(np.clip(1.0 + 0.1 * inp["psi_true"].imag, 0, None), inp["seed_key"]),
                         dev))
    batch = PWF(probs)
    try:
        set_merged_launch(False)
        ref, href = batch.solve(ys, 8)
        ref = [r.clone() for r in ref]
        set_merged_launch(True)
        assert batch.lib.pwf_version() >= 10100
        set_graph_mode(False)
        eager, he = batch.solve(ys, 8)
        set_graph_mode(True)
        for i in range(len(pick)):
            assert torch.equal(eager[i], ref[i]), i
            assert torch.equal(he[i], href[i]), i
        for _ in range(3):
            g, hg = batch.solve(ys, 8)
            torch.cuda.synchronize()
            _ = batch.forward(g)
            torch.cuda.synchronize()
            for i in range(len(pick)):
                assert torch.equal(g[i], ref[i]), i
                assert torch.equal(hg[i], href[i]), i
    finally:
        set_graph_mode(True)
        set_merged_launch(False)


def test_uneven_roi_2048_instance_100_iterations():
    """The first 2048^2 ROI instance (instance 56, its own sigma) for 100 iterations
    against the oracle; the batch test above shows its batched solve equals this one."""
    from paper_2503_20146_amd import PWF
    dev = device()
    side, sigma = S.roi_batch_specs()[56]
    inp = S.instance_inputs(3, side, instance=56, sigma_px=sigma)
    prob = O.make_problem(inp["t"], inp["geometry"])
    f, _, _ = O.physical_model(inp["psi_true"], prob)
    y = S.poisson_intensity(f, inp["seed_key"])
    say("uneven ROI 2048^2 instance: solve, 100 iterations")
    out, hist = PWF([gpu_problem(inp["geometry"], inp["t"], dev)]).solve([to_dev(y, dev)], 100)
    say("uneven ROI 2048^2 instance: oracle")
    psi_ref, hist_ref, _ = O.pwf(y, prob, 100)
    psi = out[0].cpu().numpy()
    assert _rms(psi.imag, psi_ref.imag) <= PHASE_TOL
    assert _rms(psi.real, psi_ref.real) <= PHASE_TOL
    assert np.all(np.abs(hist[0].cpu().numpy() - hist_ref) / hist_ref <= loss_history_tolerance(y, hist_ref))


def _workload_720x2048(dev, scale_psi: float):
    """The 720 x 2048^2 workload at its full size: projections of the 2048^3 phantom made on
    the device, speckle from the GPU forward model with device Poisson noise; projection 0
    replaced by the CPU recipe's psi and speckle (the oracle's inputs).  Returns the batch,
    psi [720, 2048, 2048] at scale_psi * psi_true, the speckles and projection 0's inputs."""
    import torch
    from paper_2503_20146_amd import PWF, problem_from_geometry
    n, side = 720, 2048
    torch.cuda.empty_cache()
    d = S.tomo_projection_inputs(4, [0])
    geo = d["geometry"]
    prob = O.make_problem(d["t"], geo)
    t = to_dev(d["t"], dev)
    psi = torch.empty((n, side, side), dtype=torch.complex64, device=dev)
    S.project_ellipsoids_device(S.ellipsoid_phantom(side, 40, (S.BASE_SEED + 2,), 2.0),
                                [np.pi * j / n for j in range(n)], side, side, geo.pixel_m, geo.wavelength_m, psi)
    batch = PWF([problem_from_geometry(geo, t) for _ in range(n)])
    ys = batch.forward([psi[j] for j in range(n)])
    for j in range(1, n):
        gen = torch.Generator(device=dev)
        gen.manual_seed(S.BASE_SEED + 4 + j)
        ys[j] = torch.poisson(ys[j].clamp(min=0.0) * 1.0e4, generator=gen).div_(1.0e4)
    f0, _, _ = O.physical_model(d["psi_true"][0], prob)
    y0 = S.poisson_intensity(f0, d["seed_keys"][0])
    ys[0] = to_dev(y0, dev)
    p0 = (scale_psi * d["psi_true"][0]).astype(np.complex64)
    psi.mul_(scale_psi)
    psi[0].copy_(to_dev(p0, dev))
    return batch, psi, ys, prob, y0, p0, t, geo


def test_differentiable_720x2048_full_size():
    """PWFLoss (forward: model and misfit; backward: forward fields recomputed) over all
    720 projections of 2048^2 at psi = 0.9 psi_true: projection 0's gradient against the
    oracle's and central differences of the FP64 loss on 16 pixels, and bit for bit against
    the same projection differentiated alone."""
    import torch
    from paper_2503_20146_amd import PWF, problem_from_geometry, pwf_loss
    dev = device()
    say("720 x 2048^2: generating the workload")
    batch, psi, ys, prob, y0, p0, t, geo = _workload_720x2048(dev, 0.9)
    say("720 x 2048^2: PWFLoss forward + backward over 720 projections")
    p = psi.requires_grad_(True)
    loss = pwf_loss(p, batch, ys)
    loss.sum().backward()
    assert bool(torch.isfinite(loss).all()) and bool(torch.isfinite(p.grad).all())
    grad0 = p.grad[0].cpu().numpy()
    l0 = float(loss[0].detach())
    del batch, loss, ys[1:]
    p.grad = None
    torch.cuda.empty_cache()
    say("720 x 2048^2: projection 0 alone")
    p1 = to_dev(p0[None], dev).requires_grad_(True)
    one = PWF([problem_from_geometry(geo, t)])
    l1 = pwf_loss(p1, one, [ys[0]])
    l1.sum().backward()
    assert torch.equal(p1.grad[0].cpu(), torch.from_numpy(grad0)) and float(l1[0].detach()) == l0
    say("720 x 2048^2: oracle gradient of projection 0")
    l_ref, g_ref, _ = O.gradient(p0.astype(np.complex128), y0, prob)
    f_ref, _, _ = O.physical_model(p0.astype(np.complex128), prob)
    assert abs(l0 - l_ref) <= loss_tolerance(y0, f_ref) * l_ref
    r = rel(grad0, 4 * np.max(np.abs(prob.t) ** 2) * g_ref)
    say(f"720 x 2048^2: gradient rel-L2 {r:.2e}")
    assert r <= 1e-4
    say("720 x 2048^2: central differences on 16 pixels")
    rng = np.random.default_rng(720)
    pix = [tuple(int(v) for v in divmod(int(k), 2048)) for k in rng.choice(2048 * 2048, 16, replace=False)]
    fd_check(p0, y0, prob, grad0, pix)


def test_solve_720x2048_full_size():
    """pwf_solve over all 720 projections of 2048^2, 20 iterations in one graph: projection 0
    against the oracle's trajectory."""
    import torch
    dev = device()
    say("720 x 2048^2: generating the workload")
    batch, psi, ys, prob, y0, p0, t, geo = _workload_720x2048(dev, 1.0)
    iters = 20
    say("720 x 2048^2: solve, 20 iterations")
    out, hist = batch.solve(ys, iters, psi_out=[psi[j] for j in range(720)])
    torch.cuda.synchronize()
    assert batch.sync_status() == 0
    psi0 = psi[0].cpu().numpy()
    h0 = hist[0].cpu().numpy()
    del batch, ys, out, hist, psi
    torch.cuda.empty_cache()
    say("720 x 2048^2: oracle on projection 0")
    psi_ref, hist_ref, _ = O.pwf(y0, prob, iters)
    assert _rms(psi0.imag, psi_ref.imag) <= PHASE_TOL
    assert _rms(psi0.real, psi_ref.real) <= PHASE_TOL
    assert np.all(np.abs(h0 - hist_ref) / hist_ref <= loss_history_tolerance(y0, hist_ref))


# On the 128^2 workload 1 - correlation runs 1.0e-4, 1.5e-5, 5.9e-6, ... 9.9e-7 (10th
# iteration), ... 6.0e-7 (17th): the paper's threshold stops after 2 iterations, the
# others after 10 and 17, each with a clear margin to the neighbouring iterations.
@pytest.mark.parametrize("tol", [O.PAPER_STOP_CORR, 1.0 - 1e-6, 1.0 - 6e-7])
def test_correlation_stop_matches_oracle(tol):
    from paper_2503_20146_amd import PWF
    dev = device()
    inp, geo, prob, y = instance(0)
    say(f"correlation stop {tol}")
    psi_ref, hist_ref, st = O.pwf(y, prob, 400, corr_tol=tol)
    k_ref = len(hist_ref)
    batch = PWF([gpu_problem(geo, inp["t"], dev)])
    out, hist, done = batch.solve([to_dev(y, dev)], 400, corr_tol=tol, return_iters=True)
    assert 1 <= k_ref < 400
    assert done[0] == k_ref, (done[0], k_ref)
    assert _rms(out[0].cpu().numpy(), psi_ref) <= PHASE_TOL
    assert np.all(np.abs(hist[0, :k_ref].cpu().numpy() - hist_ref) / hist_ref <= loss_history_tolerance(y, hist_ref))


# At 512^2 (split column transform; the stopping-rule S0 variant on paired rows)
# 1 - correlation runs 8.3e-6, 3.8e-6, 2.1e-6, 1.5e-6, 1.2e-6, 9.7e-7, ...: thresholds
# between neighbours with margins of 1e-7 and more.
@pytest.mark.parametrize("tol", [1.0 - 3e-6, 1.0 - 1.3e-6])
def test_correlation_stop_matches_oracle_512(tol):
    from paper_2503_20146_amd import PWF
    dev = device()
    inp, geo, prob, y = instance(0, n=512)
    say(f"correlation stop {tol} at 512^2")
    psi_ref, hist_ref, st = O.pwf(y, prob, 60, corr_tol=tol)
    k_ref = len(hist_ref)
    batch = PWF([gpu_problem(geo, inp["t"], dev)])
    out, hist, done = batch.solve([to_dev(y, dev)], 60, corr_tol=tol, return_iters=True)
    assert 1 <= k_ref < 60
    assert done[0] == k_ref, (done[0], k_ref)
    assert _rms(out[0].cpu().numpy(), psi_ref) <= PHASE_TOL
    assert np.all(np.abs(hist[0, :k_ref].cpu().numpy() - hist_ref) / hist_ref <= loss_history_tolerance(y, hist_ref))


def test_correlation_stop_per_instance_in_a_batch():
    """Instances stop independently; stopped ones keep their iterate while others run."""
    import torch
    from paper_2503_20146_amd import PWF
    dev = device()
    say("correlation stop, batch of 3")
    items = [instance(0, instance=i) for i in range(3)]
    probs = [gpu_problem(x[1], x[0]["t"], dev) for x in items]
    ys = [to_dev(x[3], dev) for x in items]
    tol = 1.0 - 6e-7
    out, hist, done = PWF(probs).solve(ys, 300, corr_tol=tol, return_iters=True)
    for i in range(3):
        one, _, d1 = PWF([probs[i]]).solve([ys[i]], 300, corr_tol=tol, return_iters=True)
        assert d1[0] == done[i]
        assert torch.equal(one[0], out[i])
