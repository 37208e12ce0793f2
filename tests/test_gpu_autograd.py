"""Differentiation through torch.autograd with recomputed forward fields.

The gradient convention is torch's for a real loss of a complex input:
dL/dRe psi + i dL/dIm psi, which equals 4 max|t|^2 g for the paper's g.
Pinned against central differences (h = 1e-4) of the FP64 oracle loss, and
against the oracle's Wirtinger derivative, at 128^2 and at the 2048^2
projection size of the 720-projection workload.
"""

import numpy as np
import pytest

import oracle as O
import synthetic as S
from gpu_helpers import device, fd_check, gpu_problem, instance, loss_tolerance, rel, say, to_dev

pytestmark = pytest.mark.gpu


GRAD_TOL = 1e-4


def _fd_check(psi, y, prob, grad, pixels, h=1e-4, rtol=1e-3):
    fd_check(psi, y, prob, grad, pixels, h, rtol, GRAD_TOL)


def test_autograd_small_matches_oracle_and_fd():
    import torch
    from paper_2503_20146_amd import PWF, pwf_loss
    dev = device()
    inp, geo, prob, y = instance(0)
    say("autograd 128^2")
    psi = (0.5 * inp["psi_true"]).astype(np.complex64)
    batch = PWF([gpu_problem(geo, inp["t"], dev)])
    p = to_dev(psi[None], dev).requires_grad_(True)
    loss = pwf_loss(p, batch, [to_dev(y, dev)])
    loss.sum().backward()
    grad = p.grad[0].cpu().numpy()
    l_ref, g_ref, _ = O.gradient(psi.astype(np.complex128), y, prob)
    assert abs(float(loss[0].detach()) - l_ref) <= 1e-5 * l_ref
    assert rel(grad, 4 * np.max(np.abs(prob.t) ** 2) * g_ref) <= GRAD_TOL
    rng = np.random.default_rng(11)
    pix = [tuple(int(v) for v in divmod(int(k), 128)) for k in rng.choice(128 * 128, 8, replace=False)]
    _fd_check(psi, y, prob, grad, pix)


def test_autograd_chain_rule_with_weights():
    """Upstream gradients scale each instance's contribution."""
    import torch
    from paper_2503_20146_amd import PWF, pwf_loss
    dev = device()
    say("autograd weights")
    items = [instance(0, instance=i) for i in range(2)]
    batch = PWF([gpu_problem(x[1], x[0]["t"], dev) for x in items])
    psi = np.stack([(0.5 * x[0]["psi_true"]).astype(np.complex64) for x in items])
    ys = [to_dev(x[3], dev) for x in items]
    p = to_dev(psi, dev).requires_grad_(True)
    loss = pwf_loss(p, batch, ys)
    (3.0 * loss[0] - 0.5 * loss[1]).backward()
    for i, w in enumerate((3.0, -0.5)):
        _, g_ref, _ = O.gradient(psi[i].astype(np.complex128), items[i][3], items[i][2])
        expect = w * 4 * np.max(np.abs(items[i][2].t) ** 2) * g_ref
        assert rel(p.grad[i].cpu().numpy(), expect) <= GRAD_TOL


def test_autograd_2048_projection_fd_and_oracle():
    """2048^2 projections of the 2048^3 phantom (four in the batch): FD on 16 pixels of one."""
    import torch
    from paper_2503_20146_amd import PWF, problem_from_geometry, pwf_loss
    dev = device()
    say("autograd 2048^2: generating 4 projections")
    d = S.tomo_projection_inputs(4, [0, 180, 360, 540])
    geo = d["geometry"]
    prob = O.make_problem(d["t"], geo)
    t = torch.from_numpy(d["t"]).to(dev)
    batch = PWF([problem_from_geometry(geo, t) for _ in range(4)])
    ys, psis = [], []
    for j in range(4):
        f, _, _ = O.physical_model(d["psi_true"][j], prob)
        ys.append(to_dev(S.poisson_intensity(f, d["seed_keys"][j]), dev))
        psis.append((0.9 * d["psi_true"][j]).astype(np.complex64))
    p = to_dev(np.stack(psis), dev).requires_grad_(True)
    say("autograd 2048^2: forward + backward")
    loss = pwf_loss(p, batch, ys)
    loss.sum().backward()
    grad0 = p.grad[0].cpu().numpy()
    say("autograd 2048^2: oracle gradient")
    y0 = ys[0].cpu().numpy()
    l_ref, g_ref, _ = O.gradient(psis[0].astype(np.complex128), y0, prob)
    f_ref, _, _ = O.physical_model(psis[0].astype(np.complex128), prob)
    assert abs(float(loss[0].detach()) - l_ref) <= loss_tolerance(y0, f_ref) * l_ref
    r = rel(grad0, 4 * np.max(np.abs(prob.t) ** 2) * g_ref)
    say(f"autograd 2048^2: gradient rel-L2 {r:.2e}")
    assert r <= GRAD_TOL
    say("autograd 2048^2: central differences on 16 pixels")
    rng = np.random.default_rng(2048)
    pix = [tuple(int(v) for v in divmod(int(k), 2048)) for k in rng.choice(2048 * 2048, 16, replace=False)]
    _fd_check(psis[0], y0, prob, grad0, pix)
