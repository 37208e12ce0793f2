"""pwf_loss_grad_noalloc (workspace in the library's static buffer) against pwf_loss_grad.

Both are called through the C ABI on the same inputs; the kernels are the same, so the
loss and the gradient must agree bit for bit.  Two calls in a row, the second with a
smaller batch, show that the buffer's leftover contents do not leak into a result.
"""

import ctypes

import numpy as np
import pytest

import synthetic as S
from gpu_helpers import device, gpu_problem, say, to_dev

pytestmark = pytest.mark.gpu


def _batch(specs, dev, seed):
    from paper_2503_20146_amd import PWF
    probs, psis, ys = [], [], []
    for k, (n, sig) in enumerate(specs):
        rng = np.random.default_rng(seed + k)
        geo = S.Geometry(ny=n, nx=n, sigma_x_px=sig, sigma_y_px=sig)
        t = S.diffuser(rng, n, n)
        psi_true = S.phase_object(rng, n, n, 4.0, 2.0)
        p = gpu_problem(geo, t, dev)
        probs.append(p)
        psis.append(to_dev((0.6 * psi_true).astype(np.complex64), dev))
        ys.append(to_dev(rng.uniform(0.7, 1.1, (n, n)).astype(np.float32), dev))
    return PWF(probs), psis, ys


def test_noalloc_loss_grad_equals_workspace_version():
    import torch
    from paper_2503_20146_amd import _lib
    dev = device()
    lib = _lib.load()
    limit = lib.pwf_loss_grad_noalloc_limit()
    say(f"noalloc: limit {limit} bytes")
    assert limit == (64 - 1) << 20
    for label, specs, seed in (("1024 + 2 x 256", [(1024, 1.5), (256, 0.8), (256, 1.2)], 40),
                               ("one 512", [(512, 1.0)], 50)):
        say(f"noalloc: {label}")
        batch, psis, ys = _batch(specs, dev, seed)
        loss_ws, grad_ws = batch.loss_grad(psis, ys)
        loss_na, grad_na = batch.loss_grad_noalloc(psis, ys)
        torch.cuda.synchronize()
        assert torch.equal(loss_ws, loss_na), label
        for a, b in zip(grad_ws, grad_na):
            assert torch.equal(a, b), label
        assert torch.all(torch.isfinite(loss_na))


def test_noalloc_rejects_batches_beyond_the_buffer():
    from paper_2503_20146_amd import PWF, PwfError, _lib
    dev = device()
    say("noalloc: oversized batch is refused before any work")
    batch, psis, ys = _batch([(1024, 1.5), (1024, 1.5)], dev, 60)
    with pytest.raises(PwfError) as err:
        batch.loss_grad_noalloc(psis, ys)
    assert err.value.status == _lib.PWF_ERR_SCRATCH
