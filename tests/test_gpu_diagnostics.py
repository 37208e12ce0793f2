"""RMSE image on the GPU (pwf_rmse_image) against the oracle: the forward
model's FP32 tolerance (relative L2 1e-5 on f) carried to |y - f| through the
misfit's size, at the 128^2 truth (pure noise) and at a 1024^2 iterate."""

import numpy as np
import pytest

import oracle as O
from gpu_helpers import device, gpu_problem, instance, rel, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("workload,frac", [(0, 1.0), (1, 0.5)])
def test_rmse_image_matches_oracle(workload, frac):
    from paper_2503_20146_amd import PWF
    dev = device()
    inp, geo, prob, y = instance(workload)
    psi = (frac * inp["psi_true"]).astype(np.complex64)
    ref_mean = 1.0 + 0.01 * workload
    say(f"rmse image workload {workload}")
    img = PWF([gpu_problem(geo, inp["t"], dev)]).rmse_image([to_dev(psi, dev)], [to_dev(y, dev)], [ref_mean])
    ref = O.rmse_image(y, psi.astype(np.complex128), prob, ref_mean)
    f, _, _ = O.physical_model(psi.astype(np.complex128), prob)
    # |d|y - f|| <= |df| pointwise, so ||img - ref|| <= 100 / ref_mean * 1e-5 ||f||
    assert np.linalg.norm(img[0].cpu().numpy() - ref) <= 100.0 / ref_mean * 1e-5 * np.linalg.norm(f)
    assert rel(img[0].cpu().numpy(), ref) <= 1e-5 * np.linalg.norm(f) / np.linalg.norm(y - f)


@pytest.mark.parametrize("n,dims", [(128, 3), (256, 2), (512, 2), (2048, 2)])
def test_shell_correlation_matches_oracle(n, dims):
    """FP32 transforms against FP64: the shell correlations agree to 1e-5; the
    shell sums run in a fixed order, so a second call gives the same bits (2048:
    two waves per workgroup instead of four)."""
    import torch
    from paper_2503_20146_amd import shell_correlation
    dev = device()
    rng = np.random.default_rng(n + dims)
    shape = (n,) * dims
    s = rng.standard_normal(shape)
    a = (s + 0.7 * rng.standard_normal(shape)) + 1j * rng.standard_normal(shape)
    b = (s + 0.7 * rng.standard_normal(shape)) + 1j * rng.standard_normal(shape)
    say(f"shell correlation {n}^{dims}")
    ta, tb = to_dev(a.astype(np.complex64), dev), to_dev(b.astype(np.complex64), dev)
    got = np.array(shell_correlation(ta, tb, part=0))
    ref = O.shell_correlation(a.real.astype(np.float32), b.real.astype(np.float32))
    assert np.max(np.abs(got - ref)) <= 1e-5
    again = np.array(shell_correlation(ta, tb, part=0))
    assert np.array_equal(got, again)
    same = np.array(shell_correlation(ta, ta, part=1))
    assert np.max(np.abs(same[1:] - 1.0)) <= 1e-6


@pytest.mark.parametrize("scale", [1e-6, 1e3])
def test_shell_correlation_is_scale_invariant(scale):
    """The correlation does not change when one input is scaled (Eq. 16 is invariant under
    positive scaling of either input): the two fields share one complex transform, so the
    library brings both to unit RMS first; without that, a 1e-6 scale cost 1e-2 here."""
    from paper_2503_20146_amd import shell_correlation
    dev = device()
    rng = np.random.default_rng(77)
    shape = (128,) * 3
    s = rng.standard_normal(shape)
    a = (s + 0.7 * rng.standard_normal(shape)) + 1j * rng.standard_normal(shape)
    b = (s + 0.7 * rng.standard_normal(shape)) + 1j * rng.standard_normal(shape)
    say(f"shell correlation, second input scaled by {scale:g}")
    got = np.array(shell_correlation(to_dev(a.astype(np.complex64), dev),
                                     to_dev((scale * b).astype(np.complex64), dev), part=0))
    ref = O.shell_correlation(a.real.astype(np.float32), b.real.astype(np.float32))
    assert np.max(np.abs(got - ref)) <= 1e-5
