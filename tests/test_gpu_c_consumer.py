"""The library without PyTorch: a plain C99 program (tests/c_consumer/pwf_c_solve.c,
built by __graft_entry__.build()) allocates with the HIP runtime, runs pwf_solve on the
128^2 workload for 50 iterations and writes the field and the loss history.  They must
match the FP64 oracle to the solve's tolerances and the Python binding's solve of the same
problem bit for bit (same kernels, same launch schedule)."""

import os
import subprocess

import numpy as np
import pytest

import oracle as O
from gpu_helpers import device, gpu_problem, instance, loss_history_tolerance, say, to_dev

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BINARY = os.path.join(ROOT, "tests", "c_consumer", "pwf_c_solve")
ITERS = 50
PHASE_TOL = 1e-3


def test_c_program_solve_matches_oracle_and_binding(tmp_path):
    if not os.path.exists(BINARY):
        pytest.skip("the C consumer is not built (__graft_entry__.build() builds it)")
    from paper_2503_20146_amd import PWF
    dev = device()
    inp, geo, prob, y = instance(0)
    p = gpu_problem(geo, inp["t"], dev)
    params = [geo.nx, geo.ny, geo.pixel_m, geo.wavelength_m, geo.z1_m, geo.z2_m, p.sigma_x_px, p.sigma_y_px,
              p.eta, p.alpha.real, p.alpha.imag, p.gamma, p.precond_scale, ITERS]
    (tmp_path / "params.txt").write_text(" ".join(repr(float(v)) if isinstance(v, float) else str(v)
                                                  for v in params) + "\n")
    np.ascontiguousarray(y, np.float32).tofile(tmp_path / "y.f32")
    np.ascontiguousarray(inp["t"], np.complex64).tofile(tmp_path / "t.c64")
    say("C consumer: pwf_solve on 128^2, 50 iterations")
    res = subprocess.run([BINARY, str(tmp_path / "params.txt"), str(tmp_path / "y.f32"), str(tmp_path / "t.c64"),
                          str(tmp_path / "psi.c64"), str(tmp_path / "loss.f64")],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    psi_c = np.fromfile(tmp_path / "psi.c64", np.complex64).reshape(geo.ny, geo.nx)
    loss_c = np.fromfile(tmp_path / "loss.f64", np.float64)
    assert loss_c.shape == (ITERS,)

    psi_ref, hist_ref, _ = O.pwf(y, prob, ITERS)
    assert np.sqrt(np.mean((psi_c.imag - psi_ref.imag) ** 2)) <= PHASE_TOL
    assert np.sqrt(np.mean((psi_c.real - psi_ref.real) ** 2)) <= PHASE_TOL
    assert np.all(np.abs(loss_c - hist_ref) / hist_ref <= loss_history_tolerance(y, hist_ref))

    out, hist = PWF([p]).solve([to_dev(y, dev)], ITERS)
    assert np.array_equal(out[0].cpu().numpy(), psi_c)
    assert np.array_equal(hist[0].cpu().numpy(), loss_c)
