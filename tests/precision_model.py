"""How FP32 rounding of the gradient reaches the update direction (test aid).

d = Preconditioner(g) + Regularizer(psi) applies P^-1 = s_P / rho^2 (Eq. 11
reading; rho in cycles/pixel) to the phase part of g.  P^-1 reaches s_P n^2 at
the lowest frequency, so a small error of g that is spread evenly over
frequencies reaches d amplified by

    A = (||P^-1 delta|| / ||delta||) / (||d|| / ||g||)

for white delta in Im g: the preconditioner's RMS gain on white noise over its
gain on this gradient.  A depends on n and on how g's energy is distributed
over frequencies, so it is computed per input.  Two FP32 models of the direction
are evaluated with the FP64 oracle: g rounded to complex64 and then
preconditioned in FP64 (storage rounding only), and the same with the forward
transform of g taken in single precision (the transform that the fused
direction sweep does in FP32 before applying P^-1).
"""

from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

import oracle as O


def white_gain(prob, rng, trials: int = 4) -> float:
    """RMS gain of the preconditioner's phase part on white noise: ||P^-1 delta|| / ||delta||."""
    gains = []
    for _ in range(trials):
        delta = rng.standard_normal(prob.shape)
        out = O.preconditioner(1j * delta, prob).imag
        gains.append(np.linalg.norm(out) / np.linalg.norm(delta))
    return float(np.mean(gains))


def amplification(g, d, prob, rng) -> float:
    """A of the module docstring for the gradient g and direction d of one input."""
    return white_gain(prob, rng) * float(np.linalg.norm(g) / np.linalg.norm(d))


def fp32_direction_errors(psi, g, d, prob) -> dict:
    """Relative L2 errors of d when g is stored in FP32, and when in addition the
    forward transform of g's phase part runs in single precision."""
    reg = O.regularizer(psi, prob)
    g32 = np.asarray(g, np.complex64).astype(np.complex128)
    d_store = O.preconditioner(g32, prob) + reg
    spec32 = sfft.fft2(np.imag(g32).astype(np.complex64)).astype(np.complex128)
    phase = np.real(O.ifft2(spec32 * prob.p_inv)) if prob.precondition else np.imag(g32)
    d_fft = (np.real(g32) + 1j * phase) + reg
    rel = lambda a: float(np.linalg.norm(a - d) / np.linalg.norm(d))
    return {"storage": rel(d_store), "storage+fft32": rel(d_fft)}


def cases():
    """The three inputs of the GPU direction test: 128^2 and 1024^2 single-projection
    workloads and projection 0 of the 720 x 2048^2 workload, at psi = psi_true / 2."""
    import synthetic as S
    for w in (0, 1):
        inp = S.instance_inputs(w)
        prob = O.make_problem(inp["t"], inp["geometry"])
        f, _, _ = O.physical_model(inp["psi_true"], prob)
        y = S.poisson_intensity(f, inp["seed_key"])
        yield f"{inp['geometry'].nx}^2", prob, (0.5 * inp["psi_true"]).astype(np.complex64), y
    d = S.tomo_projection_inputs(4, [0])
    prob = O.make_problem(d["t"], d["geometry"])
    f, _, _ = O.physical_model(d["psi_true"][0], prob)
    y = S.poisson_intensity(f, d["seed_keys"][0])
    yield "2048^2", prob, (0.5 * d["psi_true"][0]).astype(np.complex64), y


def main() -> None:
    rng = np.random.default_rng(0)
    print(f"{'case':>8} {'white gain':>11} {'||d||/||g||':>12} {'A':>8} {'storage':>10} {'fft32':>10}")
    for label, prob, psi, y in cases():
        psi64 = psi.astype(np.complex128)
        _, g, d = O.gradient(psi64, y, prob)
        wg = white_gain(prob, rng)
        ratio = float(np.linalg.norm(d) / np.linalg.norm(g))
        e = fp32_direction_errors(psi64, g, d, prob)
        print(f"{label:>8} {wg:11.2f} {ratio:12.4f} {wg / ratio:8.2f} {e['storage']:10.3e} {e['storage+fft32']:10.3e}",
              flush=True)


if __name__ == "__main__":
    main()
