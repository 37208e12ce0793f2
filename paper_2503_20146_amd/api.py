"""Torch-facing wrappers of the libpwf C ABI.

Argument marshalling only: tensors are passed to the library as device
pointers on the current HIP stream; every step of the method runs in the
library's kernels.  Torch provides device memory and streams.
"""

from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Sequence

import torch

from . import _lib
from ._lib import check

DEFAULT_ETA = 0.5
DEFAULT_ALPHA = complex(0.1, 0.01)
DEFAULT_GAMMA = 1.0
DEFAULT_PRECOND_SCALE = 1.0 / (4.0 * math.pi ** 2)
DEFAULT_ETA_T = 0.5  # diffuser step of the joint refinement (pwf_solve_joint)


@dataclasses.dataclass
class Problem:
    """One PWF instance (projection or region of interest).

    The source's partial coherence is given by ``sigma_x_px``/``sigma_y_px`` (Gaussian
    IPSF in pixels), or by ``x_coh_m``/``y_coh_m`` (coherence lengths in metres, e.g.
    from :func:`calibrate_source`), or by a separable IOTF ``iotf_x``/``iotf_y`` (float32
    GPU tensors of nx and ny values on the DFT bins); the first of these that is set,
    in the order IOTF, coherence lengths, sigma, is passed to the library."""

    nx: int
    ny: int
    pixel_m: float
    wavelength_m: float
    z1_m: float
    z2_m: float
    sigma_x_px: float
    sigma_y_px: float
    diffuser: torch.Tensor            # complex64 [ny, nx] on the GPU
    eta: float = DEFAULT_ETA
    alpha: complex = DEFAULT_ALPHA
    gamma: float = DEFAULT_GAMMA
    precond_scale: float = DEFAULT_PRECOND_SCALE
    precondition: bool = True
    x_coh_m: float | None = None
    y_coh_m: float | None = None
    iotf_x: torch.Tensor | None = None
    iotf_y: torch.Tensor | None = None

    def _source(self) -> _lib.pwf_source:
        src = _lib.pwf_source()
        if self.iotf_x is not None or self.iotf_y is not None:
            for t, n in ((self.iotf_x, self.nx), (self.iotf_y, self.ny)):
                if (t is None or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous()
                        or tuple(t.shape) != (n,)):
                    raise ValueError("iotf_x / iotf_y must be contiguous float32 GPU tensors of nx / ny values")
            src.kind = _lib.PWF_SRC_IOTF
            src.iotf_x = self.iotf_x.data_ptr()
            src.iotf_y = self.iotf_y.data_ptr()
        elif self.x_coh_m is not None or self.y_coh_m is not None:
            src.kind = _lib.PWF_SRC_COHERENCE
            src.x_coh_m = float(self.x_coh_m or 0.0)
            src.y_coh_m = float(self.y_coh_m or 0.0)
        else:
            src.kind = _lib.PWF_SRC_GAUSS
            src.sigma_x_px = float(self.sigma_x_px)
            src.sigma_y_px = float(self.sigma_y_px)
        return src

    def to_c(self) -> _lib.pwf_problem:
        d = self.diffuser
        if d.dtype != torch.complex64 or not d.is_contiguous() or tuple(d.shape) != (self.ny, self.nx):
            raise ValueError("diffuser must be a contiguous complex64 tensor of shape (ny, nx)")
        p = _lib.pwf_problem()
        p.geom = _lib.pwf_geometry(self.nx, self.ny, self.pixel_m, self.wavelength_m, self.z1_m, self.z2_m)
        p.source = self._source()
        p.params = _lib.pwf_params(self.eta, self.alpha.real, self.alpha.imag, self.gamma, self.precond_scale,
                                   1 if self.precondition else 0)
        p.diffuser = d.data_ptr()
        return p


def problem_from_geometry(geometry, diffuser: torch.Tensor, **kw) -> Problem:
    """Build a Problem from any object with nx, ny, pixel_m, wavelength_m, z1_m, z2_m, sigma_*_px."""
    g = geometry
    return Problem(nx=g.nx, ny=g.ny, pixel_m=g.pixel_m, wavelength_m=g.wavelength_m, z1_m=g.z1_m, z2_m=g.z2_m,
                   sigma_x_px=g.sigma_x_px, sigma_y_px=g.sigma_y_px, diffuser=diffuser, **kw)


def _ptrs(tensors, dtype=None, shape=None) -> ctypes.Array:
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        if t is None:
            arr[i] = None
            continue
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("buffers must be contiguous GPU tensors")
        if dtype is not None and t.dtype != dtype:
            raise ValueError(f"expected {dtype}, got {t.dtype}")
        if shape is not None and tuple(t.shape) != tuple(shape[i]):
            raise ValueError(f"expected shape {shape[i]}, got {tuple(t.shape)}")
        arr[i] = t.data_ptr()
    return arr


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class PWF:
    """A batch of PWF instances with its workspace."""

    def __init__(self, problems: Sequence[Problem]):
        if not problems:
            raise ValueError("need at least one problem")
        self.lib = _lib.load()
        self.problems = list(problems)
        self.n = len(self.problems)
        self.device = self.problems[0].diffuser.device
        self._c = (_lib.pwf_problem * self.n)(*[p.to_c() for p in self.problems])
        size = self.lib.pwf_workspace_size(self._c, self.n)
        if size == 0:
            raise ValueError("invalid problem description (see pwf_workspace_size)")
        self.workspace = torch.empty(size, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace is not 256-byte aligned")
        self.shapes = [(p.ny, p.nx) for p in self.problems]

    # -- helpers
    def _ws(self):
        return ctypes.c_void_p(self.workspace.data_ptr()), ctypes.c_size_t(self.workspace.numel())

    def _empty(self, dtype):
        return [torch.empty(s, dtype=dtype, device=self.device) for s in self.shapes]

    # -- entry points
    def forward(self, psi: Sequence[torch.Tensor], out: Sequence[torch.Tensor] | None = None):
        out = self._empty(torch.float32) if out is None else list(out)
        ws, nb = self._ws()
        check(self.lib.pwf_forward(self._c, self.n, _ptrs(psi, torch.complex64, self.shapes),
                                   _ptrs(out, torch.float32, self.shapes), ws, nb, _stream(self.device)),
              "pwf_forward")
        return out

    def rmse_image(self, psi: Sequence[torch.Tensor], y: Sequence[torch.Tensor], ref_mean: Sequence[float]):
        """RMSE images 100 |y - f(psi)| / ref_mean (pwf_rmse_image)."""
        out = self._empty(torch.float32)
        ws, nb = self._ws()
        means = (ctypes.c_double * self.n)(*[float(m) for m in ref_mean])
        check(self.lib.pwf_rmse_image(self._c, self.n, _ptrs(psi, torch.complex64, self.shapes),
                                      _ptrs(y, torch.float32, self.shapes), means,
                                      _ptrs(out, torch.float32, self.shapes), ws, nb, _stream(self.device)),
              "pwf_rmse_image")
        return out

    def gradient(self, psi, y, want_g: bool = True, want_d: bool = True):
        g = self._empty(torch.complex64) if want_g else None
        d = self._empty(torch.complex64) if want_d else None
        loss = torch.empty(self.n, dtype=torch.float64, device=self.device)
        ws, nb = self._ws()
        check(self.lib.pwf_gradient(self._c, self.n, _ptrs(psi, torch.complex64, self.shapes),
                                    _ptrs(y, torch.float32, self.shapes),
                                    _ptrs(g, torch.complex64, self.shapes) if g else None,
                                    _ptrs(d, torch.complex64, self.shapes) if d else None,
                                    ctypes.c_void_p(loss.data_ptr()), ws, nb, _stream(self.device)),
              "pwf_gradient")
        return loss, g, d

    def init_states(self, y, psi0=None):
        states = []
        arr = (_lib.pwf_state * self.n)()
        for i, s in enumerate(self.shapes):
            st = {k: torch.empty(s, dtype=torch.complex64, device=self.device)
                  for k in ("psi", "psi_hat", "z_hat", "y_hat")}
            st["k"] = 0
            states.append(st)
            arr[i] = _lib.pwf_state(st["psi"].data_ptr(), st["psi_hat"].data_ptr(), st["z_hat"].data_ptr(),
                                    st["y_hat"].data_ptr(), 0)
        ws, nb = self._ws()
        p0 = _ptrs(psi0, torch.complex64, self.shapes) if psi0 is not None else None
        check(self.lib.pwf_state_init(self._c, self.n, arr, p0, _ptrs(y, torch.float32, self.shapes), ws, nb,
                                      _stream(self.device)), "pwf_state_init")
        return states

    def step(self, states):
        arr = (_lib.pwf_state * self.n)()
        for i, st in enumerate(states):
            arr[i] = _lib.pwf_state(st["psi"].data_ptr(), st["psi_hat"].data_ptr(), st["z_hat"].data_ptr(),
                                    st["y_hat"].data_ptr(), st["k"])
        loss = torch.empty(self.n, dtype=torch.float64, device=self.device)
        ws, nb = self._ws()
        check(self.lib.pwf_step(self._c, self.n, arr, ctypes.c_void_p(loss.data_ptr()), ws, nb,
                                _stream(self.device)), "pwf_step")
        for i, st in enumerate(states):
            st["k"] = arr[i].k
        return loss

    def solve(self, y, iters: int, psi_out=None, loss_hist: bool = True, corr_tol: float = 0.0,
              return_iters: bool = False, hist_out: torch.Tensor | None = None):
        """Algorithm S1 from psi = 0.  ``corr_tol`` in (0, 1) enables the correlation stop.
        ``hist_out`` (float64 [n, iters] on the GPU) receives the loss history in place of a
        new tensor."""
        psi_out = self._empty(torch.complex64) if psi_out is None else list(psi_out)
        if hist_out is not None:
            if hist_out.dtype != torch.float64 or not hist_out.is_contiguous() or hist_out.numel() < self.n * iters:
                raise ValueError("hist_out must be a contiguous float64 tensor of n * iters values")
            hist = hist_out
        else:
            hist = (torch.empty((self.n, max(iters, 1)), dtype=torch.float64, device=self.device)
                    if loss_hist else None)
        done = (ctypes.c_int32 * self.n)()
        ws, nb = self._ws()
        check(self.lib.pwf_solve(self._c, self.n, _ptrs(y, torch.float32, self.shapes),
                                 _ptrs(psi_out, torch.complex64, self.shapes), iters, float(corr_tol),
                                 ctypes.c_void_p(hist.data_ptr()) if hist is not None else None, done, ws, nb,
                                 _stream(self.device)), "pwf_solve")
        if return_iters:
            return psi_out, hist, [done[i] for i in range(self.n)]
        return psi_out, hist

    def solve_joint(self, y, iters: int, eta_t: float = DEFAULT_ETA_T, psi_out=None, loss_hist: bool = True):
        """Joint diffuser refinement: Algorithm S1 on every instance plus a diffuser
        step per iteration (pwf_solve_joint).  All instances must share one diffuser
        tensor, which is updated in place."""
        d0 = self.problems[0].diffuser
        if any(p.diffuser.data_ptr() != d0.data_ptr() for p in self.problems):
            raise ValueError("joint refinement needs one diffuser tensor shared by every instance")
        size = self.lib.pwf_joint_workspace_size(self._c, self.n)
        if size == 0:
            raise ValueError("invalid problem description")
        if self.workspace.numel() < size:
            self.workspace = torch.empty(size, dtype=torch.uint8, device=self.device)
        psi_out = self._empty(torch.complex64) if psi_out is None else list(psi_out)
        hist = torch.empty((self.n, max(iters, 1)), dtype=torch.float64, device=self.device) if loss_hist else None
        ws, nb = self._ws()
        check(self.lib.pwf_solve_joint(self._c, self.n, _ptrs(y, torch.float32, self.shapes),
                                       _ptrs(psi_out, torch.complex64, self.shapes), iters, float(eta_t),
                                       ctypes.c_void_p(hist.data_ptr()) if hist is not None else None, ws, nb,
                                       _stream(self.device)), "pwf_solve_joint")
        return psi_out, hist

    def loss_grad(self, psi, y, grad_out=None):
        """Loss and real gradient dL/dRe psi + i dL/dIm psi (forward fields recomputed)."""
        grad = self._empty(torch.complex64) if grad_out is None else list(grad_out)
        loss = torch.empty(self.n, dtype=torch.float64, device=self.device)
        ws, nb = self._ws()
        check(self.lib.pwf_loss_grad(self._c, self.n, _ptrs(psi, torch.complex64, self.shapes),
                                     _ptrs(y, torch.float32, self.shapes), _ptrs(grad, torch.complex64, self.shapes),
                                     ctypes.c_void_p(loss.data_ptr()), ws, nb, _stream(self.device)),
              "pwf_loss_grad")
        return loss, grad

    def loss_grad_noalloc(self, psi, y, grad_out=None, loss_out=None):
        """pwf_loss_grad on the library's static buffer (pwf_loss_grad_noalloc): no
        workspace is used and, with ``grad_out`` and ``loss_out`` given, nothing is
        allocated."""
        grad = self._empty(torch.complex64) if grad_out is None else list(grad_out)
        loss = torch.empty(self.n, dtype=torch.float64, device=self.device) if loss_out is None else loss_out
        check(self.lib.pwf_loss_grad_noalloc(self._c, self.n, _ptrs(psi, torch.complex64, self.shapes),
                                             _ptrs(y, torch.float32, self.shapes),
                                             _ptrs(grad, torch.complex64, self.shapes),
                                             ctypes.c_void_p(loss.data_ptr()), _stream(self.device)),
              "pwf_loss_grad_noalloc")
        return loss, grad

    def solve_plain(self, y: torch.Tensor, iters: int, psi_out=None, loss_hist: bool = True):
        if self.n != 1:
            raise ValueError("the plain path runs one instance")
        psi_out = self._empty(torch.complex64)[0] if psi_out is None else psi_out
        hist = torch.empty(max(iters, 1), dtype=torch.float64, device=self.device) if loss_hist else None
        ws, nb = self._ws()
        check(self.lib.pwf_solve_plain(self._c, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(psi_out.data_ptr()),
                                       iters, ctypes.c_void_p(hist.data_ptr()) if hist is not None else None,
                                       ws, nb, _stream(self.device)), "pwf_solve_plain")
        return psi_out, hist

    def autotune(self, reps: int = 5, cache_path: str | None = None, force: bool = False) -> bool:
        """Pick column-tile widths and row plans for this batch's grid sides (pwf_autotune).
        With ``cache_path`` the choices come from / go to that file (pwf_autotune_cached;
        ``force`` times them again); returns True when timing ran, False when the cache
        supplied every side."""
        ws, nb = self._ws()
        if cache_path is None:
            check(self.lib.pwf_autotune(self._c, self.n, reps, ws, nb, _stream(self.device)), "pwf_autotune")
            return True
        tuned = ctypes.c_int32(0)
        check(self.lib.pwf_autotune_cached(self._c, self.n, reps, str(cache_path).encode(), 1 if force else 0,
                                           ctypes.byref(tuned), ws, nb, _stream(self.device)), "pwf_autotune_cached")
        return bool(tuned.value)

    def bench_sweep(self, sweep: int, reps: int) -> None:
        """Launch fused sweep ``sweep`` (0..11) ``reps`` times on the state of the last solve."""
        ws, nb = self._ws()
        check(self.lib.pwf_bench_sweep(self._c, self.n, sweep, reps, ws, nb, _stream(self.device)),
              "pwf_bench_sweep")

    def sync_status(self) -> int:
        ws, _ = self._ws()
        return self.lib.pwf_sync_status(ws, _stream(self.device))


def set_graph_mode(on: bool) -> None:
    _lib.load().pwf_set_graph_mode(1 if on else 0)


def set_merged_launch(on: bool) -> None:
    """Uneven batches: one launch per sweep over all size classes (True) or per-class
    launches on parallel streams (False, default)."""
    _lib.load().pwf_set_merged_launch(1 if on else 0)


def set_column_tile(n: int, width: int, sweep: int = -1) -> None:
    """Tile width of column sweep S`sweep` (1, 3, ..., 11; -1 all) for side n (0: built-in default)."""
    check(_lib.load().pwf_set_column_tile(n, sweep, width), "pwf_set_column_tile")


def set_row_plan(n: int, sweep: int, plan: int) -> None:
    """Radix plan of row sweep S`sweep` (0, 2, ..., 10) for side n: 0 default, 1 alternative, -1 built-in."""
    check(_lib.load().pwf_set_row_plan(n, sweep, plan), "pwf_set_row_plan")


# ---------------------------------------------------------------- calibration front end

def speckle_g2(ref: torch.Tensor, max_shift: int = 32):
    """Normalised autocorrelations (g2_x, g2_y) of a reference speckle (pwf_speckle_g2)."""
    if not ref.is_cuda or ref.dtype != torch.float32 or not ref.is_contiguous() or ref.dim() != 2:
        raise ValueError("ref must be a contiguous float32 GPU image")
    lib = _lib.load()
    ws = torch.empty(lib.pwf_speckle_workspace_size(), dtype=torch.uint8, device=ref.device)
    gx = (ctypes.c_double * (max_shift + 1))()
    gy = (ctypes.c_double * (max_shift + 1))()
    ny, nx = ref.shape
    check(lib.pwf_speckle_g2(ctypes.c_void_p(ref.data_ptr()), nx, ny, max_shift, gx, gy,
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(ref.device)), "pwf_speckle_g2")
    return list(gx), list(gy)


def fit_coherence(g2, pixel_m: float):
    """(coherence length in metres, contrast) of the Gaussian Siegert model (pwf_fit_coherence)."""
    arr = (ctypes.c_double * len(g2))(*g2)
    coh, c = ctypes.c_double(), ctypes.c_double()
    check(_lib.load().pwf_fit_coherence(arr, len(g2), pixel_m, ctypes.byref(coh), ctypes.byref(c)),
          "pwf_fit_coherence")
    return coh.value, c.value


def calibrate_source(ref: torch.Tensor, pixel_m: float, max_shift: int = 32):
    """Coherence lengths (x_coh, y_coh) in metres of a reference speckle (Eq. 3), to be
    passed on as ``Problem(x_coh_m=..., y_coh_m=...)``, with the fitted contrasts and g2."""
    gx, gy = speckle_g2(ref, max_shift)
    xc, cx = fit_coherence(gx, pixel_m)
    yc, cy = fit_coherence(gy, pixel_m)
    return {"x_coh_m": xc, "y_coh_m": yc, "contrast_x": cx, "contrast_y": cy, "g2x": gx, "g2y": gy}


def diffuser_from_reference(problem: Problem, ref: torch.Tensor, eps: float = 1e-3) -> torch.Tensor:
    """Diffuser estimate from the reference speckle (pwf_diffuser_from_reference)."""
    lib = _lib.load()
    c = (_lib.pwf_problem * 1)(problem.to_c())
    size = lib.pwf_workspace_size(c, 1)
    if size == 0:
        raise ValueError("invalid problem description")
    ws = torch.empty(size, dtype=torch.uint8, device=ref.device)
    t = torch.empty((problem.ny, problem.nx), dtype=torch.complex64, device=ref.device)
    check(lib.pwf_diffuser_from_reference(c, ctypes.c_void_p(ref.data_ptr()), float(eps), ctypes.c_void_p(t.data_ptr()),
                                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(ref.device)),
          "pwf_diffuser_from_reference")
    return t


# ---------------------------------------------------------------- tomography

def fbp(psis: Sequence[torch.Tensor], angles_rad: Sequence[float], n_out: int | None = None,
        scale: float = 1.0, out: torch.Tensor | None = None) -> torch.Tensor:
    """Filtered back-projection of retrieved projections (pwf_fbp): [ny, n_out, n_out] complex64.

    With ``scale = wavelength / (2 pi pixel)`` the result is ``-beta + i delta``."""
    lib = _lib.load()
    n = len(psis)
    ny, nx = psis[0].shape
    n_out = nx if n_out is None else n_out
    size = lib.pwf_fbp_workspace_size(n, nx, ny)
    if size == 0:
        raise ValueError("unsupported tomography shape (see pwf_fbp_workspace_size)")
    dev = psis[0].device
    ws = torch.empty(size, dtype=torch.uint8, device=dev)
    vol = torch.empty((ny, n_out, n_out), dtype=torch.complex64, device=dev) if out is None else out
    ang = (ctypes.c_double * n)(*[float(a) for a in angles_rad])
    check(lib.pwf_fbp(_ptrs(psis, torch.complex64, [(ny, nx)] * n), n, nx, ny, ang, n_out, float(scale),
                      ctypes.c_void_p(vol.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                      _stream(dev)), "pwf_fbp")
    return vol


def background_quadratic(vol: torch.Tensor, r_bg: float, coefficients: bool = False):
    """Quadratic background removal of a tomogram [slices, n, n] complex64, in place
    (pwf_background_quadratic): per slice, the least-squares quadratic fitted to the
    voxels at radius >= r_bg (voxels) from the rotation axis is subtracted.  With
    ``coefficients`` also returns the fitted coefficients [slices][2][6] (FP64)."""
    if vol.dtype != torch.complex64 or vol.dim() != 3 or vol.shape[1] != vol.shape[2]:
        raise ValueError("a complex64 volume [slices, n, n]")
    if not (vol.is_cuda and vol.is_contiguous()):
        raise ValueError("a contiguous GPU array")
    lib = _lib.load()
    n_slices, n = vol.shape[0], vol.shape[1]
    size = lib.pwf_background_workspace_size(n_slices, n)
    if size == 0:
        raise ValueError("unsupported size for the background fit")
    ws = torch.empty(size, dtype=torch.uint8, device=vol.device)
    coef = (ctypes.c_double * (12 * n_slices))() if coefficients else None
    check(lib.pwf_background_quadratic(ctypes.c_void_p(vol.data_ptr()), n_slices, n, float(r_bg), coef,
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(vol.device)),
          "pwf_background_quadratic")
    if coefficients:
        return vol, [[list(coef[(12 * s + 6 * p):(12 * s + 6 * p + 6)]) for p in range(2)] for s in range(n_slices)]
    return vol


def shell_correlation(g1: torch.Tensor, g2: torch.Tensor, part: int = 1):
    """Fourier shell (3-D) or ring (2-D) correlation of Eq. 16 (pwf_shell_correlation):
    a list over shells 0..n/2 of the real (part 0) or imaginary (part 1) parts' FSC."""
    if g1.shape != g2.shape or g1.dtype != torch.complex64 or g2.dtype != torch.complex64:
        raise ValueError("two complex64 arrays of one shape")
    if not (g1.is_cuda and g2.is_cuda and g1.is_contiguous() and g2.is_contiguous()):
        raise ValueError("contiguous GPU arrays")
    n, dims = g1.shape[0], g1.dim()
    if any(s != n for s in g1.shape):
        raise ValueError("a square image or a cubic volume")
    lib = _lib.load()
    size = lib.pwf_shell_correlation_workspace_size(n, dims)
    if size == 0:
        raise ValueError("unsupported size for the shell correlation")
    ws = torch.empty(size, dtype=torch.uint8, device=g1.device)
    out = (ctypes.c_double * (n // 2 + 1))()
    check(lib.pwf_shell_correlation(ctypes.c_void_p(g1.data_ptr()), ctypes.c_void_p(g2.data_ptr()), n, dims, part,
                                    out, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(g1.device)),
          "pwf_shell_correlation")
    return list(out)
