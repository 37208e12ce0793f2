#!/usr/bin/env python3
"""Throughput of batched PWF on one MI355X.

Workload: 180 projections of 1024^2 (the 40-ellipsoid phantom over 0-180 deg,
one shared diffuser, source sigma 1.5 px, Poisson noise at 1e4 photons/px).
One step is one pwf_solve call: 100 iterations of Algorithm S1 on every
projection (forward model, loss, Wirtinger gradient, preconditioner,
regulariser, Nesterov step), captured as one hipGraph.  The value is
projection-iterations per second with all inputs resident in HBM.

Prints ONE JSON line.  Extra objects:
  roofline      the dominant sweep kernel, timed live with HIP events
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload
  plain_baseline the unfused one-kernel-per-operation GPU path on one projection
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PWF projection-iterations/s (fwd+grad) at 1024^2; % HBM roofline vs plain"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per pixel of each fused sweep (reads + writes of
# complex64 fields; windows and chirps are generated from indices).
SWEEP_BYTES_PER_PX = [24, 16, 24, 16, 20, 12, 20, 16, 24, 16, 24, 40]
SWEEP_NAMES = ["S0 row psi-update", "S1 col Q_L1", "S2 row x t", "S3 col Q_L2", "S4 row |v|^2",
               "S5 col blur+loss", "S6 row back-blur", "S7 col conj Q_L2", "S8 row x conj t",
               "S9 col conj Q_L1", "S10 row gradient", "S11 col direction+Nesterov"]
ITER_BYTES_PER_PX = sum(SWEEP_BYTES_PER_PX)   # 252
# the unfused-state schedule the roofline was first stated for (psi written and read, both
# Nesterov spectra read and written, real intensity spectra in full): reported beside it
SURVEY_SCHEDULE_BYTES_PER_PX = 280


# sources that define the 1024^2 sweep kernels: counters taken before a change to any
# of them no longer describe the kernels that run
SWEEP_SOURCES = ["pwf_device.h", "pwf_fft.h", "pwf_sweeps.h", "pwf_sweeps_1024.hip"]


def kernel_source_hash() -> str:
    """Hash of the code of SWEEP_SOURCES with comments and whitespace removed (a change
    of comments leaves the kernels, and so the counters, as they were)."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2503_20146_amd", "csrc")
    for f in SWEEP_SOURCES:
        with open(os.path.join(csrc, f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(sweep: int, pixels: int, width: int = 0):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None if stale."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    sweeps = rec.get("sweeps", {})
    ent = sweeps.get(str(sweep)) or sweeps.get(f"{sweep}:{width}")
    if not ent:
        return None
    return ent["hbm_bytes_per_px"] * pixels


COPY_BYTES = 1 << 30
# kernel-name fragments of each fused sweep at 1024^2 (template op ids of row_sweep / col_sweep;
# a row sweep's third template argument is its radix plan)
SWEEP_KERNELS = ["row_sweep<1024, 0,", "col_sweep<1024, {w}, 0>", "row_sweep<1024, 2,", "col_sweep<1024, {w}, 1>",
                 "row_sweep<1024, 4,", "col_sweep<1024, {w}, 4>", "row_sweep<1024, 5,", "col_sweep<1024, {w}, 2>",
                 "row_sweep<1024, 3,", "col_sweep<1024, {w}, 3>", "row_sweep<1024, 6,", "col_sweep<1024, {w}, 6>"]


TUNING_CACHE = os.path.join(ROOT, "paper_2503_20146_amd", "tuning_cache.txt")
RETUNE = False   # --retune: time every candidate again and rewrite this batch's cache entries


def autotune(batch) -> dict:
    """Column-tile widths and row plans per grid side from the persistent tuning cache
    (pwf_autotune_cached), timed afresh when the cache has no entry for this architecture and
    class mix, or with --retune; returns the chosen schedule and where it came from."""
    timed = batch.autotune(5, TUNING_CACHE, force=RETUNE)
    lib = batch.lib
    sides = sorted({p.ny for p in batch.problems} | {p.nx for p in batch.problems})
    return {"source": "timed, written to the tuning cache" if timed else "tuning cache",
            "column_tiles_S1_S3_S5_S7_S9_S11": {n: [lib.pwf_column_tile(n, s) for s in range(1, 12, 2)] for n in sides},
            "row_plans_S0_S2_S4_S6_S8_S10": {n: [lib.pwf_row_plan(n, s) for s in range(0, 12, 2)] for n in sides}}


def _counter_rows(path: str, counter: str):
    """(kernel name, dispatch id, value) of `counter` from rocprofv3 output: a
    counter_collection.csv (--output-format csv) or the rocpd SQLite database it writes by
    default (its counters_collection view)."""
    if path.endswith(".db"):
        import sqlite3
        con = sqlite3.connect(f"file:{path}?mode=ro", uri=True)
        try:
            yield from con.execute("select kernel_name, dispatch_id, value from counters_collection "
                                   "where counter_name = ?", (counter,))
        finally:
            con.close()
        return
    import csv
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row.get("Counter_Name") == counter:
                yield row["Kernel_Name"], row.get("Dispatch_Id"), float(row["Counter_Value"])


def _read_counter_csv(path: str, counter: str):
    """Per-kernel mean of `counter` over dispatches, and the largest single dispatch of a copy
    or fill kernel (the calibration launch)."""
    sums = {}
    for name, disp, val in _counter_rows(path, counter):
        key = (name, disp)
        sums[key] = sums.get(key, 0.0) + float(val)
    per_kernel = {}
    calib = 0.0
    for (name, _), val in sums.items():
        per_kernel.setdefault(name, []).append(val)
        if "copy" in name.lower() or "elementwise" in name.lower():
            calib = max(calib, val)
    return {k: sum(v) / len(v) for k, v in per_kernel.items()}, calib


def ingest_counters(fetch_csv: str, write_csv: str, projections: int, side: int = 1024) -> int:
    """Scale FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by the copy-kernel calibration.  The
    1024^2 run goes to profiles/traffic_counters.json (the bench's roofline.traffic), other
    sides to profiles/traffic_counters_<side>.json (documentation only)."""
    fetch, copy_f = _read_counter_csv(fetch_csv, "FETCH_SIZE")
    write, copy_w = _read_counter_csv(write_csv, "WRITE_SIZE")
    if copy_f <= 0 or copy_w <= 0:
        print("no calibration copy in the counter files", file=sys.stderr)
        return 1
    # the calibration launch copies COPY_BYTES: scale each counter so it reads exactly that
    kib = COPY_BYTES / 1024.0
    f_scale = kib / copy_f
    w_scale = kib / copy_w
    pixels = projections * side * side
    out = {"source_hash": kernel_source_hash(), "copy_bytes": COPY_BYTES, "side": side,
           "fetch_scale": f_scale, "write_scale": w_scale, "pixels_per_launch": pixels, "sweeps": {}}
    for s, frag in enumerate(SWEEP_KERNELS):
        frag = frag.replace("<1024,", f"<{side},")
        for w in (4, 8, 16, 32):
            names = [k for k in fetch if frag.format(w=w) in k]
            if not names:
                continue
            name = names[0]
            fb = fetch[name] * 1024.0 * f_scale
            wb = write.get(name, 0.0) * 1024.0 * w_scale
            key = f"{s}" if "row_sweep" in frag else f"{s}:{w}"
            out["sweeps"][key] = {"kernel": name, "fetch_bytes": fb, "write_bytes": wb,
                                  "hbm_bytes_per_px": (fb + wb) / pixels,
                                  "algorithmic_bytes_per_px": SWEEP_BYTES_PER_PX[s]}
    name = "traffic_counters.json" if side == 1024 else f"traffic_counters_{side}.json"
    path = os.path.join(ROOT, "profiles", name)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))
    return 0


def compiled_widths(lib, side: int) -> list:
    """Column-tile widths the library holds for `side` (pwf_set_column_tile accepts exactly
    those; host-side calls only), the default first."""
    default = lib.pwf_column_tile(side, 1)
    found = [w for w in (4, 8, 16, 32) if lib.pwf_set_column_tile(side, -1, w) == 0]
    lib.pwf_set_column_tile(side, -1, 0)
    return sorted(found, key=lambda w: w != default)


def sweep_only_side(side: int, n: int, which: str, reps: int, dev) -> int:
    """Counter runs at a side other than 1024: a batch of n instances of side^2 (the shared
    diffuser a seeded random phase screen, flat intensities: the sweeps' traffic does not
    depend on the values), a 2-iteration solve, the calibration copy, then every sweep
    `reps` times at each compiled column-tile width and the built-in row plans."""
    import numpy as np
    import torch

    import synthetic as S
    from paper_2503_20146_amd import PWF, _lib, problem_from_geometry
    geo = S.Geometry(ny=side, nx=side, sigma_x_px=1.5, sigma_y_px=1.5)
    rng = np.random.default_rng(S.BASE_SEED + side)
    t = torch.from_numpy(np.exp(1j * rng.uniform(0.0, 3.0, (side, side))).astype(np.complex64)).to(dev)
    batch = PWF([problem_from_geometry(geo, t) for _ in range(n)])
    ys = [torch.full((side, side), 0.9, device=dev) for _ in range(n)]
    batch.solve(ys, 2)
    torch.cuda.synchronize()
    sweeps = range(12) if which == "all" else [int(which)]
    if which == "all":
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    lib = _lib.load()
    for w in compiled_widths(lib, side):
        _lib.check(lib.pwf_set_column_tile(side, -1, w), "pwf_set_column_tile")
        for sw in sweeps:
            batch.bench_sweep(sw, reps)
        torch.cuda.synchronize()
    lib.pwf_set_column_tile(side, -1, 0)
    print(f"[bench] {n} x {side}^2: sweeps {list(sweeps)} x {reps} done", file=sys.stderr, flush=True)
    return 0


def build_workload(n_proj: int, dev):
    import numpy as np
    import torch

    import synthetic as S
    from paper_2503_20146_amd import PWF, problem_from_geometry

    d = S.tomo_projection_inputs(2, range(n_proj))
    geo = d["geometry"]
    t = torch.from_numpy(d["t"]).to(dev)
    probs = [problem_from_geometry(geo, t) for _ in range(n_proj)]
    batch = PWF(probs)
    psi_true = [torch.from_numpy(p.astype(np.complex64)).to(dev) for p in d["psi_true"]]
    f = batch.forward(psi_true)          # noise-free speckle from the GPU forward model
    torch.cuda.synchronize()
    ys = []
    for j in range(n_proj):
        y = S.poisson_intensity(f[j].cpu().numpy(), d["seed_keys"][j])
        ys.append(torch.from_numpy(y).to(dev))
    del f, psi_true
    return batch, ys, geo, probs, d


# Algorithmic FP32 flops of one voxel-angle step of the back-projection: the
# detector coordinate (mul, fma, add), the interpolation weight (sub) and, per
# real/imaginary part, the difference, the interpolating fma and the sum.
FBP_FLOPS_PER_VOXEL_ANGLE = 13
FP32_VECTOR_PEAK_TFLOPS = 157.3
# background removal: a read and a write of every voxel for the subtraction, plus a read of
# the background voxels for the moments (added per workload)
BACKGROUND_BYTES_PER_VOXEL = 16


def secondary_measurements(batch, ys, out, probs, geo, d, dev) -> dict:
    """Joint diffuser refinement, calibration front end and tomography on the same workload."""
    import math

    import torch

    import numpy as np

    from paper_2503_20146_amd import (PWF, background_quadratic, calibrate_source, diffuser_from_reference, fbp,
                                      problem_from_geometry, shell_correlation)

    res = {}
    n = len(probs)
    # joint diffuser refinement: the same 100-iteration solve, t stepped every iteration
    t_joint = probs[0].diffuser.clone()
    jb = PWF([problem_from_geometry(geo, t_joint) for _ in range(n)])
    jb.solve_joint(ys, 2, loss_hist=False)
    torch.cuda.synchronize()
    iters = 100
    t_joint.copy_(probs[0].diffuser)
    sec = time_events(lambda: jb.solve_joint(ys, iters, loss_hist=False))
    res["joint_diffuser"] = {"value": round(n * iters / sec, 1), "unit": "proj-iter/s",
                             "config": f"{n} projections x 1024^2, {iters} iterations, diffuser step every iteration"}
    del jb, t_joint
    torch.cuda.empty_cache()
    print(f"[bench] joint {res['joint_diffuser']['value']} proj-iter/s", file=sys.stderr, flush=True)
    # calibration on the reference speckle of the workload's diffuser (GPU forward at psi = 0)
    zero = torch.zeros((geo.ny, geo.nx), dtype=torch.complex64, device=dev)
    ref = PWF([probs[0]]).forward([zero])[0]
    calibrate_source(ref, geo.pixel_m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cal = calibrate_source(ref, geo.pixel_m)
    t_cal = time.perf_counter() - t0
    sec_t = time_events(lambda: diffuser_from_reference(probs[0], ref, 1e-3))
    res["calibration"] = {"coherence_ms": round(t_cal * 1e3, 3), "diffuser_ms": round(sec_t * 1e3, 3),
                          "coherence_um_fitted": [round(cal["x_coh_m"] * 1e6, 3), round(cal["y_coh_m"] * 1e6, 3)],
                          "coherence_um_of_the_blur": round(2.0 * math.sqrt(math.pi) * geo.sigma_x_px * geo.pixel_m * 1e6, 3),
                          "config": "one 1024^2 reference speckle, shifts 0..32"}
    print(f"[bench] calibration {res['calibration']}", file=sys.stderr, flush=True)
    # tomography of the retrieved projections
    angles = [math.pi * j / n for j in range(n)]
    scale = geo.wavelength_m / (2.0 * math.pi * geo.pixel_m)
    vol = fbp(out, angles, geo.nx, scale)
    torch.cuda.synchronize()
    sec_f = time_events(lambda: fbp(out, angles, geo.nx, scale, out=vol))
    va = float(geo.ny) * geo.nx * geo.nx * n
    achieved = va * FBP_FLOPS_PER_VOXEL_ANGLE / sec_f / 1e12
    res["tomography"] = {"ms": round(sec_f * 1e3, 2), "voxel_angles_per_s": round(va / sec_f, 1),
                         "roofline": {"bound": "alu", "achieved": round(achieved, 2),
                                      "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                      "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                                      "flops_per_voxel_angle": FBP_FLOPS_PER_VOXEL_ANGLE},
                         "config": f"FBP of {n} retrieved 1024^2 projections -> {geo.ny} x {geo.nx}^2 volume"}
    print(f"[bench] tomography {res['tomography']}", file=sys.stderr, flush=True)
    # Fourier shell correlation of the delta tomogram with that of the true projections
    if geo.ny == geo.nx:
        true_psis = [torch.from_numpy(p.astype(np.complex64)).to(dev) for p in d["psi_true"]]
        vol_true = fbp(true_psis, angles, geo.nx, scale)
        del true_psis
        shell_correlation(vol, vol_true, part=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fsc = shell_correlation(vol, vol_true, part=1)
        t_fsc = time.perf_counter() - t0
        kappa = next((k for k in range(1, len(fsc)) if fsc[k] < 0.5), len(fsc) - 1)
        kappa_q = next((k for k in range(1, len(fsc)) if fsc[k] < 0.25), len(fsc) - 1)   # Eqs. 17-18
        res["fsc_vs_truth"] = {"ms": round(t_fsc * 1e3, 2),
                               "resolution_um_at_quarter": round(geo.nx * geo.pixel_m / kappa_q * 1e6, 3),
                               "resolution_um_at_half": round(geo.nx * geo.pixel_m / kappa * 1e6, 3),
                               "fsc_at_shells_64_128_256_512": [round(fsc[k], 4) for k in (64, 128, 256, 512)],
                               "config": f"delta tomograms {geo.nx}^3 from retrieved vs true projections"}
        print(f"[bench] fsc {res['fsc_vs_truth']}", file=sys.stderr, flush=True)
        del vol_true
    # quadratic background removal of the tomogram (outside the 0.46 n cylinder)
    r_bg = 0.46 * geo.nx
    background_quadratic(vol, r_bg)
    torch.cuda.synchronize()
    sec_b = time_events(lambda: background_quadratic(vol, r_bg))
    vox = float(vol.numel())
    c = np.arange(geo.nx) + 0.5 - geo.nx / 2.0
    f_bg = float(np.mean(np.hypot(c[None, :], c[:, None]) >= r_bg))   # share of voxels the fit reads
    bytes_per_voxel = BACKGROUND_BYTES_PER_VOXEL + 8.0 * f_bg
    bg_gbs = vox * bytes_per_voxel / sec_b / 1e9
    res["background"] = {"ms": round(sec_b * 1e3, 2),
                         "roofline": {"bound": "hbm", "achieved": round(bg_gbs, 1), "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": round(bg_gbs / HBM_PEAK_GBS, 4),
                                      "bytes_per_voxel": round(bytes_per_voxel, 3)},
                         "config": f"quadratic background fit per slice of the {geo.ny} x {geo.nx}^2 tomogram, "
                                   f"background at radius >= {r_bg:g} voxels"}
    print(f"[bench] background {res['background']}", file=sys.stderr, flush=True)
    del vol
    torch.cuda.empty_cache()
    return res


def device_poisson(f, seed: int):
    """Flat-field-normalised Poisson counts of the noise-free speckle f (a GPU tensor), drawn
    on the device from a seeded generator (1e4 photons per pixel of unit flat field)."""
    import torch
    gen = torch.Generator(device=f.device)
    gen.manual_seed(seed)
    return torch.poisson(f.clamp(min=0.0) * 1.0e4, generator=gen).div_(1.0e4)


def workload_720x2048(dev, iters: int) -> dict:
    """The 720 x 2048^2 workload at its full size on one GPU: 720 projections of the 2048^3
    ellipsoid phantom over 0-180 deg (generated on the device), one shared 2048^2 diffuser,
    sigma 1.5 px, Poisson noise at 1e4 photons/px on the GPU forward model.  Timed: an
    autotuned pwf_solve of `iters` iterations on all 720 projections, and one forward and
    one backward of the differentiable loss (PWFLoss: the backward recomputes the forward
    fields) at the retrieved psi."""
    import numpy as np
    import torch

    import synthetic as S
    from paper_2503_20146_amd import PWF, problem_from_geometry, pwf_loss

    n, side = 720, 2048
    d = S.tomo_projection_inputs(4, [])
    geo = d["geometry"]
    t = torch.from_numpy(d["t"]).to(dev)
    phantom = S.ellipsoid_phantom(side, 40, (S.BASE_SEED + 2,), 2.0)
    psi = torch.empty((n, side, side), dtype=torch.complex64, device=dev)
    t0 = time.perf_counter()
    S.project_ellipsoids_device(phantom, [math.pi * j / n for j in range(n)], side, side, geo.pixel_m,
                                geo.wavelength_m, psi)
    torch.cuda.synchronize()
    print(f"[bench] 720 x 2048^2: projections generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    batch = PWF([problem_from_geometry(geo, t) for _ in range(n)])
    views = [psi[j] for j in range(n)]
    ys = batch.forward(views)
    for j in range(n):
        ys[j] = device_poisson(ys[j], S.BASE_SEED + 4 + j)
    torch.cuda.synchronize()
    tiles = autotune(batch)
    print(f"[bench] 720 x 2048^2: workspace {batch.workspace.numel() / 2**30:.1f} GiB, tiles {tiles}",
          file=sys.stderr, flush=True)
    batch.solve(ys, iters, psi_out=views, loss_hist=False)   # same length: graph captured here
    torch.cuda.synchronize()
    sec = time_events(lambda: batch.solve(ys, iters, psi_out=views, loss_hist=True))
    status = batch.sync_status()
    value = n * iters / sec
    roof = HBM_PEAK_GBS * 1e9 / (ITER_BYTES_PER_PX * side * side)
    print(f"[bench] 720 x 2048^2: {value:.1f} proj-iter/s", file=sys.stderr, flush=True)
    # differentiable loss at the retrieved psi: forward (model + misfit), backward (recomputed fields)
    p = psi.requires_grad_(True)
    torch.cuda.synchronize()
    a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    a.record()
    loss = pwf_loss(p, batch, ys)
    b.record()
    loss.sum().backward()
    c.record()
    c.synchronize()
    fwd_ms, bwd_ms = a.elapsed_time(b), b.elapsed_time(c)
    finite = bool(torch.isfinite(loss).all()) and bool(torch.isfinite(p.grad).all())
    res = {"value": round(value, 1), "unit": "proj-iter/s",
           "iteration_frac_of_hbm_roofline": round(value / roof, 4),
           "iteration_ms": round(sec / iters * 1e3, 2),
           "schedule": tiles,
           "autograd": {"forward_ms": round(fwd_ms, 1), "backward_ms": round(bwd_ms, 1),
                        "backward_proj_per_s": round(n / (bwd_ms / 1e3), 1), "finite": finite},
           "nonfinite_flag": status != 0,
           "workspace_gib": round(batch.workspace.numel() / 2 ** 30, 1),
           "config": f"{n} x {side}^2 projections of the 2048^3 40-ellipsoid phantom over 0-180 deg (generated on "
                     f"the device), shared diffuser, {iters} iterations in one hipGraph; PWFLoss forward and "
                     "backward over all 720"}
    del batch, ys, psi, p, views, loss
    torch.cuda.empty_cache()
    print(f"[bench] 720 x 2048^2 {res}", file=sys.stderr, flush=True)
    return res


def uneven_batch(dev, iters: int = 50) -> dict:
    """The uneven ROI batch: 64 distinct generated instances (24 x 512^2, 32 x 1024^2,
    8 x 2048^2, each with its own phase object, diffuser and IPSF sigma), the noise-free
    speckle from the GPU forward model with device Poisson noise; autotuned; one solve of
    `iters` iterations timed after a warm-up."""
    import numpy as np
    import torch

    import synthetic as S
    from paper_2503_20146_amd import PWF, problem_from_geometry

    specs = S.roi_batch_specs()
    probs, psis = [], []
    for i, (side, sigma) in enumerate(specs):
        inp = S.instance_inputs(3, side, instance=i, sigma_px=sigma)
        probs.append(problem_from_geometry(inp["geometry"], torch.from_numpy(inp["t"]).to(dev)))
        psis.append(torch.from_numpy(inp["psi_true"].astype(np.complex64)).to(dev))
    batch = PWF(probs)
    f = batch.forward(psis)
    ys = [device_poisson(f[j], S.BASE_SEED + 3000 + j) for j in range(len(specs))]
    del f, psis
    from paper_2503_20146_amd import set_merged_launch
    sched = autotune(batch)
    # warm-up of the same length: the solve's hipGraph (keyed by the iteration count) is
    # captured and instantiated there, outside the timed region
    batch.solve(ys, iters, loss_hist=False)
    torch.cuda.synchronize()
    sec = time_events(lambda: batch.solve(ys, iters, loss_hist=False))
    # the same batch with one launch per sweep over the three size classes (merged kernels,
    # tile widths and plans as tuned, the classes those kernels do not hold on their own)
    set_merged_launch(True)
    sched_m = autotune(batch)   # tuned for merged launches (its own cache entries)
    batch.solve(ys, iters, loss_hist=False)
    torch.cuda.synchronize()
    sec_m = time_events(lambda: batch.solve(ys, iters, loss_hist=False))
    set_merged_launch(False)
    autotune(batch)             # the per-class schedule again
    px = sum(side * side for side, _ in specs)
    frac = px * iters / sec * ITER_BYTES_PER_PX / (HBM_PEAK_GBS * 1e9)
    res = {"iteration_ms": round(sec / iters * 1e3, 3), "iteration_frac_of_hbm_roofline": round(frac, 4),
           "launch": "one launch per size class per sweep, the classes on parallel streams",
           "merged_launch_iteration_ms": round(sec_m / iters * 1e3, 3),
           "schedule": sched, "merged_launch_schedule": sched_m,
           "config": f"24 x 512^2 + 32 x 1024^2 + 8 x 2048^2, 64 distinct instances, {iters} iterations"}
    del batch, ys, probs
    torch.cuda.empty_cache()
    print(f"[bench] uneven batch {res}", file=sys.stderr, flush=True)
    return res


def streaming_reference(dev, iter_tbps: float):
    """Rates of plain streaming kernels (torch's own elementwise kernels over 1 GiB fp32
    operands, HIP events, 20 launches each) on this GPU: what a kernel that only streams
    reaches here, beside the published 8 TB/s the roofline fractions are taken against."""
    import torch
    n = 1 << 28
    a = torch.ones(n, device=dev)
    c = torch.ones(n, device=dev)
    b = torch.empty_like(a)
    out = {}
    for key, fn, nbytes in (("add_2read_1write_TBps", lambda: torch.add(a, c, out=b), 12 * n),
                            ("scale_1read_1write_TBps", lambda: torch.mul(a, 2.0, out=b), 8 * n),
                            ("fill_write_TBps", lambda: b.fill_(2.0), 4 * n),
                            ("memcpy_d2d_TBps", lambda: b.copy_(a), 8 * n)):
        fn()
        torch.cuda.synchronize()
        sec = time_events(lambda: [fn() for _ in range(20)]) / 20
        out[key] = round(nbytes / sec / 1e12, 2)
    del a, b, c
    torch.cuda.empty_cache()
    out["iteration_TBps"] = round(iter_tbps, 2)
    out["iteration_frac_of_add_rate"] = round(iter_tbps / out["add_2read_1write_TBps"], 3)
    return out


def time_events(fn, reps_note=None):
    import torch
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    fn()
    b.record(s)
    b.synchronize()
    return a.elapsed_time(b) / 1e3


def cpu_baseline(iters: int):
    import numpy as np

    import oracle as O
    import synthetic as S
    # threads: OMP_NUM_THREADS if set, else every core, at most 16
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    threads = max(1, min(threads, 16))
    O.FFT_WORKERS = threads
    d = S.tomo_projection_inputs(2, [0])
    prob = O.make_problem(d["t"], d["geometry"])
    f, _, _ = O.physical_model(d["psi_true"][0], prob)
    y = S.poisson_intensity(f, d["seed_keys"][0])
    st = O.initial_state(prob.shape)
    st, _ = O.pwf_step(st, y, prob)       # warm-up iteration (not timed)
    t0 = time.perf_counter()
    for _ in range(iters):
        st, _ = O.pwf_step(st, y, prob)
    dt = time.perf_counter() - t0
    # the same oracle on one thread, a shorter sample
    O.FFT_WORKERS = 1
    it1 = max(1, iters // 8)
    t0 = time.perf_counter()
    for _ in range(it1):
        st, _ = O.pwf_step(st, y, prob)
    dt1 = time.perf_counter() - t0
    O.FFT_WORKERS = threads
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": iters / dt, "unit": "proj-iter/s", "cores": threads, "kind": "oracle",
            "sample": f"1 projection of 1024^2 (projection 0 of the workload), {iters} iterations of the "
                      f"FP64 scipy.fft oracle after 1 warm-up iteration, {dt:.1f} s",
            "single_thread": {"value": it1 / dt1, "sample": f"{it1} further iterations on 1 thread, {dt1:.1f} s"},
            "cpu_model": model, "cpu_count": os.cpu_count(),
            "threads_note": "scipy.fft workers = OMP_NUM_THREADS (else all cores), capped at 16"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--projections", type=int, default=180)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--sweep-reps", type=int, default=10)
    ap.add_argument("--plain-iters", type=int, default=20)
    ap.add_argument("--cpu-iters", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the joint-diffuser, calibration and tomography measurements")
    ap.add_argument("--sweep-only", default=None,
                    help="after setup, only launch sweep K (0..11) or 'all' plus a 1 GiB copy (counter runs)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH", "WRITE"),
                    help="turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE output (counter_collection.csv or "
                         "the rocpd .db) of a --sweep-only all run "
                         "into profiles/traffic_counters.json and exit")
    ap.add_argument("--side", type=int, default=1024,
                    help="grid side of --sweep-only / --ingest-counters runs (1024: the headline batch; "
                         "others: --projections synthetic instances of that side)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--retune", action="store_true",
                    help="time every tile width and row plan again and rewrite the tuning cache's entries")
    ap.add_argument("--tuning-cache", default=None, help="tuning cache file (default: the package's)")
    ap.add_argument("--iters-2048", type=int, default=50,
                    help="iterations of the timed 720 x 2048^2 solve (extras)")
    ap.add_argument("--workload", choices=["720x2048", "uneven"], default=None,
                    help="only run this secondary workload and print its record (profiling runs)")
    ap.add_argument("--col-tile", type=int, default=0,
                    help="fix the column-tile width at 1024 instead of autotuning (counter runs)")
    args = ap.parse_args()

    global RETUNE, TUNING_CACHE
    RETUNE = args.retune
    if args.tuning_cache:
        TUNING_CACHE = args.tuning_cache
    if args.ingest_counters:
        return ingest_counters(*args.ingest_counters, projections=args.projections, side=args.side)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}); the "
              "projections are independent problems that shard across GPUs with no exchange", file=sys.stderr)
        return 2

    import torch
    dev = torch.device("cuda:0")
    if args.workload == "720x2048":
        print(json.dumps(workload_720x2048(dev, args.iters_2048)), flush=True)
        return 0
    if args.workload == "uneven":
        print(json.dumps(uneven_batch(dev, args.iters)), flush=True)
        return 0
    if args.sweep_only is not None and args.side != 1024:
        if args.side not in (128, 256, 512, 2048):
            print(f"bench.py: --side {args.side} is not a supported grid side", file=sys.stderr)
            return 2
        return sweep_only_side(args.side, args.projections, args.sweep_only, args.sweep_reps, dev)
    print(f"[bench] building workload: {args.projections} x 1024^2", file=sys.stderr, flush=True)
    batch, ys, geo, probs, d_inputs = build_workload(args.projections, dev)
    pixels = args.projections * geo.nx * geo.ny

    sched = {"source": "built-in defaults"}
    if args.col_tile:
        from paper_2503_20146_amd import _lib
        _lib.check(_lib.load().pwf_set_column_tile(1024, -1, args.col_tile), "pwf_set_column_tile")
        sched = {"source": f"--col-tile {args.col_tile}"}
    elif not args.no_autotune and args.sweep_only is None:
        sched = autotune(batch)
        print(f"[bench] schedule {sched}", file=sys.stderr, flush=True)
    from paper_2503_20146_amd import _lib as _l
    sched["column_tiles_S1_S3_S5_S7_S9_S11"] = {1024: [_l.load().pwf_column_tile(1024, s) for s in range(1, 12, 2)]}
    sched["row_plans_S0_S2_S4_S6_S8_S10"] = {1024: [_l.load().pwf_row_plan(1024, s) for s in range(0, 12, 2)]}

    if args.sweep_only is not None:
        batch.solve(ys, 2)
        torch.cuda.synchronize()
        sweeps = range(12) if args.sweep_only == "all" else [int(args.sweep_only)]
        if args.sweep_only == "all":
            # calibration: a plain device copy of exactly COPY_BYTES
            src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
        # every compiled column-tile width in turn unless one is fixed
        for w in ([args.col_tile] if args.col_tile else compiled_widths(_l.load(), 1024)):
            _l.load().pwf_set_column_tile(1024, -1, w)
            for sw in sweeps:
                batch.bench_sweep(sw, args.sweep_reps)
            torch.cuda.synchronize()
        print(f"[bench] sweeps {list(sweeps)} x {args.sweep_reps} done", file=sys.stderr, flush=True)
        return 0

    out = [torch.empty((geo.ny, geo.nx), dtype=torch.complex64, device=dev) for _ in range(args.projections)]
    # the loss history stays on in the timed run: its FP64 sums set the device's non-finite flag
    hist = torch.empty((args.projections, args.iters), dtype=torch.float64, device=dev)
    for w in range(args.warmup):
        batch.solve(ys, args.iters, psi_out=out, hist_out=hist)
        torch.cuda.synchronize()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        batch.solve(ys, args.iters, psi_out=out, hist_out=hist)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if batch.sync_status() != 0 or not bool(torch.isfinite(hist).all()):
        print("[bench] non-finite loss during the timed run", file=sys.stderr)
        return 1
    value = args.projections * args.iters * args.steps / dt
    print(f"[bench] timed {args.steps} steps in {dt:.3f} s -> {value:.1f} proj-iter/s", file=sys.stderr, flush=True)

    # per-sweep kernel durations, live, with HIP events on the launch stream
    sweep_s = []
    for s in range(12):
        batch.bench_sweep(s, 1)   # warm-up: the first direct launch of a kernel after the graph
        sec = time_events(lambda: batch.bench_sweep(s, args.sweep_reps)) / args.sweep_reps
        sweep_s.append(sec)
    # restore a meaningful state is not needed: timing only
    dom = max(range(12), key=lambda s: sweep_s[s])
    alg_bytes = SWEEP_BYTES_PER_PX[dom] * pixels
    achieved = alg_bytes / sweep_s[dom] / 1e9
    traffic = measured_traffic(dom, pixels, _l.load().pwf_column_tile(1024, dom) if dom % 2 else 0)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": SWEEP_NAMES[dom], "launch_ms": round(sweep_s[dom] * 1e3, 4),
                "algorithmic_bytes_per_launch": alg_bytes,
                "per_sweep_ms": [round(x * 1e3, 4) for x in sweep_s],
                "iteration_frac_of_hbm_roofline": round(value * ITER_BYTES_PER_PX * geo.nx * geo.ny / 1e9
                                                        / HBM_PEAK_GBS, 4),
                "iteration_frac_of_280B_schedule": round(value * SURVEY_SCHEDULE_BYTES_PER_PX * geo.nx * geo.ny
                                                         / 1e9 / HBM_PEAK_GBS, 4),
                "iteration_bytes_per_px": ITER_BYTES_PER_PX}
    print(f"[bench] sweeps ms: {[round(x * 1e3, 3) for x in sweep_s]}", file=sys.stderr, flush=True)

    plain = None
    if not args.no_plain:
        from paper_2503_20146_amd import PWF
        one = PWF([probs[0]])
        one.solve_plain(ys[0], 2)
        torch.cuda.synchronize()
        sec = time_events(lambda: one.solve_plain(ys[0], args.plain_iters, loss_hist=False))
        pv = args.plain_iters / sec
        plain = {"value": round(pv, 2), "unit": "proj-iter/s",
                 "path": "pwf_solve_plain: one projection, one kernel per operation (16 2-D FFTs per iteration), "
                         "no batching, no graph", "speedup_of_batched": round(value / pv, 2)}
        print(f"[bench] plain {pv:.1f} proj-iter/s", file=sys.stderr, flush=True)

    extras = None if args.no_extras else secondary_measurements(batch, ys, out, probs, geo, d_inputs, dev)
    if extras is not None:
        iter_tbps = value * ITER_BYTES_PER_PX * geo.nx * geo.ny / 1e12
        extras["streaming_reference"] = streaming_reference(dev, iter_tbps)
        print(f"[bench] streaming reference {extras['streaming_reference']}", file=sys.stderr, flush=True)
    del batch, ys, out, hist
    torch.cuda.empty_cache()
    if extras is not None:
        extras["workload_720x2048"] = workload_720x2048(dev, args.iters_2048)
        extras["uneven_roi_batch"] = uneven_batch(dev)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_iters)
        print(f"[bench] cpu oracle {cpu['value']:.3f} proj-iter/s on {cpu['cores']} threads", file=sys.stderr,
              flush=True)

    rec = {
        "metric": METRIC, "value": round(value, 2), "unit": "proj-iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"{args.projections} projections x 1024^2 of a 40-ellipsoid phantom over 0-180 deg, "
                               f"shared diffuser, {args.iters} PWF iterations per step in one hipGraph",
                   "projections": args.projections, "grid": [geo.ny, geo.nx], "iterations_per_step": args.iters,
                   "schedule": sched,
                   "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "plain_baseline": plain, "extras": extras,
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
