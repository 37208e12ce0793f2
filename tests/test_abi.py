"""Host-side checks of the C ABI (no GPU work: every call here fails validation
before anything is queued, or only queries sizes and strings)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pwf.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2503_20146_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpwf.so not built")
    return _lib.load()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pwf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = header_functions()
    for required in ("pwf_forward", "pwf_gradient", "pwf_step", "pwf_solve", "pwf_workspace_size",
                     "pwf_status_string", "pwf_solve_plain", "pwf_state_init"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_2503_20146_amd import _lib
    assert set(_lib.SIGNATURES) == set(header_functions())


def test_status_strings(lib):
    from paper_2503_20146_amd import _lib
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        s = lib.pwf_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.pwf_status_string(42).decode() == "unknown status"
    assert lib.pwf_version() >= 10000
    assert _lib.status_string(-3).startswith("geometry has evanescent")


def test_tuning_settings(lib):
    """Tile widths and row plans: defaults, settable values, errors (host-only calls)."""
    # defaults: 16 columns at 1024 and 8 at 2048 (one half of the split column transform)
    assert lib.pwf_column_tile(1024, 1) == 16 and lib.pwf_column_tile(2048, 11) == 8
    assert lib.pwf_column_tile(100, 1) == 0 and lib.pwf_column_tile(1024, 2) == 0
    assert lib.pwf_set_column_tile(1024, -1, 3) == -1
    assert lib.pwf_set_column_tile(1024, -1, 4) == -1    # not compiled at 1024 (16 and 8 are)
    assert lib.pwf_set_column_tile(2048, -1, 4) == -1    # nor at 2048 (8 and 16 are)
    assert lib.pwf_set_column_tile(1024, 4, 8) == -1     # S4 is a row sweep
    assert lib.pwf_set_column_tile(100, -1, 8) == -2
    try:
        assert lib.pwf_set_column_tile(1024, 11, 8) == 0
        assert lib.pwf_column_tile(1024, 11) == 8 and lib.pwf_column_tile(1024, 1) == 16
        assert lib.pwf_set_column_tile(1024, -1, 8) == 0
        assert all(lib.pwf_column_tile(1024, s) == 8 for s in range(1, 12, 2))
        assert lib.pwf_set_column_tile(2048, 11, 16) == 0
        assert lib.pwf_column_tile(2048, 11) == 16 and lib.pwf_column_tile(2048, 1) == 8
    finally:
        lib.pwf_set_column_tile(1024, -1, 0)
        lib.pwf_set_column_tile(2048, -1, 0)
    assert lib.pwf_column_tile(1024, 11) == 16 and lib.pwf_column_tile(2048, 11) == 8
    # built-in plans at 1024: every tunable row sweep on the alternative plan
    assert [lib.pwf_row_plan(1024, s) for s in range(0, 12, 2)] == [1, 1, 1, 1, 1, 1]
    assert [lib.pwf_row_plan(2048, s) for s in range(0, 12, 2)] == [1, 0, 1, 0, 0, 1]
    assert lib.pwf_row_plan(1024, 1) == -1 and lib.pwf_row_plan(100, 0) == -1
    assert lib.pwf_set_row_plan(1024, 3, 0) == -1      # S3 is a column sweep
    assert lib.pwf_set_row_plan(1024, 2, 3) == -1
    assert lib.pwf_set_row_plan(512, 2, 2) == -1        # two plans below 1024
    assert lib.pwf_set_row_plan(96, 2, 1) == -2
    try:
        assert lib.pwf_set_row_plan(1024, 2, 0) == 0
        assert lib.pwf_row_plan(1024, 2) == 0
        assert lib.pwf_set_row_plan(2048, 2, 1) == 0
        assert lib.pwf_row_plan(2048, 2) == 1
        assert lib.pwf_set_row_plan(1024, 4, 2) == 0
        assert lib.pwf_row_plan(1024, 4) == 2
    finally:
        lib.pwf_set_row_plan(1024, 2, -1)
        lib.pwf_set_row_plan(1024, 4, -1)
        lib.pwf_set_row_plan(2048, 2, -1)
    assert lib.pwf_row_plan(1024, 2) == 1 and lib.pwf_row_plan(2048, 2) == 0


def _problem(nx=128, ny=128, **kw):
    from paper_2503_20146_amd import _lib
    p = _lib.pwf_problem()
    p.geom = _lib.pwf_geometry(nx, ny, kw.get("pixel", 1e-6), kw.get("lam", 0.05e-9), kw.get("z1", 5e-3),
                               kw.get("z2", 0.2))
    p.source = _lib.pwf_source(kind=kw.get("kind", _lib.PWF_SRC_GAUSS), sigma_x_px=kw.get("sx", 1.0),
                               sigma_y_px=kw.get("sy", 1.0), x_coh_m=kw.get("xc", 0.0), y_coh_m=kw.get("yc", 0.0),
                               iotf_x=kw.get("ix", None), iotf_y=kw.get("iy", None))
    p.params = _lib.pwf_params(kw.get("eta", 0.5), 0.1, 0.01, kw.get("gamma", 1.0), kw.get("sp", 0.025), 1)
    p.diffuser = kw.get("diffuser", 0x1000)
    return p


def test_source_forms_accepted(lib):
    """Every source form with valid members passes validation (pwf_workspace_size > 0)."""
    from paper_2503_20146_amd import _lib
    for kw in (dict(kind=0, sx=0.0, sy=2.0), dict(kind=1, xc=3.47e-6, yc=4.31e-6), dict(kind=1, xc=0.0, yc=0.0),
               dict(kind=2, ix=0x4000, iy=0x5000)):
        arr = (_lib.pwf_problem * 1)(_problem(**kw))
        assert lib.pwf_workspace_size(arr, 1) > 0, kw


def test_workspace_size(lib):
    from paper_2503_20146_amd import _lib
    arr = (_lib.pwf_problem * 2)(_problem(), _problem(256, 512))
    size = lib.pwf_workspace_size(arr, 2)
    fields = 6 * (128 * 128 + 256 * 512) * 8 + 2 * 128 * 128 * 8
    assert fields < size < fields + (1 << 20)
    assert lib.pwf_workspace_size(arr, 0) == 0
    bad = (_lib.pwf_problem * 1)(_problem(100, 128))
    assert lib.pwf_workspace_size(bad, 1) == 0


@pytest.mark.parametrize("kw,expect", [
    (dict(nx=100), -2), (dict(ny=4096), -2), (dict(pixel=0.0), -1), (dict(lam=float("nan")), -1),
    (dict(z1=-1e-3), -1), (dict(sx=-1.0), -1), (dict(eta=float("inf")), -1), (dict(sp=0.0), -1),
    (dict(diffuser=0), -1), (dict(lam=2e-6, pixel=1e-6), -3),
    (dict(kind=3), -1), (dict(kind=1, xc=-1e-6), -1), (dict(kind=1, yc=float("nan")), -1),
    (dict(kind=2, ix=0x4000), -1), (dict(kind=2, iy=0x4000), -1),
])
def test_invalid_problems_rejected_before_any_gpu_work(lib, kw, expect):
    from paper_2503_20146_amd import _lib
    arr = (_lib.pwf_problem * 1)(_problem(**kw))
    ptrs = (ctypes.c_void_p * 1)(0x2000)
    ws = ctypes.c_void_p(0x100000)
    assert lib.pwf_forward(arr, 1, ptrs, ptrs, ws, 1 << 40, None) == expect
    assert lib.pwf_solve(arr, 1, ptrs, ptrs, 10, 0.0, None, None, ws, 1 << 40, None) == expect


def test_bad_workspace_and_pointers(lib):
    from paper_2503_20146_amd import _lib
    arr = (_lib.pwf_problem * 1)(_problem())
    ptrs = (ctypes.c_void_p * 1)(0x2000)
    null = (ctypes.c_void_p * 1)(None)
    size = lib.pwf_workspace_size(arr, 1)
    assert lib.pwf_forward(arr, 1, ptrs, ptrs, ctypes.c_void_p(0x100001), size, None) == -4
    assert lib.pwf_forward(arr, 1, ptrs, ptrs, ctypes.c_void_p(0x100000), size - 1, None) == -4
    assert lib.pwf_forward(arr, 1, ptrs, ptrs, None, size, None) == -4
    assert lib.pwf_forward(arr, 1, null, ptrs, ctypes.c_void_p(0x100000), size, None) == -1
    assert lib.pwf_forward(None, 1, ptrs, ptrs, ctypes.c_void_p(0x100000), size, None) == -1
    assert lib.pwf_solve(arr, 1, ptrs, ptrs, -1, 0.0, None, None, ctypes.c_void_p(0x100000), size, None) == -1
    assert lib.pwf_solve(arr, 1, ptrs, ptrs, 5, 1.5, None, None, ctypes.c_void_p(0x100000), size, None) == -1
    assert lib.pwf_solve(arr, 1, ptrs, ptrs, 5, float("nan"), None, None, ctypes.c_void_p(0x100000), size,
                         None) == -1
    assert lib.pwf_sync_status(ctypes.c_void_p(0x100001), None) == -4


def test_noalloc_limits_checked_before_any_gpu_work(lib):
    """pwf_loss_grad_noalloc: batches beyond its static buffer (63 MiB of workspace, 64
    instances) and null pointers are refused on the host."""
    from paper_2503_20146_amd import _lib
    assert lib.pwf_loss_grad_noalloc_limit() == 63 << 20
    two = (_lib.pwf_problem * 2)(_problem(1024, 1024), _problem(1024, 1024))
    ptrs2 = (ctypes.c_void_p * 2)(0x2000, 0x3000)
    assert lib.pwf_loss_grad_noalloc(two, 2, ptrs2, ptrs2, ptrs2, None, None) == _lib.PWF_ERR_SCRATCH
    many = (_lib.pwf_problem * 65)(*[_problem() for _ in range(65)])
    ptrs65 = (ctypes.c_void_p * 65)(*([0x2000] * 65))
    assert lib.pwf_loss_grad_noalloc(many, 65, ptrs65, ptrs65, ptrs65, None, None) == _lib.PWF_ERR_SCRATCH
    one = (_lib.pwf_problem * 1)(_problem())
    null = (ctypes.c_void_p * 1)(None)
    ptrs1 = (ctypes.c_void_p * 1)(0x2000)
    assert lib.pwf_loss_grad_noalloc(one, 1, ptrs1, ptrs1, null, None, None) == _lib.PWF_ERR_ARG
    assert lib.pwf_loss_grad_noalloc(one, 1, None, ptrs1, ptrs1, None, None) == _lib.PWF_ERR_ARG
    bad = (_lib.pwf_problem * 1)(_problem(100, 128))
    assert lib.pwf_loss_grad_noalloc(bad, 1, ptrs1, ptrs1, ptrs1, None, None) == _lib.PWF_ERR_SIZE


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2503_20146_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def test_product_code_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2503_20146_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "synthetic" not in text, f


def test_fit_coherence_host(lib):
    """pwf_fit_coherence is host arithmetic: exact on a model curve, errors on degenerate input."""
    import math
    d = [float(i) for i in range(40)]
    g2 = [1.0 + 0.37 * math.exp(-math.pi * (x * 0.65e-6) ** 2 / (4.1e-6) ** 2) for x in d]
    g2[0] += 0.8
    arr = (ctypes.c_double * 40)(*g2)
    coh, c = ctypes.c_double(), ctypes.c_double()
    assert lib.pwf_fit_coherence(arr, 40, 0.65e-6, ctypes.byref(coh), ctypes.byref(c)) == 0
    assert abs(coh.value / 4.1e-6 - 1) < 1e-12 and abs(c.value - 0.37) < 1e-12
    flat = (ctypes.c_double * 5)(*([1.0] * 5))
    assert lib.pwf_fit_coherence(flat, 5, 1e-6, ctypes.byref(coh), None) == -1
    assert lib.pwf_fit_coherence(arr, 2, 1e-6, ctypes.byref(coh), None) == -1
    assert lib.pwf_fit_coherence(arr, 40, 0.0, ctypes.byref(coh), None) == -1


def test_calibration_and_joint_argument_errors(lib):
    from paper_2503_20146_amd import _lib
    g = (ctypes.c_double * 40)()
    ws = ctypes.c_void_p(0x100000)
    big = lib.pwf_speckle_workspace_size()
    assert big > 0
    img = ctypes.c_void_p(0x2000)
    assert lib.pwf_speckle_g2(img, 128, 128, 33, g, g, ws, big, None) == -1     # shift above 32
    assert lib.pwf_speckle_g2(img, 16, 16, 16, g, g, ws, big, None) == -1      # shift >= side
    assert lib.pwf_speckle_g2(img, 128, 128, 8, g, g, ws, big - 1, None) == -4
    assert lib.pwf_speckle_g2(None, 128, 128, 8, g, g, ws, big, None) == -1
    arr = (_lib.pwf_problem * 1)(_problem())
    size = lib.pwf_workspace_size(arr, 1)
    assert lib.pwf_diffuser_from_reference(arr, img, -1.0, img, ws, size, None) == -1
    assert lib.pwf_diffuser_from_reference(arr, img, 1e-3, None, ws, size, None) == -1
    two = (_lib.pwf_problem * 2)(_problem(diffuser=0x1000), _problem(diffuser=0x3000))
    ptrs = (ctypes.c_void_p * 2)(0x2000, 0x2000)
    jsize = lib.pwf_joint_workspace_size(two, 2)
    assert jsize > lib.pwf_workspace_size(two, 2)
    assert lib.pwf_solve_joint(two, 2, ptrs, ptrs, 5, 0.5, None, ws, jsize, None) == -1   # distinct diffusers
    one = (_lib.pwf_problem * 1)(_problem())
    assert lib.pwf_solve_joint(one, 1, ptrs, ptrs, 5, float("nan"), None, ws, 1 << 40, None) == -1
    assert lib.pwf_solve_joint(one, 1, ptrs, ptrs, 5, 0.5, None, ws, lib.pwf_workspace_size(one, 1), None) == -4


def test_fbp_argument_errors(lib):
    assert lib.pwf_fbp_workspace_size(180, 1024, 1024) > 180 * 1024 * 2048 * 8
    assert lib.pwf_fbp_workspace_size(0, 1024, 1024) == 0
    assert lib.pwf_fbp_workspace_size(180, 2048, 1024) == 0      # padded rows beyond 2048
    assert lib.pwf_fbp_workspace_size(180, 1024, 1000) == 0      # ny not a multiple of 32
    ang = (ctypes.c_double * 2)(0.0, 1.0)
    ptrs = (ctypes.c_void_p * 2)(0x2000, 0x3000)
    size = lib.pwf_fbp_workspace_size(2, 128, 64)
    ws = ctypes.c_void_p(0x100000)
    assert lib.pwf_fbp(ptrs, 2, 128, 64, ang, 120, 1.0, ctypes.c_void_p(0x4000), ws, size, None) == -1   # n_out % 16
    assert lib.pwf_fbp(ptrs, 2, 128, 64, ang, 128, 1.0, None, ws, size, None) == -1
    assert lib.pwf_fbp(ptrs, 2, 128, 64, ang, 128, 1.0, ctypes.c_void_p(0x4000), ws, size - 1, None) == -4
    assert lib.pwf_fbp(ptrs, 2, 100, 60, ang, 128, 1.0, ctypes.c_void_p(0x4000), ws, size, None) == -2


def test_shell_correlation_argument_errors(lib):
    assert lib.pwf_shell_correlation_workspace_size(128, 3) > 128 ** 3 * 8   # one complex field + partials
    assert lib.pwf_shell_correlation_workspace_size(100, 3) == 0
    assert lib.pwf_shell_correlation_workspace_size(128, 4) == 0
    out = (ctypes.c_double * 65)()
    size = lib.pwf_shell_correlation_workspace_size(128, 2)
    ws = ctypes.c_void_p(0x100000)
    p = ctypes.c_void_p(0x2000)
    assert lib.pwf_shell_correlation(p, p, 128, 2, 2, out, ws, size, None) == -1
    assert lib.pwf_shell_correlation(None, p, 128, 2, 0, out, ws, size, None) == -1
    assert lib.pwf_shell_correlation(p, p, 128, 2, 0, out, ws, size - 1, None) == -4
    assert lib.pwf_shell_correlation(p, p, 96, 2, 0, out, ws, size, None) == -2


def test_background_argument_errors(lib):
    """Every refusal of pwf_background_quadratic happens on the host, before any GPU work."""
    assert lib.pwf_background_workspace_size(4, 64) > 0
    assert lib.pwf_background_workspace_size(0, 64) == 0
    assert lib.pwf_background_workspace_size(4, 40) == 0
    assert lib.pwf_background_workspace_size(4, 8) == 0
    size = lib.pwf_background_workspace_size(4, 64)
    ws = ctypes.c_void_p(0x100000)
    v = ctypes.c_void_p(0x2000)
    assert lib.pwf_background_quadratic(None, 4, 64, 20.0, None, ws, size, None) == -1
    assert lib.pwf_background_quadratic(v, 4, 64, -1.0, None, ws, size, None) == -1
    assert lib.pwf_background_quadratic(v, 4, 64, float("nan"), None, ws, size, None) == -1
    assert lib.pwf_background_quadratic(v, 4, 64, 32.0 * 2 ** 0.5, None, ws, size, None) == -1  # no background
    assert lib.pwf_background_quadratic(v, 4, 64, 20.0, None, ws, size - 1, None) == -4
    assert lib.pwf_background_quadratic(v, 4, 48 + 2, 20.0, None, ws, size, None) == -2
