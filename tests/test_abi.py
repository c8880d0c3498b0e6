"""C-ABI checks that need no GPU: every symbol of include/sop.h is exported, the Python
binding declares exactly those symbols, and argument validation returns its status codes
before any device work."""
import ctypes as C
import math
import os
import re

import pytest

from paper_2510_07729_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sop.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(sop_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_parses_to_functions():
    names = declared_functions()
    for must in ("sop_shade", "sop_shade_backward", "sop_bake", "sop_knn", "sop_query",
                 "sop_plan_create", "sop_workspace_size"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(L.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_exactly_the_header():
    assert sorted(L.SIGNATURES) == declared_functions()


def test_misc_entry_points():
    lib = L.load()
    assert lib.sop_version() == 100
    assert lib.sop_status_string(L.SOP_OK) == b"ok"
    assert lib.sop_status_string(L.SOP_ERR_WORKSPACE_TOO_SMALL) == b"workspace too small"
    assert lib.sop_status_string(99) == b"unknown status"


def probe_set(count=4, lo=(-1, -1, -1), hi=(1, 1, 1), pos=0x1000):
    ps = L.sop_probe_set()
    ps.count = count
    ps.pos = pos
    ps.bounds_lo = (C.c_float * 3)(*lo)
    ps.bounds_hi = (C.c_float * 3)(*hi)
    return ps


@pytest.mark.parametrize("kwargs,msg", [
    (dict(count=-1), "count"),
    (dict(pos=0), "pos"),
    (dict(pos=0x1001), "misaligned"),
    (dict(lo=(0, 0, 0), hi=(1, 0, 1)), "hi > lo"),
    (dict(lo=(0, 0, float("nan"))), "finite"),
])
def test_plan_create_validation(kwargs, msg):
    lib = L.load()
    h = C.c_void_p()
    st = lib.sop_plan_create(C.byref(probe_set(**kwargs)), None, C.byref(h))
    assert st == L.SOP_ERR_INVALID_ARGUMENT
    assert msg in lib.sop_last_error().decode()
    assert not h.value


def test_null_plan_and_null_out_are_rejected():
    lib = L.load()
    assert lib.sop_plan_create(C.byref(probe_set()), None, None) == L.SOP_ERR_INVALID_ARGUMENT
    assert lib.sop_plan_rebuild(None, None, None) == L.SOP_ERR_INVALID_ARGUMENT
    assert lib.sop_plan_destroy(None) == L.SOP_OK
    assert lib.sop_bake_plan_destroy(None) == L.SOP_OK
    assert lib.sop_workspace_size(None, 0, 10, 4, 64, 32, 64, 0) == 0
    pts = L.sop_points()
    assert lib.sop_knn(None, C.byref(pts), 4, math.inf, None, None, None, None, 0,
                       None) == L.SOP_ERR_INVALID_ARGUMENT
    o = L.sop_shade_opts()
    assert lib.sop_shade(None, None, None, None, None, C.byref(o), None, None, 0,
                         None) == L.SOP_ERR_INVALID_ARGUMENT
    assert lib.sop_shade_backward(None, None, None, None, None, C.byref(o), None, None, None,
                                  None, None, None, None, 0, None) == L.SOP_ERR_INVALID_ARGUMENT
    assert lib.sop_bake(None, None, 0, 16, None, None, None, None) == L.SOP_ERR_INVALID_ARGUMENT
    assert lib.sop_bake_plan_check(None, None) == L.SOP_ERR_INVALID_ARGUMENT


def test_bake_plan_validation():
    lib = L.load()
    g = L.sop_gaussians()
    g.count = 10
    h = C.c_void_p()
    assert lib.sop_bake_plan_create(C.byref(g), None, None, C.byref(h)) == \
        L.SOP_ERR_INVALID_ARGUMENT
    assert "Gaussian" in lib.sop_last_error().decode()
    g.count = -3
    assert lib.sop_bake_plan_create(C.byref(g), None, None, C.byref(h)) == \
        L.SOP_ERR_INVALID_ARGUMENT
    g.count = 1
    for p in ("mean", "scale", "rotation", "opacity", "color"):
        setattr(g, p, 0x1000)
    o = L.sop_bake_opts(0.0, 0.5, 0.4, 1e-4, 0.0)     # alpha_max < alpha_min
    assert lib.sop_bake_plan_create(C.byref(g), C.byref(o), None, C.byref(h)) == \
        L.SOP_ERR_INVALID_ARGUMENT
    assert "bake options" in lib.sop_last_error().decode()
    o = L.sop_bake_opts(-1e-3, 1 / 255, 0.99, 1e-4, 0.0)   # rays start at the probe: t_min >= 0
    assert lib.sop_bake_plan_create(C.byref(g), C.byref(o), None, C.byref(h)) == \
        L.SOP_ERR_INVALID_ARGUMENT


def test_errors_are_thread_local():
    import threading
    lib = L.load()
    h = C.c_void_p()
    lib.sop_plan_create(C.byref(probe_set(count=-1)), None, C.byref(h))
    other = {}

    def worker():
        lib.sop_plan_create(C.byref(probe_set(pos=0)), None, C.byref(h))
        other["msg"] = lib.sop_last_error().decode()

    t = threading.Thread(target=worker)
    t.start()
    t.join()
    assert "count" in lib.sop_last_error().decode()
    assert "pos" in other["msg"]


def test_traced_shading_validation():
    """Every call below fails validation, so the stand-in plan pointer is never read."""
    lib = L.load()
    fake = C.c_void_p(0x1000)
    pts = L.sop_points()
    pts.count = 10
    for f in ("pos", "normal", "view", "albedo", "roughness", "metallic"):
        setattr(pts, f, 0x1000)
    env = L.sop_envmap()
    env.height, env.width, env.texels = 4, 8, 0x1000
    o = L.sop_shade_opts()
    o.n_dirs = 16
    rgb = 0x2000
    big = 1 << 30

    def call(gauss=fake, opts=o, offset=0.01, samples=None, ws_bytes=big, ws=0x10000):
        return lib.sop_shade_traced(gauss, None, C.byref(env), C.byref(pts),
                                    C.byref(opts) if opts is not None else None, offset, rgb,
                                    samples, ws, ws_bytes, None)

    assert call(gauss=None) == L.SOP_ERR_INVALID_ARGUMENT
    assert call(opts=None) == L.SOP_ERR_INVALID_ARGUMENT
    for bad in (-1e-3, math.inf, math.nan):
        assert call(offset=bad) == L.SOP_ERR_INVALID_ARGUMENT
        assert "offset" in lib.sop_last_error().decode()
    assert call(samples=0x2004) == L.SOP_ERR_INVALID_ARGUMENT       # not 16-byte aligned
    env.layout = 2                                                  # unknown layout
    assert call() == L.SOP_ERR_INVALID_ARGUMENT
    env.layout = L.SOP_ENV_OCTAHEDRAL                               # 4 x 8 is not square
    assert call() == L.SOP_ERR_INVALID_ARGUMENT
    assert "octahedral" in lib.sop_last_error().decode()
    env.layout = L.SOP_ENV_EQUIRECT
    o.sampler = L.SOP_SAMPLER_PROPOSAL
    assert call() == L.SOP_ERR_UNSUPPORTED
    o.sampler = L.SOP_SAMPLER_HAMMERSLEY
    o.n_dirs = 0
    assert call() == L.SOP_ERR_INVALID_ARGUMENT
    o.n_dirs = 16
    need = lib.sop_shade_traced_workspace_size(None, 10, 16, 4, 8, 0)
    assert need >= 10 * 16 * 16
    assert lib.sop_shade_traced_workspace_size(None, 10, 16, 4, 8, 1) < need
    assert call(ws_bytes=need - 256) == L.SOP_ERR_WORKSPACE_TOO_SMALL
    assert lib.sop_shade_traced_workspace_size(None, 10, 0, 4, 8, 0) == 0
    assert lib.sop_shade_traced_workspace_size(None, 10, 5000, 4, 8, 0) == 0
    assert lib.sop_shade_traced_workspace_size(None, -1, 16, 4, 8, 0) == 0


def test_shadow_ratio_validation():
    lib = L.load()
    o = L.sop_shadow_opts()
    o.n_dirs, o.k, o.radius = 16, 4, math.inf
    assert lib.sop_shadow_ratio(None, None, None, None, None, C.byref(o), None, None, 0,
                                None) == L.SOP_ERR_INVALID_ARGUMENT
    assert "plan" in lib.sop_last_error().decode()
    assert lib.sop_shadow_workspace_size(None, 10, 4, 16, 64, 0) == 0


def test_placement_and_loss_validation():
    lib = L.load()
    big = 1 << 20
    assert lib.sop_place_probes(0x1000, 0x1000, 0, 1, 0, 0.0, None, 0x2000, 0x10000, big,
                                None) == L.SOP_ERR_INVALID_ARGUMENT
    assert lib.sop_place_probes(0x1000, 0x1000, 10, 11, 0, 0.0, None, 0x2000, 0x10000, big,
                                None) == L.SOP_ERR_INVALID_ARGUMENT
    assert lib.sop_place_probes(0x1000, 0x1000, 10, 5, 10, 0.0, None, 0x2000, 0x10000, big,
                                None) == L.SOP_ERR_INVALID_ARGUMENT
    assert lib.sop_place_probes(0x1000, 0x1000, 10, 5, 0, math.inf, None, 0x2000, 0x10000, big,
                                None) == L.SOP_ERR_INVALID_ARGUMENT
    need = lib.sop_place_workspace_size(10, 5)
    assert need > 0 and lib.sop_place_workspace_size(10, 11) == 0
    assert lib.sop_place_probes(0x1000, 0x1000, 10, 5, 0, 0.0, None, 0x2000, 0x10000,
                                need - 256, None) == L.SOP_ERR_WORKSPACE_TOO_SMALL
    assert lib.sop_sops_loss(0x1008, 0x1000, 4, 0x2000, None, 0x10000, big,
                             None) == L.SOP_ERR_INVALID_ARGUMENT          # not 16-byte aligned
    assert lib.sop_lam_loss(None, 0x1000, 4, 0x2000, None, None, 0x10000, big,
                            None) == L.SOP_ERR_INVALID_ARGUMENT
    assert lib.sop_loss_workspace_size(-1) == 0


def test_peaks_library_exports_and_names():
    """The microbenchmark library (bench.py --peaks) loads and describes its benchmarks
    without touching a device; an unknown benchmark is refused before any HIP call."""
    lib = C.CDLL(os.path.join(ROOT, "paper_2510_07729_amd", "libsop_peaks.so"))
    lib.sop_peak_name.restype = C.c_char_p
    lib.sop_peak_unit.restype = C.c_char_p
    n = lib.sop_peak_count()
    assert n >= 10
    names = [lib.sop_peak_name(i).decode() for i in range(n)]
    assert len(set(names)) == n and all(names)
    assert lib.sop_peak_unit(0) == b"GB/s" and lib.sop_peak_name(n) == b""
    rate, ms = C.c_double(), C.c_double()
    assert lib.sop_peak_run(n, 1, C.byref(rate), C.byref(ms)) == -1
    assert lib.sop_peak_run(0, 0, C.byref(rate), C.byref(ms)) == -1
