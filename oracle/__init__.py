"""CPU FP64 oracle of the SOP query-and-shade path (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use this package.
It wraps ``sop_oracle.c`` (plain C, double precision, OpenMP over points) with ctypes; the
GPU library never imports it and shares no source with it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sop_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (always when force, else only if missing or stale)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


dptr = C.POINTER(C.c_double)
fptr = C.POINTER(C.c_float)
iptr = C.POINTER(C.c_int32)


def _sig(lib):
    u32 = C.c_uint32
    lib.orc_bitreverse32.restype = u32
    lib.orc_bitreverse32.argtypes = [u32]
    lib.orc_pcg_hash.restype = u32
    lib.orc_pcg_hash.argtypes = [u32]
    lib.orc_rotation24.restype = u32
    lib.orc_rotation24.argtypes = [u32, C.c_int, u32]
    lib.orc_oct_encode.argtypes = [dptr, C.c_int, dptr]
    lib.orc_oct_decode.argtypes = [C.c_double, C.c_double, C.c_int, dptr]
    lib.orc_oct_taps.argtypes = [C.c_double, C.c_double, C.c_int, iptr, dptr]
    lib.orc_oct_fetch.argtypes = [dptr, C.c_int, C.c_int, dptr, dptr]
    lib.orc_env_taps.argtypes = [dptr, C.c_int, C.c_int, iptr, dptr]
    lib.orc_env_fetch.argtypes = [dptr, C.c_int, C.c_int, dptr, dptr]
    lib.orc_frame.argtypes = [dptr, dptr, dptr]
    lib.orc_direction.restype = C.c_double
    lib.orc_direction.argtypes = [C.c_int, C.c_int, u32, dptr, dptr]
    lib.orc_ggx_D.restype = C.c_double
    lib.orc_ggx_D.argtypes = [C.c_double, C.c_double]
    lib.orc_smith_G1.restype = C.c_double
    lib.orc_smith_G1.argtypes = [C.c_double, C.c_double]
    lib.orc_schlick_F.restype = C.c_double
    lib.orc_schlick_F.argtypes = [C.c_double, C.c_double]
    lib.orc_brdf.argtypes = [dptr, dptr, dptr, dptr, C.c_double, C.c_double, dptr]
    lib.orc_lattice_scale.restype = C.c_float
    lib.orc_lattice_scale.argtypes = [fptr, fptr]
    lib.orc_quantize.argtypes = [fptr, fptr, C.c_float, iptr]
    lib.orc_radius_limit.restype = u32
    lib.orc_radius_limit.argtypes = [C.c_float, C.c_float]
    lib.orc_knn.argtypes = [fptr, C.c_int, fptr, fptr, fptr, fptr, C.c_long, C.c_int,
                            C.c_float, iptr, dptr]
    lib.orc_query.argtypes = [dptr, C.c_int, iptr, dptr, C.c_int, C.c_long, dptr, C.c_int,
                              dptr, dptr]
    lib.orc_shade.argtypes = [C.c_long, dptr, dptr, dptr, dptr, C.c_long, dptr, dptr, dptr,
                              dptr, C.c_int, dptr, C.c_int, C.c_int, iptr, dptr, C.c_int,
                              C.c_int, u32, C.c_int, dptr, dptr]
    lib.orc_shade_backward.argtypes = [C.c_long, dptr, dptr, dptr, dptr, C.c_long, dptr, dptr,
                                       dptr, dptr, C.c_int, dptr, C.c_int, C.c_int, iptr,
                                       dptr, C.c_int, C.c_int, u32, C.c_int, dptr, dptr, dptr,
                                       dptr, dptr, dptr, dptr, dptr, dptr, dptr, dptr]
    lib.orc_bake_rays.argtypes = [C.c_int, dptr, dptr, dptr, dptr, dptr, dptr, C.c_int,
                                  C.c_long, iptr, iptr, C.c_double, C.c_double, C.c_double,
                                  C.c_double, dptr, iptr, iptr]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            _lib = C.CDLL(_LIB_PATH)
            _sig(_lib)
    return _lib


def set_threads(n: int) -> None:
    """OpenMP thread count of the oracle (omp_set_num_threads via libgomp)."""
    lib()
    gomp = C.CDLL("libgomp.so.1")
    gomp.omp_set_num_threads(int(n))


def max_threads() -> int:
    lib()
    gomp = C.CDLL("libgomp.so.1")
    return int(gomp.omp_get_max_threads())


# ------------------------------------------------------------------------------------------
def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(dptr)


def _f(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(fptr)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(iptr)


def _opt(a):
    if a is None:
        return None, None
    return _d(a)


def bitreverse32(x: int) -> int:
    return int(lib().orc_bitreverse32(x))


def pcg_hash(x: int) -> int:
    return int(lib().orc_pcg_hash(x))


def rotation24(seed: int, per_point: bool, i: int) -> int:
    return int(lib().orc_rotation24(seed, int(per_point), i))


def oct_encode(w, R: int):
    w, pw = _d(w)
    out = np.zeros(2)
    lib().orc_oct_encode(pw, R, out.ctypes.data_as(dptr))
    return out


def oct_decode(u: float, v: float, R: int):
    out = np.zeros(3)
    lib().orc_oct_decode(u, v, R, out.ctypes.data_as(dptr))
    return out


def oct_taps(u: float, v: float, R: int):
    tap = np.zeros(4, np.int32)
    wt = np.zeros(4)
    lib().orc_oct_taps(u, v, R, tap.ctypes.data_as(iptr), wt.ctypes.data_as(dptr))
    return tap, wt


def oct_fetch(tex, w):
    """tex [R,R,C]; bilinear octahedral fetch in direction w."""
    tex, pt = _d(tex)
    w, pw = _d(w)
    out = np.zeros(tex.shape[2])
    lib().orc_oct_fetch(pt, tex.shape[0], tex.shape[2], pw, out.ctypes.data_as(dptr))
    return out


def env_fetch(env, w):
    env, pe = _d(env)
    w, pw = _d(w)
    out = np.zeros(3)
    lib().orc_env_fetch(pe, env.shape[0], env.shape[1], pw, out.ctypes.data_as(dptr))
    return out


def env_taps(w, H: int, W: int):
    w, pw = _d(w)
    tap = np.zeros(4, np.int32)
    wt = np.zeros(4)
    lib().orc_env_taps(pw, H, W, tap.ctypes.data_as(iptr), wt.ctypes.data_as(dptr))
    return tap, wt


def frame(n):
    n, pn = _d(n)
    t = np.zeros(3)
    b = np.zeros(3)
    lib().orc_frame(pn, t.ctypes.data_as(dptr), b.ctypes.data_as(dptr))
    return t, b


def direction(j: int, S: int, rho24: int, n):
    n, pn = _d(n)
    w = np.zeros(3)
    ct = lib().orc_direction(j, S, rho24, pn, w.ctypes.data_as(dptr))
    return w, ct


def ggx_D(NoH: float, alpha: float) -> float:
    return float(lib().orc_ggx_D(NoH, alpha))


def smith_G1(c: float, k: float) -> float:
    return float(lib().orc_smith_G1(c, k))


def schlick_F(F0: float, VoH: float) -> float:
    return float(lib().orc_schlick_F(F0, VoH))


def brdf(n, v, l, a, r, m):
    n, pn = _d(n)
    v, pv = _d(v)
    l, pl = _d(l)
    a, pa = _d(a)
    f = np.zeros(3)
    lib().orc_brdf(pn, pv, pl, pa, r, m, f.ctypes.data_as(dptr))
    return f


def lattice_scale(lo, hi) -> float:
    lo, plo = _f(lo)
    hi, phi = _f(hi)
    return float(lib().orc_lattice_scale(plo, phi))


def quantize(x, lo, sc):
    x, px = _f(x)
    lo, plo = _f(lo)
    q = np.zeros(3, np.int32)
    lib().orc_quantize(px, plo, C.c_float(sc), q.ctypes.data_as(iptr))
    return q


def radius_limit(radius: float, sc: float) -> int:
    return int(lib().orc_radius_limit(C.c_float(radius), C.c_float(sc)))


def knn(probe_pos, lo, hi, pts, normals, k: int, radius: float = float("inf")):
    """Brute-force neighbour search: (idx [N,K] int32, w [N,K] float64)."""
    probe_pos, pp = _f(probe_pos)
    lo, plo = _f(lo)
    hi, phi = _f(hi)
    pts, px = _f(pts)
    normals, pn = _f(normals)
    N = pts.shape[0]
    idx = np.zeros((N, k), np.int32)
    w = np.zeros((N, k))
    lib().orc_knn(pp, probe_pos.shape[0], plo, phi, px, pn, N, k, C.c_float(radius),
                  idx.ctypes.data_as(iptr), w.ctypes.data_as(dptr))
    return idx, w


def query(tex, idx, w, dirs):
    """Eq. 9 at world directions dirs [N,D,3]: (Lin [N,D,3], O [N,D])."""
    tex, pt = _d(tex)
    idx, pi = _i(idx)
    w, pw = _d(w)
    dirs, pd = _d(dirs)
    N, D = dirs.shape[0], dirs.shape[1]
    Lin = np.zeros((N, D, 3))
    O = np.zeros((N, D))
    lib().orc_query(pt, tex.shape[1], pi, pw, idx.shape[1], N, pd, D,
                    Lin.ctypes.data_as(dptr), O.ctypes.data_as(dptr))
    return Lin, O


def _scene_args(sc, albedo=None, rough=None, metal=None, texels=None, env=None):
    keep = []

    def d(a):
        a2, p = _d(a)
        keep.append(a2)
        return a2, p

    pos, ppos = d(sc.pos)
    _, pn = d(sc.normal)
    if sc.view is not None:
        _, pv = d(sc.view)
        pc, ppf = None, 1
    else:
        pv = None
        _, pc = d(sc.cam_pos)
        ppf = sc.points_per_frame
    _, pa = d(sc.albedo if albedo is None else albedo)
    _, pr = d(sc.rough if rough is None else rough)
    _, pm = d(sc.metal if metal is None else metal)
    tex, ptex = d(sc.texels.astype(np.float64) if texels is None else texels)
    envd, penv = d(sc.env if env is None else env)
    return keep, (pos.shape[0], ppos, pn, pv, pc, ppf, pa, pr, pm, ptex, tex.shape[1], penv,
                  envd.shape[0], envd.shape[1])


def shade(sc, idx, w, albedo=None, rough=None, metal=None, texels=None, env=None,
          n_dirs=None, seed=None, per_point=False, irradiance=False):
    """Oracle shading of a ShadeScene (or a scene with overridden inputs) with neighbour
    lists (idx, w) from :func:`knn`. Returns rgb [N,3] (and irradiance [N,3])."""
    keep, a = _scene_args(sc, albedo, rough, metal, texels, env)
    idx, pi = _i(idx)
    w, pw = _d(w)
    N = a[0]
    rgb = np.zeros((N, 3))
    irr = np.zeros((N, 3)) if irradiance else None
    S = sc.n_dirs if n_dirs is None else n_dirs
    sd = sc.seed if seed is None else seed
    lib().orc_shade(*a, pi, pw, idx.shape[1], S, sd, int(per_point),
                    rgb.ctypes.data_as(dptr), irr.ctypes.data_as(dptr) if irradiance else None)
    del keep
    return (rgb, irr) if irradiance else rgb


def shade_backward(sc, idx, w, grad, albedo=None, rough=None, metal=None, texels=None,
                   env=None, n_dirs=None, seed=None, per_point=False, mass=False):
    """Analytic adjoint: dict with g_albedo [N,3], g_rough [N], g_metal [N],
    g_tex [P,R,R,4], g_env [H,W,3] (texture gradients start from zero). With mass=True
    also m_* arrays of the same shapes: the sum of |term| of every gradient entry."""
    keep, a = _scene_args(sc, albedo, rough, metal, texels, env)
    idx, pi = _i(idx)
    w, pw = _d(w)
    grad, pg = _d(grad)
    N = a[0]
    out = {
        "g_albedo": np.zeros((N, 3)), "g_rough": np.zeros(N), "g_metal": np.zeros(N),
        "g_tex": np.zeros(sc.texels.shape, np.float64),
        "g_env": np.zeros((sc.env if env is None else env).shape, np.float64),
    }
    keys = ("albedo", "rough", "metal", "tex", "env")
    if mass:
        for k in keys:
            out["m_" + k] = np.zeros_like(out["g_" + k])
    S = sc.n_dirs if n_dirs is None else n_dirs
    sd = sc.seed if seed is None else seed
    lib().orc_shade_backward(*a, pi, pw, idx.shape[1], S, sd, int(per_point), pg,
                             *(out["g_" + k].ctypes.data_as(dptr) for k in keys),
                             *((out["m_" + k].ctypes.data_as(dptr) if mass else None)
                               for k in keys))
    del keep
    return out


def bake_rays(gs, probe_pos, res, ray_probe, ray_texel, t_min=0.0, alpha_min=1.0 / 255.0,
              alpha_max=0.99, T_min=1e-4, used=False):
    """Brute-force trace of the given (probe, texel) rays through every Gaussian.
    Returns (out [n,5] = R,G,B,O,depth ; ambiguous [n] bool), and with used=True also the
    number of accepted Gaussians each ray resolves (up to and including the one ending it)."""
    keep = []

    def d(a):
        a2, p = _d(a)
        keep.append(a2)
        return p

    ray_probe, prp = _i(ray_probe)
    ray_texel, prt = _i(ray_texel)
    n = ray_probe.shape[0]
    out = np.zeros((n, 5))
    flags = np.zeros(n, np.int32)
    n_used = np.zeros(n, np.int32)
    lib().orc_bake_rays(gs.count, d(gs.mean), d(gs.scale), d(gs.rotation), d(gs.opacity),
                        d(gs.color), d(probe_pos), res, n, prp, prt, t_min, alpha_min,
                        alpha_max, T_min, out.ctypes.data_as(dptr),
                        flags.ctypes.data_as(iptr), n_used.ctypes.data_as(iptr))
    if used:
        return out, flags.astype(bool), n_used
    return out, flags.astype(bool)
