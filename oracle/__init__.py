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
_SRCS = [_SRC, os.path.join(_HERE, "proposal_oracle.c"), os.path.join(_HERE, "shadow_oracle.c"),
         os.path.join(_HERE, "placement_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (always when force, else only if missing or stale)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, *_SRCS, "-lm"])
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
                              dptr, C.c_int, dptr, C.c_int, C.c_int, C.c_int, iptr, dptr,
                              C.c_int, C.c_int, u32, C.c_int, dptr, dptr]
    lib.orc_shade_cosine.argtypes = lib.orc_shade.argtypes
    lib.orc_direction_cos.restype = C.c_double
    lib.orc_direction_cos.argtypes = [C.c_int, C.c_int, u32, dptr, dptr]
    lib.orc_shade_backward.argtypes = [C.c_long, dptr, dptr, dptr, dptr, C.c_long, dptr, dptr,
                                       dptr, dptr, C.c_int, dptr, C.c_int, C.c_int, C.c_int,
                                       iptr,
                                       dptr, C.c_int, C.c_int, u32, C.c_int, dptr, dptr, dptr,
                                       dptr, dptr, dptr, dptr, dptr, dptr, dptr, dptr]
    u64 = C.c_uint64
    u32p = C.POINTER(u32)
    fl = C.c_float
    lib.orc_mlp_param_count.restype = C.c_int
    lib.orc_bf16.restype = C.c_double
    lib.orc_bf16.argtypes = [C.c_double]
    lib.orc_pe_features.argtypes = [dptr, dptr, dptr, C.c_double, dptr, dptr, dptr]
    lib.orc_mlp_forward.argtypes = [dptr, dptr, C.c_int] + [dptr] * 7
    lib.orc_mlp_infer.argtypes = [dptr, C.c_long, dptr, dptr, dptr, dptr, dptr, dptr, C.c_int,
                                  dptr, dptr]
    lib.orc_mlp_loss_grad.argtypes = [dptr, C.c_long, dptr, dptr, dptr, dptr, dptr, dptr, dptr,
                                      C.c_int, dptr, dptr, dptr]
    lib.orc_adam.argtypes = [C.c_long, dptr, dptr, dptr, dptr, C.c_double, C.c_double,
                             C.c_double, C.c_double, C.c_int]
    lib.orc_hash24.restype = u32
    lib.orc_hash24.argtypes = [u32, u32, u32, u32]
    lib.orc_prop_masses.restype = u64
    lib.orc_prop_masses.argtypes = [fptr, fl, u32p]
    lib.orc_prop_bin.restype = C.c_int
    lib.orc_prop_bin.argtypes = [dptr, dptr]
    lib.orc_prop_pdf.restype = C.c_double
    lib.orc_prop_pdf.argtypes = [fptr, fl, dptr]
    lib.orc_prop_samples.argtypes = [fptr, fl, C.c_int, u32, u32, iptr, dptr, dptr]
    lib.orc_prop_shade.argtypes = [C.c_long, dptr, dptr, dptr, dptr, C.c_long, dptr, dptr, dptr,
                                   dptr, C.c_int, dptr, C.c_int, C.c_int, C.c_int, iptr, dptr,
                                   C.c_int,
                                   fptr, fl, C.c_int, u32, dptr, dptr]
    lib.orc_dump_integrand.argtypes = [C.c_long, dptr, dptr, dptr, dptr, C.c_long, dptr, dptr,
                                       dptr, dptr, C.c_int, dptr, C.c_int, C.c_int, C.c_int,
                                       iptr, dptr,
                                       C.c_int, C.c_int, u32, dptr]
    lib.orc_bake_rays.argtypes = [C.c_int, dptr, dptr, dptr, dptr, dptr, dptr, C.c_int,
                                  C.c_long, iptr, iptr, C.c_double, C.c_double, C.c_double,
                                  C.c_double, dptr, iptr, iptr]
    u64p = C.POINTER(C.c_uint64)
    lib.orc_env_masses.argtypes = [fptr, C.c_int, u32p, u64p]
    lib.orc_env_masses.restype = C.c_uint64
    lib.orc_env_draw.argtypes = [u32p, u64p, C.c_int, C.c_int, C.c_int, u32, u32, C.c_int,
                                 dptr, dptr]
    lib.orc_env_draw.restype = C.c_int
    lib.orc_shadow_ratio.argtypes = [C.c_long, dptr, dptr, C.c_int, iptr, dptr, C.c_int, fptr,
                                     C.c_int, C.c_int, u32, C.c_int, C.c_int, dptr, dptr, iptr,
                                     C.POINTER(C.c_uint32)]
    lib.orc_shade_envis.argtypes = [C.c_long, dptr, dptr, dptr, dptr, C.c_long, dptr, dptr,
                                    dptr, dptr, C.c_int, iptr, dptr, C.c_int, fptr, C.c_int,
                                    C.c_int, u32, C.POINTER(C.c_uint32), C.c_int, dptr, dptr,
                                    iptr]
    lib.orc_fps.argtypes = [fptr, C.c_long, C.c_int, C.c_long, iptr]
    lib.orc_place.argtypes = [fptr, fptr, iptr, C.c_int, C.c_float, fptr]
    lib.orc_sops_loss.argtypes = [fptr, fptr, C.c_long, dptr, dptr]
    lib.orc_lam_loss.argtypes = [fptr, fptr, C.c_long, dptr, dptr, dptr]
    lib.orc_shade_traced.argtypes = [C.c_int, dptr, dptr, dptr, dptr, dptr, C.c_long, dptr,
                                     dptr, dptr, dptr, C.c_long, dptr, dptr, dptr, dptr,
                                     C.c_int, C.c_int, C.c_int, C.c_int, u32, C.c_int,
                                     C.c_float,
                                     C.c_double, C.c_double, C.c_double, C.c_double, dptr,
                                     dptr, dptr, iptr]


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
    # octahedral environments are read like probe maps (H = W = their side)
    return keep, (pos.shape[0], ppos, pn, pv, pc, ppf, pa, pr, pm, ptex, tex.shape[1], penv,
                  envd.shape[0], envd.shape[1], int(getattr(sc, "env_oct", False)))


def shade(sc, idx, w, albedo=None, rough=None, metal=None, texels=None, env=None,
          n_dirs=None, seed=None, per_point=False, irradiance=False, cosine=False):
    """Oracle shading of a ShadeScene (or a scene with overridden inputs) with neighbour
    lists (idx, w) from :func:`knn`. Returns rgb [N,3] (and irradiance [N,3]). cosine=True
    takes the cosine-weighted direction set (orc_shade_cosine)."""
    keep, a = _scene_args(sc, albedo, rough, metal, texels, env)
    idx, pi = _i(idx)
    w, pw = _d(w)
    N = a[0]
    rgb = np.zeros((N, 3))
    irr = np.zeros((N, 3)) if irradiance else None
    S = sc.n_dirs if n_dirs is None else n_dirs
    sd = sc.seed if seed is None else seed
    fn = lib().orc_shade_cosine if cosine else lib().orc_shade
    fn(*a, pi, pw, idx.shape[1], S, sd, int(per_point),
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



def shade_traced(gs, sc, offset, n_dirs=None, seed=None, per_point=False, t_min=0.0,
                 alpha_min=1.0 / 255.0, alpha_max=0.99, T_min=1e-4, env=None):
    """Traced shading of the points of ShadeScene ``sc`` through Gaussians ``gs``: every
    sample's O and L_in from its own ray, starting at fmaf(offset, n, x) (float32).
    Returns a dict: rgb [N,3], irr [N,3], samples [N,S,4] (R,G,B,O), ray_amb [N,S] and
    amb [N] (some ray of the point is ambiguous)."""
    keep = []

    def d(a):
        a2, p = _d(a)
        keep.append(a2)
        return p

    N = sc.pos.shape[0]
    S = sc.n_dirs if n_dirs is None else n_dirs
    sd = sc.seed if seed is None else seed
    envd = np.ascontiguousarray(sc.env if env is None else env, dtype=np.float64)
    keep.append(envd)
    if sc.view is not None:
        pv, pc, ppf = d(sc.view), None, 1
    else:
        pv, pc, ppf = None, d(sc.cam_pos), sc.points_per_frame
    rgb = np.zeros((N, 3))
    irr = np.zeros((N, 3))
    samples = np.zeros((N, S, 4))
    flags = np.zeros((N, S), np.int32)
    lib().orc_shade_traced(gs.count, d(gs.mean), d(gs.scale), d(gs.rotation), d(gs.opacity),
                           d(gs.color), N, d(sc.pos), d(sc.normal), pv, pc, ppf,
                           d(sc.albedo), d(sc.rough), d(sc.metal), envd.ctypes.data_as(dptr),
                           envd.shape[0], envd.shape[1], int(getattr(sc, "env_oct", False)), S,
                           sd & 0xFFFFFFFF, int(per_point),
                           float(offset), t_min, alpha_min, alpha_max, T_min,
                           rgb.ctypes.data_as(dptr), irr.ctypes.data_as(dptr),
                           samples.ctypes.data_as(dptr), flags.ctypes.data_as(iptr))
    del keep
    amb = flags.astype(bool)
    return {"rgb": rgb, "irr": irr, "samples": samples, "ray_amb": amb, "amb": amb.any(axis=1)}



# ------------------------------------------------------------------------------------------
# cast-shadow ratio (Eq. 15-18) on an octahedral environment map
# ------------------------------------------------------------------------------------------
def env_masses(env):
    """Integer texel masses of an octahedral environment [R,R,3] (float32 decisions):
    (mass [R*R] uint32, prefix [R*R+1] uint64)."""
    env = np.ascontiguousarray(env, np.float32)
    R = env.shape[0]
    mass = np.zeros(R * R, np.uint32)
    prefix = np.zeros(R * R + 1, np.uint64)
    lib().orc_env_masses(env.ctypes.data_as(fptr), R, mass.ctypes.data_as(C.POINTER(C.c_uint32)),
                         prefix.ctypes.data_as(C.POINTER(C.c_uint64)))
    return mass, prefix


def env_draw(mass, prefix, R, S, j, seed, i, exact=False):
    """Draw j of S for point i: (texel, direction [3], pdf); pdf of Eq. 18, or with exact
    the draw's own density on the octahedral map."""
    mass = np.ascontiguousarray(mass, np.uint32)
    prefix = np.ascontiguousarray(prefix, np.uint64)
    w = np.zeros(3)
    pdf = C.c_double()
    t = lib().orc_env_draw(mass.ctypes.data_as(C.POINTER(C.c_uint32)),
                           prefix.ctypes.data_as(C.POINTER(C.c_uint64)), R, S, j,
                           seed & 0xFFFFFFFF, i & 0xFFFFFFFF, int(bool(exact)),
                           w.ctypes.data_as(dptr), C.byref(pdf))
    return t, w, pdf.value


def shadow_ratio(normal, texels, idx, w, env, S, seed=0, per_point=False, sampler=0,
                 ids=None):
    """Cast-shadow ratio of the points with normals [N,3]: probe maps [P,R,R,4] (channel 3 =
    the object's occlusion O'), neighbours (idx, w) [N,K], octahedral environment [Re,Re,3].
    sampler 0 = Hammersley, 1 = environment importance sampling with the density of Eq. 18,
    2 = the same draws weighted by their exact density. Returns a dict with ratio
    [N,3], irr [N,3] (the unshadowed estimate) and texels [N,S] (importance draws). ids:
    the points' indices in the full set they come from (keys of draws and rotations)."""
    normal, pn = _d(normal)
    tex, pt = _d(np.asarray(texels, np.float64))
    idx, pi = _i(idx)
    w, pw = _d(w)
    env, pe = _f(env)
    N = normal.shape[0]
    ratio = np.zeros((N, 3))
    irr = np.zeros((N, 3))
    tx = np.zeros((N, S), np.int32)
    lib().orc_shadow_ratio(N, pn, pt, tex.shape[1], pi, pw, idx.shape[1], pe, env.shape[0], S,
                           seed & 0xFFFFFFFF, int(per_point), int(sampler),
                           ratio.ctypes.data_as(dptr), irr.ctypes.data_as(dptr),
                           tx.ctypes.data_as(iptr),
                           None if ids is None else
                           np.ascontiguousarray(ids, np.uint32).ctypes.data_as(
                               C.POINTER(C.c_uint32)))
    return {"ratio": ratio, "irr": irr, "texels": tx}


def shade_envis(sc, idx, w, n_dirs=None, seed=None, ids=None, irradiance=False, texels_out=False,
                texels=None, env=None, exact=False):
    """Relighting of a ShadeScene with environment importance sampling (Eq. 18 draws and
    density on the octahedral environment sc.env [Re,Re,3]; with exact, the draws' exact
    density) instead of the Hammersley set. Returns rgb [N,3] (and irradiance [N,3], and the
    texel of every draw [N,S])."""
    keep = []

    def d(a):
        a2, p = _d(a)
        keep.append(a2)
        return p

    N = sc.pos.shape[0]
    S = sc.n_dirs if n_dirs is None else n_dirs
    sd = sc.seed if seed is None else seed
    envf, pe = _f(sc.env if env is None else env)
    tex = sc.texels.astype(np.float64) if texels is None else np.asarray(texels, np.float64)
    idx, pi = _i(idx)
    w, pw = _d(w)
    if sc.view is not None:
        pv, pc, ppf = d(sc.view), None, 1
    else:
        pv, pc, ppf = None, d(sc.cam_pos), sc.points_per_frame
    rgb = np.zeros((N, 3))
    irr = np.zeros((N, 3))
    tx = np.zeros((N, S), np.int32)
    idp = None
    if ids is not None:
        ida = np.ascontiguousarray(ids, np.uint32)
        keep.append(ida)
        idp = ida.ctypes.data_as(C.POINTER(C.c_uint32))
    lib().orc_shade_envis(N, d(sc.pos), d(sc.normal), pv, pc, ppf, d(sc.albedo), d(sc.rough),
                          d(sc.metal), d(tex), tex.shape[1], pi, pw, idx.shape[1], pe,
                          envf.shape[0], S, sd & 0xFFFFFFFF, idp, int(bool(exact)),
                          rgb.ctypes.data_as(dptr),
                          irr.ctypes.data_as(dptr), tx.ctypes.data_as(iptr))
    del keep
    out = (rgb,) + ((irr,) if irradiance else ()) + ((tx,) if texels_out else ())
    return out[0] if len(out) == 1 else out


# ------------------------------------------------------------------------------------------
# probe placement (farthest point sampling + normal offset) and the L_lam / L_sops losses
# ------------------------------------------------------------------------------------------
def fps(pts, P, start=0):
    """Indices [P] of the farthest point sampling of pts [M,3] (float32 decisions)."""
    pts, pp = _f(pts)
    out = np.zeros(P, np.int32)
    lib().orc_fps(pp, pts.shape[0], P, int(start), out.ctypes.data_as(iptr))
    return out


def place(pts, normals, chosen, offset):
    """Probe positions [P,3] = fmaf(offset, n, x) of the chosen points (float32)."""
    pts, pp = _f(pts)
    normals, pn = _f(normals)
    chosen, pc = _i(chosen)
    out = np.zeros((chosen.shape[0], 3), np.float32)
    lib().orc_place(pp, pn, pc, chosen.shape[0], float(offset), out.ctypes.data_as(fptr))
    return out


def sops_loss(tex, target):
    """(loss [2] = (L1(L_in, L_tr), L1(O, O_tr)), grad [...,4]) of probe textures."""
    tex, pt = _f(tex)
    target, pg = _f(target)
    T = tex.size // 4
    loss = np.zeros(2)
    grad = np.zeros(tex.shape)
    lib().orc_sops_loss(pt, pg, T, loss.ctypes.data_as(dptr), grad.ctypes.data_as(dptr))
    return loss, grad


def lam_loss(rough, metal):
    """(loss [2] = (L1(R, 1), L1(M, 0)), g_rough [N], g_metal [N])."""
    rough, pr = _f(rough)
    metal, pm = _f(metal)
    N = rough.shape[0]
    loss = np.zeros(2)
    gr, gm = np.zeros(N), np.zeros(N)
    lib().orc_lam_loss(pr, pm, N, loss.ctypes.data_as(dptr), gr.ctypes.data_as(dptr),
                       gm.ctypes.data_as(dptr))
    return loss, gr, gm

# ------------------------------------------------------------------------------------------
# learned direction proposal (features, network, training, bin sampler, shading, targets)
# ------------------------------------------------------------------------------------------
MLP_IN, MLP_HIDDEN, MLP_BINS = 320, 64, 256


def mlp_param_count() -> int:
    return int(lib().orc_mlp_param_count())


def mlp_offsets() -> dict:
    """Slices of the parameter blob: W1 [320,64], b1, W2 [64,64], b2, W3 [64,256], b3."""
    sizes = [("W1", MLP_IN * MLP_HIDDEN), ("b1", MLP_HIDDEN), ("W2", MLP_HIDDEN * MLP_HIDDEN),
             ("b2", MLP_HIDDEN), ("W3", MLP_HIDDEN * MLP_BINS), ("b3", MLP_BINS)]
    out, o = {}, 0
    for name, n in sizes:
        out[name] = slice(o, o + n)
        o += n
    return out


def bf16(x: float) -> float:
    return float(lib().orc_bf16(float(x)))


def pe_features(pos, n, v, r, lo, hi):
    """320 sinusoidal features of one point."""
    out = np.zeros(MLP_IN)
    a = [_d(x) for x in (pos, n, v)]
    lo_, plo = _d(lo)
    hi_, phi = _d(hi)
    lib().orc_pe_features(a[0][1], a[1][1], a[2][1], float(r), plo, phi,
                          out.ctypes.data_as(dptr))
    return out


def mlp_forward(params, feat, emulate_bf16=True):
    """dict of a0, z1, h1, z2, h2, z3 (logits), q (softmax) for one feature vector."""
    P, pp = _d(params)
    f, pf = _d(feat)
    out = {k: np.zeros(n) for k, n in (("a0", MLP_IN), ("z1", 64), ("h1", 64), ("z2", 64),
                                       ("h2", 64), ("z3", MLP_BINS), ("q", MLP_BINS))}
    lib().orc_mlp_forward(pp, pf, int(emulate_bf16),
                          *(out[k].ctypes.data_as(dptr) for k in ("a0", "z1", "h1", "z2", "h2",
                                                                  "z3", "q")))
    return out


def _pts(pos, normal, view, rough):
    arrs = [_d(pos), _d(normal), _d(view), _d(rough)]
    return [a for a, _ in arrs], [p for _, p in arrs]


def mlp_infer(params, pos, normal, view, rough, lo, hi, emulate_bf16=True):
    """(logits [N,256], probs [N,256]) of the proposal network."""
    P, pp = _d(params)
    keep, ptrs = _pts(pos, normal, view, rough)
    lo_, plo = _d(lo)
    hi_, phi = _d(hi)
    N = keep[0].shape[0]
    logits = np.zeros((N, MLP_BINS))
    probs = np.zeros((N, MLP_BINS))
    lib().orc_mlp_infer(pp, N, *ptrs, plo, phi, int(emulate_bf16),
                        logits.ctypes.data_as(dptr), probs.ctypes.data_as(dptr))
    return logits, probs


def mlp_loss_grad(params, pos, normal, view, rough, lo, hi, targets, emulate_bf16=True,
                  mass=False):
    """(loss, grad [P]) of the mean cross entropy against row-normalised targets [B,256];
    with mass=True (loss, grad, mass [P]), mass = the sum of |terms| of each entry."""
    P, pp = _d(params)
    keep, ptrs = _pts(pos, normal, view, rough)
    lo_, plo = _d(lo)
    hi_, phi = _d(hi)
    T, pt = _d(targets)
    grad = np.zeros(P.shape[0])
    m = np.zeros(P.shape[0]) if mass else None
    loss = np.zeros(1)
    lib().orc_mlp_loss_grad(pp, keep[0].shape[0], *ptrs, plo, phi, pt, int(emulate_bf16),
                            grad.ctypes.data_as(dptr), loss.ctypes.data_as(dptr),
                            m.ctypes.data_as(dptr) if mass else None)
    return (float(loss[0]), grad, m) if mass else (float(loss[0]), grad)


def adam(params, m, v, grad, lr, beta1, beta2, eps, step):
    """One Adam update in place on float64 arrays."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g, pg = _d(grad)
    lib().orc_adam(params.shape[0], params.ctypes.data_as(dptr), m.ctypes.data_as(dptr),
                   v.ctypes.data_as(dptr), pg, lr, beta1, beta2, eps, int(step))


def hash24(seed, i, j, k) -> int:
    return int(lib().orc_hash24(seed, i, j, k))


def prop_masses(probs, eps):
    """(integer bin masses [256] uint32, total)"""
    p, pp = _f(probs)
    c = np.zeros(MLP_BINS, np.uint32)
    total = lib().orc_prop_masses(pp, eps, c.ctypes.data_as(C.POINTER(C.c_uint32)))
    return c, int(total)


def prop_bin(wl):
    a, p = _d(wl)
    uv = np.zeros(2)
    b = lib().orc_prop_bin(p, uv.ctypes.data_as(dptr))
    return int(b), uv


def prop_pdf(probs, eps, wl) -> float:
    p, pp = _f(probs)
    a, pw = _d(wl)
    return float(lib().orc_prop_pdf(pp, eps, pw))


def prop_samples(probs, eps, S, seed, i):
    """(bins [S], local directions [S,3], densities [S]) of point i's draws."""
    p, pp = _f(probs)
    bins = np.zeros(S, np.int32)
    wl = np.zeros((S, 3))
    pdf = np.zeros(S)
    lib().orc_prop_samples(pp, eps, S, seed, i, bins.ctypes.data_as(iptr),
                           wl.ctypes.data_as(dptr), pdf.ctypes.data_as(dptr))
    return bins, wl, pdf


def prop_shade(sc, idx, w, probs, eps, n_dirs, seed, albedo=None, rough=None, metal=None,
               texels=None, env=None, irradiance=False):
    """Proposal-sampled shading of a ShadeScene with probs [N,256] (float32 decisions)."""
    keep, a = _scene_args(sc, albedo, rough, metal, texels, env)
    idx, pi = _i(idx)
    w, pw = _d(w)
    pr, ppr = _f(probs)
    N = a[0]
    rgb = np.zeros((N, 3))
    irr = np.zeros((N, 3)) if irradiance else None
    lib().orc_prop_shade(*a, pi, pw, idx.shape[1], ppr, eps, n_dirs, seed,
                         rgb.ctypes.data_as(dptr), irr.ctypes.data_as(dptr) if irradiance else None)
    del keep
    return (rgb, irr) if irradiance else rgb


def dump_integrand(sc, idx, w, samples_per_bin, seed, albedo=None, rough=None, metal=None,
                   texels=None, env=None):
    """Per-point bin integrals [N,256] of lum(f L_i cos) (training targets)."""
    keep, a = _scene_args(sc, albedo, rough, metal, texels, env)
    idx, pi = _i(idx)
    w, pw = _d(w)
    N = a[0]
    T = np.zeros((N, MLP_BINS))
    lib().orc_dump_integrand(*a, pi, pw, idx.shape[1], samples_per_bin, seed,
                             T.ctypes.data_as(dptr))
    del keep
    return T
