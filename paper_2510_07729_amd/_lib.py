"""ctypes declarations of include/sop.h and the loader of libsop.so.

There is no fallback: if the HIP library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
# SOP_LIBRARY names another build of the same library to load instead (for instance one
# whose host code carries sanitizers); it must exist like the in-tree one.
LIB_PATH = os.environ.get("SOP_LIBRARY") or os.path.join(HERE, "libsop.so")

c_i32, c_i64, c_u32, c_f32, c_vp = C.c_int32, C.c_int64, C.c_uint32, C.c_float, C.c_void_p

SOP_OK = 0
SOP_ERR_INVALID_ARGUMENT = 1
SOP_ERR_UNSUPPORTED = 2
SOP_ERR_WORKSPACE_TOO_SMALL = 3
SOP_ERR_DEVICE = 4
SOP_ERR_OUT_OF_MEMORY = 5

SOP_TEXEL_F32 = 0
SOP_TEXEL_F16 = 1

SOP_OP_KNN, SOP_OP_QUERY, SOP_OP_SHADE, SOP_OP_SHADE_BACKWARD = 0, 1, 2, 3
SOP_OP_DUMP_INTEGRAND, SOP_OP_PROPOSAL_INFER, SOP_OP_PROPOSAL_TRAIN = 4, 5, 6
SOP_SAMPLER_HAMMERSLEY, SOP_SAMPLER_PROPOSAL, SOP_SAMPLER_PROPOSAL_NET = 0, 1, 2
SOP_SAMPLER_ENV, SOP_SAMPLER_ENV_EXACT, SOP_SAMPLER_COSINE = 3, 4, 5
SOP_MLP_IN, SOP_MLP_HIDDEN, SOP_MLP_BINS, SOP_MLP_PARAMS = 320, 64, 256, 41344
SOP_SHADOW_HAMMERSLEY, SOP_SHADOW_ENV, SOP_SHADOW_ENV_EXACT = 0, 1, 2
SOP_ENV_EQUIRECT, SOP_ENV_OCTAHEDRAL = 0, 1
SOP_NOALLOC_SCRATCH_BYTES = 32 << 20


class sop_probe_set(C.Structure):
    _fields_ = [("count", c_i32), ("pos", c_vp), ("bounds_lo", c_f32 * 3),
                ("bounds_hi", c_f32 * 3)]


class sop_probe_maps(C.Structure):
    _fields_ = [("res", c_i32), ("format", c_i32), ("texels", c_vp)]


class sop_envmap(C.Structure):
    _fields_ = [("height", c_i32), ("width", c_i32), ("texels", c_vp), ("layout", c_i32)]


class sop_points(C.Structure):
    _fields_ = [("count", c_i64), ("pos", c_vp), ("normal", c_vp), ("view", c_vp),
                ("cam_pos", c_vp), ("points_per_frame", c_i64), ("n_frames", c_i32),
                ("albedo", c_vp), ("roughness", c_vp), ("metallic", c_vp)]


class sop_neighbors(C.Structure):
    _fields_ = [("k", c_i32), ("order", c_vp), ("idx", c_vp), ("weight", c_vp)]


class sop_shade_opts(C.Structure):
    _fields_ = [("n_dirs", c_i32), ("k", c_i32), ("radius", c_f32), ("seed", c_u32),
                ("rotate_per_point", c_i32), ("sampler", c_i32), ("out_irradiance", c_vp),
                ("probs", c_vp), ("mix_eps", c_f32), ("net", c_vp)]


class sop_env_oct(C.Structure):
    _fields_ = [("res", c_i32), ("texels", c_vp)]


class sop_shadow_opts(C.Structure):
    _fields_ = [("n_dirs", c_i32), ("k", c_i32), ("radius", c_f32), ("seed", c_u32),
                ("rotate_per_point", c_i32), ("sampler", c_i32), ("out_irradiance", c_vp)]


class sop_gaussians(C.Structure):
    _fields_ = [("count", c_i32), ("mean", c_vp), ("scale", c_vp), ("rotation", c_vp),
                ("opacity", c_vp), ("color", c_vp)]


class sop_bake_opts(C.Structure):
    _fields_ = [("t_min", c_f32), ("alpha_min", c_f32), ("alpha_max", c_f32), ("T_min", c_f32),
                ("cell_scale", c_f32)]


class sop_mlp(C.Structure):
    _fields_ = [("params", c_vp), ("bounds_lo", c_f32 * 3), ("bounds_hi", c_f32 * 3)]


class sop_adam(C.Structure):
    _fields_ = [("lr", c_f32), ("beta1", c_f32), ("beta2", c_f32), ("eps", c_f32),
                ("step", c_i32)]


P = C.POINTER

# name -> (restype, argtypes); every symbol declared in include/sop.h
SIGNATURES = {
    "sop_plan_create": (c_i32, [P(sop_probe_set), c_vp, P(c_vp)]),
    "sop_plan_rebuild": (c_i32, [c_vp, c_vp, c_vp]),
    "sop_plan_destroy": (c_i32, [c_vp]),
    "sop_plan_info": (c_i32, [c_vp, P(c_i32), P(c_i32), P(c_f32)]),
    "sop_knn": (c_i32, [c_vp, P(sop_points), c_i32, c_f32, c_vp, c_vp, c_vp, c_vp, C.c_size_t,
                        c_vp]),
    "sop_query": (c_i32, [c_vp, P(sop_probe_maps), P(sop_points), P(sop_neighbors), c_vp,
                          c_i32, c_i32, c_f32, c_vp, c_vp, c_vp, C.c_size_t, c_vp]),
    "sop_shade": (c_i32, [c_vp, P(sop_probe_maps), P(sop_envmap), P(sop_points),
                          P(sop_neighbors), P(sop_shade_opts), c_vp, c_vp, C.c_size_t, c_vp]),
    "sop_shade_noalloc": (c_i32, [c_vp, P(sop_probe_maps), P(sop_envmap), P(sop_points),
                                  P(sop_neighbors), P(sop_shade_opts), c_vp, c_vp]),
    "sop_shade_backward": (c_i32, [c_vp, P(sop_probe_maps), P(sop_envmap), P(sop_points),
                                   P(sop_neighbors), P(sop_shade_opts), c_vp, c_vp, c_vp, c_vp,
                                   c_vp, c_vp, c_vp, C.c_size_t, c_vp]),
    "sop_shade_backward_deterministic": (c_i32, [c_vp, P(sop_probe_maps), P(sop_envmap),
                                                 P(sop_points), P(sop_neighbors),
                                                 P(sop_shade_opts), c_vp, c_vp, c_vp, c_vp,
                                                 c_vp, c_vp, c_vp, C.c_size_t, c_vp,
                                                 C.c_size_t, c_vp]),
    "sop_shade_backward_acc_size": (C.c_size_t, [c_i32, c_i32, c_i32, c_i32]),
    "sop_workspace_size": (C.c_size_t, [c_vp, c_i32, c_i64, c_i32, c_i32, c_i32, c_i32, c_i32]),
    "sop_bake_plan_create": (c_i32, [P(sop_gaussians), P(sop_bake_opts), c_vp, P(c_vp)]),
    "sop_bake_plan_update": (c_i32, [c_vp, P(sop_gaussians), c_vp]),
    "sop_bake_plan_check": (c_i32, [c_vp, c_vp]),
    "sop_bake_plan_destroy": (c_i32, [c_vp]),
    "sop_bake": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp]),
    "sop_shadow_ratio": (c_i32, [c_vp, P(sop_probe_maps), P(sop_env_oct), P(sop_points),
                                 P(sop_neighbors), P(sop_shadow_opts), c_vp, c_vp, C.c_size_t,
                                 c_vp]),
    "sop_shadow_workspace_size": (C.c_size_t, [c_vp, c_i64, c_i32, c_i32, c_i32, c_i32]),
    "sop_place_probes": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_i64, c_f32, c_vp, c_vp, c_vp,
                                 C.c_size_t, c_vp]),
    "sop_place_workspace_size": (C.c_size_t, [c_i64, c_i32]),
    "sop_sops_loss": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, C.c_size_t, c_vp]),
    "sop_lam_loss": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, C.c_size_t, c_vp]),
    "sop_loss_workspace_size": (C.c_size_t, [c_i64]),
    "sop_shade_traced": (c_i32, [c_vp, c_vp, P(sop_envmap), P(sop_points), P(sop_shade_opts),
                                 c_f32, c_vp, c_vp, c_vp, C.c_size_t, c_vp]),
    "sop_shade_traced_workspace_size": (C.c_size_t, [c_vp, c_i64, c_i32, c_i32, c_i32, c_i32]),
    "sop_proposal_workspace_size": (C.c_size_t, [c_i32, c_i64]),
    "sop_proposal_infer": (c_i32, [P(sop_mlp), P(sop_points), c_vp, c_vp, c_vp, C.c_size_t,
                                   c_vp]),
    "sop_proposal_train_step": (c_i32, [P(sop_mlp), P(sop_points), c_vp, P(sop_adam), c_vp,
                                        c_vp, c_vp, c_vp, c_vp, C.c_size_t, c_vp]),
    "sop_adam_update": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i64, P(sop_adam), c_vp]),
    "sop_dump_integrand": (c_i32, [c_vp, P(sop_probe_maps), P(sop_envmap), P(sop_points),
                                   P(sop_neighbors), P(sop_shade_opts), c_i32, c_vp, c_vp,
                                   C.c_size_t, c_vp]),
    "sop_status_string": (C.c_char_p, [c_i32]),
    "sop_last_error": (C.c_char_p, []),
    "sop_version": (c_i32, []),
}

_lock = threading.Lock()
_lib = None


class SopError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn}: status {status}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    """Loads libsop.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise RuntimeError(
                    f"{path} is missing: build the HIP library first "
                    "(python -m paper_2510_07729_amd.build)")
            lib = C.CDLL(path)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def check(status: int, fn: str) -> None:
    if status != SOP_OK:
        lib = load()
        raise SopError(status, fn, lib.sop_last_error().decode())
