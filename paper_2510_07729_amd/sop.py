"""Python binding of the SOP C ABI (include/sop.h) over torch tensors.

Argument marshalling only: tensors' device pointers and the current HIP stream go to
libsop.so, which does every step on the GPU. Tensors must be CUDA (HIP) tensors,
contiguous, float32 (texels may be float16). Names follow the C entry points.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
from typing import Optional

import torch

from . import _lib as L


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor], dtype=None, what: str = "tensor") -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{what} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise ValueError(f"{what} has dtype {t.dtype}")
    return t.data_ptr()


def _shape(t: Optional[torch.Tensor], shape, what: str, dtype=None) -> None:
    """Raises ValueError unless t (when given) has `shape` (None matches any size) and, when
    asked, `dtype`. The C ABI receives bare pointers and cannot check sizes itself: a
    mismatch here would otherwise become an out-of-bounds device access."""
    if t is None:
        return
    if t.dim() != len(shape) or any(s is not None and int(t.shape[i]) != int(s)
                                    for i, s in enumerate(shape)):
        want = "[" + ",".join("*" if s is None else str(int(s)) for s in shape) + "]"
        raise ValueError(f"{what} has shape {list(t.shape)}, expected {want}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what} has dtype {t.dtype}, expected {dtype}")


def workspace(nbytes: int, device) -> torch.Tensor:
    """A 256-byte-aligned byte buffer of at least nbytes (the tensor may be larger)."""
    buf = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off: off + max(int(nbytes), 1)]


# ------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Points:
    """Shading points: pos/normal/albedo [N,3], rough/metal [N]; view [N,3] or camera
    positions cam_pos [F,3] with points_per_frame points per frame."""
    pos: torch.Tensor
    normal: torch.Tensor
    albedo: torch.Tensor
    rough: torch.Tensor
    metal: torch.Tensor
    view: Optional[torch.Tensor] = None
    cam_pos: Optional[torch.Tensor] = None
    points_per_frame: int = 0

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def check(self) -> None:
        """Every per-point array has N rows; camera mode needs F * points_per_frame == N."""
        n = self.n
        _shape(self.pos, (n, 3), "pos")
        _shape(self.normal, (n, 3), "normal")
        _shape(self.albedo, (n, 3), "albedo")
        _shape(self.rough, (n,), "rough")
        _shape(self.metal, (n,), "metal")
        _shape(self.view, (n, 3), "view")
        if self.view is None:
            if self.cam_pos is None:
                raise ValueError("points need view vectors or camera positions")
            _shape(self.cam_pos, (None, 3), "cam_pos")
            if int(self.cam_pos.shape[0]) * int(self.points_per_frame) != n:
                raise ValueError("cam_pos rows * points_per_frame must equal the point count")

    def c(self) -> L.sop_points:
        self.check()
        f = torch.float32
        s = L.sop_points()
        s.count = self.n
        s.pos = _ptr(self.pos, f, "pos")
        s.normal = _ptr(self.normal, f, "normal")
        s.view = _ptr(self.view, f, "view")
        s.cam_pos = _ptr(self.cam_pos, f, "cam_pos")
        s.points_per_frame = int(self.points_per_frame)
        s.n_frames = int(self.cam_pos.shape[0]) if self.cam_pos is not None else 0
        s.albedo = _ptr(self.albedo, f, "albedo")
        s.roughness = _ptr(self.rough, f, "rough")
        s.metallic = _ptr(self.metal, f, "metal")
        return s


@dataclasses.dataclass
class Neighbors:
    order: torch.Tensor   # [N] int32
    idx: torch.Tensor     # [N,K] int32
    w: torch.Tensor       # [N,K] float32

    @property
    def k(self) -> int:
        return int(self.idx.shape[1])

    def check(self, n: Optional[int] = None) -> None:
        k = self.k
        rows = int(self.idx.shape[0]) if n is None else int(n)
        _shape(self.idx, (rows, k), "nb.idx")
        _shape(self.w, (rows, k), "nb.w")
        _shape(self.order, (rows,), "nb.order")

    def c(self, n: Optional[int] = None) -> L.sop_neighbors:
        self.check(n)
        s = L.sop_neighbors()
        s.k = self.k
        s.order = _ptr(self.order, torch.int32, "order")
        s.idx = _ptr(self.idx, torch.int32, "idx")
        s.weight = _ptr(self.w, torch.float32, "w")
        return s


def _maps_shape(tex: torch.Tensor, plan=None) -> None:
    if tex.dim() != 4 or tex.shape[1] != tex.shape[2] or tex.shape[3] != 4:
        raise ValueError("probe textures must be [P,R,R,4]")
    if plan is not None and int(tex.shape[0]) != int(plan.n_probes):
        raise ValueError(f"probe textures hold {int(tex.shape[0])} maps, the plan "
                         f"{int(plan.n_probes)} probes")


def _maps(tex: torch.Tensor, plan=None) -> L.sop_probe_maps:
    _maps_shape(tex, plan)
    m = L.sop_probe_maps()
    m.res = int(tex.shape[1])
    if tex.dtype == torch.float32:
        m.format = L.SOP_TEXEL_F32
    elif tex.dtype == torch.float16:
        m.format = L.SOP_TEXEL_F16
    else:
        raise ValueError("probe textures must be float32 or float16")
    m.texels = _ptr(tex, None, "texels")
    return m


class OctEnv:
    """An octahedral environment map [R,R,3] (+z at the centre, read like a probe map) for
    the shading calls, which otherwise take an equirectangular [H,W,3] tensor."""

    def __init__(self, texels: torch.Tensor):
        if texels.dim() != 3 or texels.shape[2] != 3 or texels.shape[0] != texels.shape[1]:
            raise ValueError("an octahedral env must be [R,R,3]")
        self.texels = texels

    @property
    def shape(self):
        return self.texels.shape


def _env_shape(env) -> None:
    t = env.texels if isinstance(env, OctEnv) else env
    if t.dim() != 3 or t.shape[2] != 3:
        raise ValueError("env must be [H,W,3]")


def _env(env) -> L.sop_envmap:
    _env_shape(env)
    oct_ = isinstance(env, OctEnv)
    t = env.texels if oct_ else env
    e = L.sop_envmap()
    e.height, e.width = int(t.shape[0]), int(t.shape[1])
    e.texels = _ptr(t, torch.float32, "env")
    e.layout = L.SOP_ENV_OCTAHEDRAL if oct_ else L.SOP_ENV_EQUIRECT
    return e


# ------------------------------------------------------------------------------------------
class Plan:
    """Probe grid for the neighbour search (sop_plan_create / sop_plan_destroy)."""

    def __init__(self, probe_pos: torch.Tensor, bounds_lo, bounds_hi):
        _shape(probe_pos, (None, 3), "probe_pos")
        self._lib = L.load()
        ps = L.sop_probe_set()
        ps.count = int(probe_pos.shape[0])
        ps.pos = _ptr(probe_pos, torch.float32, "probe_pos")
        ps.bounds_lo = (C.c_float * 3)(*[float(x) for x in bounds_lo])
        ps.bounds_hi = (C.c_float * 3)(*[float(x) for x in bounds_hi])
        h = C.c_void_p()
        L.check(self._lib.sop_plan_create(C.byref(ps), _stream(), C.byref(h)), "sop_plan_create")
        self.handle = h
        self.n_probes = ps.count
        self.device = probe_pos.device

    def rebuild(self, probe_pos: torch.Tensor) -> None:
        _shape(probe_pos, (self.n_probes, 3), "probe_pos")
        L.check(self._lib.sop_plan_rebuild(self.handle, _ptr(probe_pos, torch.float32, "pos"),
                                           _stream()), "sop_plan_rebuild")

    def info(self):
        n = C.c_int32()
        dims = (C.c_int32 * 3)()
        sc = C.c_float()
        L.check(self._lib.sop_plan_info(self.handle, C.byref(n), dims, C.byref(sc)),
                "sop_plan_info")
        return n.value, tuple(dims), sc.value

    def workspace_size(self, op: int, n: int, k: int, n_dirs: int = 1, env_hw=(0, 0),
                       with_neighbors: bool = False) -> int:
        return int(self._lib.sop_workspace_size(self.handle, op, n, k, n_dirs, int(env_hw[0]),
                                                int(env_hw[1]), int(with_neighbors)))

    def close(self) -> None:
        if getattr(self, "handle", None):
            self._lib.sop_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sop_knn(plan: Plan, pts: Points, k: int, radius: float = math.inf) -> Neighbors:
    dev = pts.pos.device
    n = pts.n
    _shape(pts.pos, (n, 3), "pos")
    _shape(pts.normal, (n, 3), "normal")
    order = torch.empty(n, dtype=torch.int32, device=dev)
    idx = torch.empty((n, k), dtype=torch.int32, device=dev)
    w = torch.empty((n, k), dtype=torch.float32, device=dev)
    ws = workspace(plan.workspace_size(L.SOP_OP_KNN, n, k), dev)
    cp = L.sop_points()
    cp.count = n
    cp.pos = _ptr(pts.pos, torch.float32, "pos")
    cp.normal = _ptr(pts.normal, torch.float32, "normal")
    L.check(plan._lib.sop_knn(plan.handle, C.byref(cp), k, radius, order.data_ptr(),
                              idx.data_ptr(), w.data_ptr(), ws.data_ptr(), ws.numel(),
                              _stream()), "sop_knn")
    return Neighbors(order, idx, w)


def sop_query(plan: Plan, texels: torch.Tensor, pts: Points, dirs: torch.Tensor,
              nb: Optional[Neighbors] = None, k: int = 4, radius: float = math.inf):
    """Eq. 9 at given world directions dirs [N,D,3]: returns (L_in [N,D,3], O [N,D])."""
    n, D = pts.n, int(dirs.shape[1]) if dirs.dim() == 3 else -1
    _shape(dirs, (n, None, 3), "dirs")
    pts.check()
    _maps_shape(texels, plan)
    if nb is not None:
        nb.check(n)
    dev = dirs.device
    Lin = torch.empty((n, D, 3), dtype=torch.float32, device=dev)
    O = torch.empty((n, D), dtype=torch.float32, device=dev)
    kk = nb.k if nb is not None else k
    ws = workspace(plan.workspace_size(L.SOP_OP_QUERY, n, kk, D, with_neighbors=nb is not None),
                   dev)
    m, cp = _maps(texels, plan), pts.c()
    nbc = nb.c(n) if nb is not None else None
    L.check(plan._lib.sop_query(plan.handle, C.byref(m), C.byref(cp),
                                C.byref(nbc) if nbc is not None else None,
                                _ptr(dirs, torch.float32, "dirs"), D, k, radius, Lin.data_ptr(),
                                O.data_ptr(), ws.data_ptr(), ws.numel(), _stream()), "sop_query")
    return Lin, O


def shade_opts(n_dirs: int, k: int, seed: int = 0, radius: float = math.inf,
               rotate_per_point: bool = False, irradiance: Optional[torch.Tensor] = None,
               probs: Optional[torch.Tensor] = None, mix_eps: float = 0.1, net=None,
               env_sampling=False, cosine: bool = False):
    """Shading options; `net` (an Mlp) selects the fused proposal sampler, env_sampling the
    environment importance sampler (True: Eq. 18's density, "exact": the draws' exact
    density), cosine the cosine-weighted direction set. The returned object keeps the
    network's C struct alive (attribute _net)."""
    o = L.sop_shade_opts()
    o.n_dirs, o.k, o.radius, o.seed = int(n_dirs), int(k), float(radius), int(seed) & 0xFFFFFFFF
    o.rotate_per_point = int(rotate_per_point)
    if cosine:
        if env_sampling or net is not None or probs is not None:
            raise ValueError("cosine is a direction set of its own: no probs, net or env_sampling")
        o.sampler = L.SOP_SAMPLER_COSINE
    elif env_sampling == "exact":
        o.sampler = L.SOP_SAMPLER_ENV_EXACT
    elif env_sampling:
        if env_sampling is not True:
            raise ValueError(f"env_sampling must be False, True or 'exact', not {env_sampling!r}")
        o.sampler = L.SOP_SAMPLER_ENV
    elif net is not None:
        o.sampler = L.SOP_SAMPLER_PROPOSAL_NET
        o._net = net.c()
        o.net = C.addressof(o._net)
    else:
        o.sampler = L.SOP_SAMPLER_HAMMERSLEY if probs is None else L.SOP_SAMPLER_PROPOSAL
    o.out_irradiance = _ptr(irradiance, torch.float32, "irradiance")
    o.probs = _ptr(probs, torch.float32, "probs")
    o.mix_eps = float(mix_eps)
    return o


def sop_shade(plan: Plan, texels: torch.Tensor, env: torch.Tensor, pts: Points, n_dirs: int,
              k: int = 4, nb: Optional[Neighbors] = None, seed: int = 0,
              radius: float = math.inf, rotate_per_point: bool = False,
              irradiance: bool = False, ws: Optional[torch.Tensor] = None,
              out: Optional[torch.Tensor] = None, probs: Optional[torch.Tensor] = None,
              mix_eps: float = 0.1, net=None, env_sampling=False, cosine: bool = False):
    """Forward shading: rgb [N,3] (and irradiance [N,3] when asked). With probs [N,256] the
    directions are drawn from those bin distributions (mixed with mix_eps of uniform bins);
    with net (an Mlp) from the network's distributions, evaluated inside the call; with
    env_sampling (env an OctEnv) by environment importance sampling (Eq. 18; "exact" weights
    the draws by their exact density); with cosine from the cosine-weighted set."""
    dev = pts.pos.device
    n = pts.n
    pts.check()
    _maps_shape(texels, plan)
    _env_shape(env)
    _shape(out, (n, 3), "out", torch.float32)
    _shape(probs, (n, L.SOP_MLP_BINS), "probs", torch.float32)
    if nb is not None:
        nb.check(n)
    rgb = out if out is not None else torch.empty((n, 3), dtype=torch.float32, device=dev)
    irr = torch.empty((n, 3), dtype=torch.float32, device=dev) if irradiance else None
    kk = nb.k if nb is not None else k
    if ws is None:
        ws = workspace(plan.workspace_size(L.SOP_OP_SHADE, n, kk, n_dirs, env.shape[:2],
                                           nb is not None), dev)
    o = shade_opts(n_dirs, kk, seed, radius, rotate_per_point, irr, probs, mix_eps, net,
                   env_sampling, cosine)
    m, e, cp = _maps(texels, plan), _env(env), pts.c()
    nbc = nb.c(n) if nb is not None else None
    L.check(plan._lib.sop_shade(plan.handle, C.byref(m), C.byref(e), C.byref(cp),
                                C.byref(nbc) if nbc is not None else None, C.byref(o),
                                _ptr(rgb, torch.float32, "rgb"), ws.data_ptr(), ws.numel(),
                                _stream()), "sop_shade")
    return (rgb, irr) if irradiance else rgb


def sop_shade_noalloc(plan: Plan, texels: torch.Tensor, env: torch.Tensor, pts: Points,
                      n_dirs: int, out: torch.Tensor, k: int = 4,
                      nb: Optional[Neighbors] = None, seed: int = 0, radius: float = math.inf,
                      rotate_per_point: bool = False,
                      irradiance: Optional[torch.Tensor] = None) -> torch.Tensor:
    """sop_shade into the caller's out [N,3] (and irradiance [N,3] when given) with the
    library's fixed device scratch instead of a workspace: the call allocates nothing."""
    n = pts.n
    pts.check()
    _maps_shape(texels, plan)
    _env_shape(env)
    _shape(out, (n, 3), "out", torch.float32)
    _shape(irradiance, (n, 3), "irradiance", torch.float32)
    if nb is not None:
        nb.check(n)
    kk = nb.k if nb is not None else k
    o = shade_opts(n_dirs, kk, seed, radius, rotate_per_point, irradiance)
    m, e, cp = _maps(texels, plan), _env(env), pts.c()
    nbc = nb.c(n) if nb is not None else None
    L.check(plan._lib.sop_shade_noalloc(plan.handle, C.byref(m), C.byref(e), C.byref(cp),
                                        C.byref(nbc) if nbc is not None else None, C.byref(o),
                                        _ptr(out, torch.float32, "out"), _stream()),
            "sop_shade_noalloc")
    return out


def sop_shade_backward(plan: Plan, texels: torch.Tensor, env: torch.Tensor, pts: Points,
                       grad_rgb: torch.Tensor, n_dirs: int, k: int = 4,
                       nb: Optional[Neighbors] = None, seed: int = 0,
                       radius: float = math.inf, rotate_per_point: bool = False,
                       want=("albedo", "rough", "metal", "env", "tex"),
                       g_env: Optional[torch.Tensor] = None,
                       g_tex: Optional[torch.Tensor] = None,
                       ws: Optional[torch.Tensor] = None, deterministic: bool = False,
                       acc: Optional[torch.Tensor] = None):
    """Adjoint: dict of gradients. g_env/g_tex accumulate into the given tensors (zeroed
    new ones otherwise); per-point gradients are fresh tensors. deterministic=True calls
    sop_shade_backward_deterministic (g_env/g_tex exact sums, the same bits on every run);
    acc is its accumulator (allocated when not given)."""
    dev = pts.pos.device
    n = pts.n
    pts.check()
    _maps_shape(texels, plan)
    _env_shape(env)
    _shape(grad_rgb, (n, 3), "grad_rgb", torch.float32)
    # the library adds float32 gradients over exactly these sizes
    _shape(g_env, tuple(env.shape), "g_env", torch.float32)
    _shape(g_tex, tuple(texels.shape), "g_tex", torch.float32)
    if nb is not None:
        nb.check(n)
    out = {}
    if "albedo" in want:
        out["albedo"] = torch.empty((n, 3), dtype=torch.float32, device=dev)
    if "rough" in want:
        out["rough"] = torch.empty(n, dtype=torch.float32, device=dev)
    if "metal" in want:
        out["metal"] = torch.empty(n, dtype=torch.float32, device=dev)
    if "env" in want:
        out["env"] = g_env if g_env is not None else torch.zeros(env.shape, dtype=torch.float32,
                                                                 device=dev)
    if "tex" in want:
        out["tex"] = g_tex if g_tex is not None else torch.zeros(
            texels.shape, dtype=torch.float32, device=dev)
    kk = nb.k if nb is not None else k
    if ws is None:
        ws = workspace(plan.workspace_size(L.SOP_OP_SHADE_BACKWARD, n, kk, n_dirs, env.shape[:2],
                                           nb is not None), dev)
    o = shade_opts(n_dirs, kk, seed, radius, rotate_per_point)
    m, e, cp = _maps(texels, plan), _env(env), pts.c()
    nbc = nb.c(n) if nb is not None else None
    g = grad_rgb.contiguous()
    if deterministic:
        et = env.texels if isinstance(env, OctEnv) else env
        need = plan._lib.sop_shade_backward_acc_size(int(plan.n_probes), int(texels.shape[1]),
                                                     int(et.shape[0]), int(et.shape[1]))
        if acc is None:
            acc = workspace(need, dev)
        elif acc.numel() < need:
            raise ValueError(f"acc holds {acc.numel()} bytes, the call needs {need}")
        L.check(plan._lib.sop_shade_backward_deterministic(
            plan.handle, C.byref(m), C.byref(e), C.byref(cp),
            C.byref(nbc) if nbc is not None else None, C.byref(o),
            _ptr(g, torch.float32, "grad"), _ptr(out.get("albedo")), _ptr(out.get("rough")),
            _ptr(out.get("metal")), _ptr(out.get("env")), _ptr(out.get("tex")), ws.data_ptr(),
            ws.numel(), acc.data_ptr(), acc.numel(), _stream()),
            "sop_shade_backward_deterministic")
        return out
    L.check(plan._lib.sop_shade_backward(
        plan.handle, C.byref(m), C.byref(e), C.byref(cp),
        C.byref(nbc) if nbc is not None else None, C.byref(o), _ptr(g, torch.float32, "grad"),
        _ptr(out.get("albedo")), _ptr(out.get("rough")), _ptr(out.get("metal")),
        _ptr(out.get("env")), _ptr(out.get("tex")), ws.data_ptr(), ws.numel(), _stream()),
        "sop_shade_backward")
    return out


# ------------------------------------------------------------------------------------------
# learned direction proposal
# ------------------------------------------------------------------------------------------
def sop_dump_integrand(plan: Plan, texels: torch.Tensor, env: torch.Tensor, pts: Points,
                       samples_per_bin: int, k: int = 4, nb: Optional[Neighbors] = None,
                       seed: int = 0, radius: float = math.inf,
                       out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None):
    """Training targets [N,256]: per-bin integrals of the luminance of f L_i cos."""
    dev = pts.pos.device
    n = pts.n
    pts.check()
    _maps_shape(texels, plan)
    _env_shape(env)
    _shape(out, (n, L.SOP_MLP_BINS), "out", torch.float32)
    if nb is not None:
        nb.check(n)
    T = out if out is not None else torch.empty((n, L.SOP_MLP_BINS), dtype=torch.float32,
                                                device=dev)
    kk = nb.k if nb is not None else k
    if ws is None:
        ws = workspace(plan.workspace_size(L.SOP_OP_DUMP_INTEGRAND, n, kk, 1, env.shape[:2],
                                           nb is not None), dev)
    o = shade_opts(1, kk, seed, radius)
    m, e, cp = _maps(texels, plan), _env(env), pts.c()
    nbc = nb.c(n) if nb is not None else None
    L.check(plan._lib.sop_dump_integrand(
        plan.handle, C.byref(m), C.byref(e), C.byref(cp),
        C.byref(nbc) if nbc is not None else None, C.byref(o), int(samples_per_bin),
        _ptr(T, torch.float32, "targets"), ws.data_ptr(), ws.numel(), _stream()),
        "sop_dump_integrand")
    return T


def save_probe_maps(path: str, texels: torch.Tensor, depth: Optional[torch.Tensor] = None,
                    probe_pos: Optional[torch.Tensor] = None, **meta) -> None:
    """Baked probe maps for reuse (the bake runs once per scene): texels [P,R,R,4] (float32
    or float16), optionally the depth maps [P,R,R] and the probe positions [P,3], in a
    safetensors file with string metadata."""
    from safetensors.torch import save_file
    _maps_shape(texels)
    if texels.dtype not in (torch.float32, torch.float16):
        raise ValueError("probe textures must be float32 or float16")
    P, R = int(texels.shape[0]), int(texels.shape[1])
    t = {"texels": texels.detach().cpu().contiguous()}
    if depth is not None:
        _shape(depth, (P, R, R), "depth", torch.float32)
        t["depth"] = depth.detach().cpu().contiguous()
    if probe_pos is not None:
        _shape(probe_pos, (P, 3), "probe_pos", torch.float32)
        t["probe_pos"] = probe_pos.detach().cpu().contiguous()
    save_file(t, path, metadata={str(k): str(v) for k, v in meta.items()})


def load_probe_maps(path: str, device=None):
    """Maps written by save_probe_maps: (dict of tensors on `device`, metadata). Refuses a
    file whose tensors do not have the shapes and types save_probe_maps writes."""
    from safetensors import safe_open
    with safe_open(path, framework="pt") as f:
        meta = dict(f.metadata() or {})
        t = {k: f.get_tensor(k) for k in f.keys()}
    if set(t) - {"texels", "depth", "probe_pos"} or "texels" not in t:
        raise ValueError("not a probe-map file: expected texels [, depth, probe_pos]")
    _maps_shape(t["texels"])
    if t["texels"].dtype not in (torch.float32, torch.float16):
        raise ValueError("probe textures must be float32 or float16")
    P, R = int(t["texels"].shape[0]), int(t["texels"].shape[1])
    if "depth" in t:
        _shape(t["depth"], (P, R, R), "depth", torch.float32)
    if "probe_pos" in t:
        _shape(t["probe_pos"], (P, 3), "probe_pos", torch.float32)
    dev = device if device is not None else "cpu"
    return {k: v.to(dev) for k, v in t.items()}, meta


class Mlp:
    """Proposal network parameters (f32 [41344] on the GPU) with the scene box of its
    position features, and optional Adam state."""

    def __init__(self, params: torch.Tensor, bounds_lo, bounds_hi):
        if params.numel() != L.SOP_MLP_PARAMS:
            raise ValueError(f"params must have {L.SOP_MLP_PARAMS} entries")
        self.params = params
        self.lo = [float(x) for x in bounds_lo]
        self.hi = [float(x) for x in bounds_hi]
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.step = 0
        self._lib = L.load()

    def save(self, path: str, **meta) -> None:
        """Checkpoint: parameters, Adam moments and step count, and the feature box, in a
        safetensors file (extra string metadata, e.g. the training iteration, is kept)."""
        from safetensors.torch import save_file
        info = {"step": str(self.step), "bounds_lo": repr(self.lo), "bounds_hi": repr(self.hi)}
        info.update({str(k): str(v) for k, v in meta.items()})
        save_file({"params": self.params.detach().cpu().contiguous(),
                   "adam_m": self.m.detach().cpu().contiguous(),
                   "adam_v": self.v.detach().cpu().contiguous()}, path, metadata=info)

    @classmethod
    def load(cls, path: str, device=None):
        """A checkpoint written by save(): returns (mlp, metadata dict). Training resumed
        from it continues bit for bit (the same steps, moments and bias corrections)."""
        import ast

        from safetensors import safe_open
        with safe_open(path, framework="pt") as f:
            meta = dict(f.metadata() or {})
            t = {k: f.get_tensor(k) for k in ("params", "adam_m", "adam_v")}
        for k, x in t.items():
            if x.dtype != torch.float32 or x.numel() != L.SOP_MLP_PARAMS:
                raise ValueError(f"checkpoint tensor {k} is not float32[{L.SOP_MLP_PARAMS}]")
        dev = device if device is not None else "cpu"
        mlp = cls(t["params"].to(dev), ast.literal_eval(meta["bounds_lo"]),
                  ast.literal_eval(meta["bounds_hi"]))
        mlp.m = t["adam_m"].to(dev)
        mlp.v = t["adam_v"].to(dev)
        mlp.step = int(meta["step"])
        return mlp, meta

    def c(self) -> L.sop_mlp:
        m = L.sop_mlp()
        m.params = _ptr(self.params, torch.float32, "params")
        m.bounds_lo = (C.c_float * 3)(*self.lo)
        m.bounds_hi = (C.c_float * 3)(*self.hi)
        return m


def proposal_workspace(op: int, n: int, device) -> torch.Tensor:
    return workspace(L.load().sop_proposal_workspace_size(op, int(n)), device)


def sop_proposal_infer(mlp: Mlp, pts: Points, logits: bool = False,
                       ws: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None):
    """probs [N,256] (and logits [N,256] when asked)."""
    dev = pts.pos.device
    n = pts.n
    pts.check()
    _shape(out, (n, L.SOP_MLP_BINS), "out", torch.float32)
    probs = out if out is not None else torch.empty((n, L.SOP_MLP_BINS), dtype=torch.float32,
                                                    device=dev)
    lg = torch.empty((n, L.SOP_MLP_BINS), dtype=torch.float32, device=dev) if logits else None
    if ws is None:
        ws = proposal_workspace(L.SOP_OP_PROPOSAL_INFER, n, dev)
    mc, cp = mlp.c(), pts.c()
    L.check(mlp._lib.sop_proposal_infer(C.byref(mc), C.byref(cp), _ptr(probs, torch.float32),
                                        _ptr(lg, torch.float32), ws.data_ptr(), ws.numel(),
                                        _stream()), "sop_proposal_infer")
    return (probs, lg) if logits else probs


def adam_opts(lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8) -> L.sop_adam:
    return L.sop_adam(float(lr), float(beta1), float(beta2), float(eps), int(step))


def sop_proposal_train_step(mlp: Mlp, pts: Points, targets: torch.Tensor,
                            lr: Optional[float] = None, grad: Optional[torch.Tensor] = None,
                            loss: Optional[torch.Tensor] = None,
                            ws: Optional[torch.Tensor] = None, **adam_kw):
    """One step: returns the batch loss (device scalar tensor). With lr the parameters are
    updated by Adam (mlp.step advances); with grad the batch gradient is written there."""
    dev = pts.pos.device
    pts.check()
    _shape(targets, (pts.n, L.SOP_MLP_BINS), "targets")
    _shape(grad, (L.SOP_MLP_PARAMS,), "grad", torch.float32)
    _shape(loss, (1,), "loss", torch.float32)
    lo = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=dev)
    if ws is None:
        ws = proposal_workspace(L.SOP_OP_PROPOSAL_TRAIN, pts.n, dev)
    opt = None
    if lr is not None:
        mlp.step += 1
        opt = adam_opts(lr, mlp.step, **adam_kw)
    mc, cp = mlp.c(), pts.c()
    L.check(mlp._lib.sop_proposal_train_step(
        C.byref(mc), C.byref(cp), _ptr(targets.contiguous(), torch.float32, "targets"),
        C.byref(opt) if opt is not None else None, _ptr(mlp.m), _ptr(mlp.v),
        _ptr(lo, torch.float32), _ptr(grad, torch.float32, "grad"), ws.data_ptr(), ws.numel(),
        _stream()), "sop_proposal_train_step")
    return lo


def sop_adam_update(params: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                    grad: torch.Tensor, lr: float, step: int, **adam_kw) -> None:
    for t, what in ((m, "m"), (v, "v"), (grad, "grad")):
        if t.numel() != params.numel():
            raise ValueError(f"{what} has {t.numel()} entries, params {params.numel()}")
    opt = adam_opts(lr, step, **adam_kw)
    L.check(L.load().sop_adam_update(_ptr(params, torch.float32), _ptr(m, torch.float32),
                                     _ptr(v, torch.float32), _ptr(grad, torch.float32),
                                     params.numel(), C.byref(opt), _stream()),
            "sop_adam_update")


# ------------------------------------------------------------------------------------------
class BakePlan:
    """Gaussian grid for sop_bake (sop_bake_plan_create / _update / _destroy)."""

    def __init__(self, mean, scale, rotation, opacity, color, t_min=0.0, alpha_min=1.0 / 255.0,
                 alpha_max=0.99, T_min=1e-4, cell_scale=0.0):
        self._lib = L.load()
        self._keep = None
        g = self._gaussians(mean, scale, rotation, opacity, color)
        o = L.sop_bake_opts(float(t_min), float(alpha_min), float(alpha_max), float(T_min),
                            float(cell_scale))
        h = C.c_void_p()
        L.check(self._lib.sop_bake_plan_create(C.byref(g), C.byref(o), _stream(), C.byref(h)),
                "sop_bake_plan_create")
        self.handle = h

    @staticmethod
    def _gaussians(mean, scale, rotation, opacity, color) -> L.sop_gaussians:
        f = torch.float32
        g = L.sop_gaussians()
        g.count = int(mean.shape[0])
        g.mean = _ptr(mean, f, "mean")
        g.scale = _ptr(scale, f, "scale")
        g.rotation = _ptr(rotation, f, "rotation")
        g.opacity = _ptr(opacity, f, "opacity")
        g.color = _ptr(color, f, "color")
        return g

    def update(self, mean, scale, rotation, opacity, color) -> None:
        g = self._gaussians(mean, scale, rotation, opacity, color)
        L.check(self._lib.sop_bake_plan_update(self.handle, C.byref(g), _stream()),
                "sop_bake_plan_update")

    def check(self) -> None:
        L.check(self._lib.sop_bake_plan_check(self.handle, _stream()), "sop_bake_plan_check")

    def close(self) -> None:
        if getattr(self, "handle", None):
            self._lib.sop_bake_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sop_bake(plan: BakePlan, probe_pos: torch.Tensor, res: int, depth: bool = True,
             texels: Optional[torch.Tensor] = None, depth_out: Optional[torch.Tensor] = None,
             order_by: Optional[Plan] = None):
    """Probe textures [P,res,res,4] (R,G,B,O) and depth [P,res,res] by ray tracing; with
    order_by (a probe Plan over the same probes) the probes are traced in its Morton order."""
    _shape(probe_pos, (None, 3), "probe_pos")
    P = int(probe_pos.shape[0])
    _shape(texels, (P, res, res, 4), "texels", torch.float32)
    _shape(depth_out, (P, res, res), "depth_out", torch.float32)
    if order_by is not None and int(order_by.n_probes) != P:
        raise ValueError(f"order_by plan has {int(order_by.n_probes)} probes, not {P}")
    dev = probe_pos.device
    tex = texels if texels is not None else torch.empty((P, res, res, 4), dtype=torch.float32,
                                                        device=dev)
    dep = None
    if depth:
        dep = depth_out if depth_out is not None else torch.empty((P, res, res),
                                                                  dtype=torch.float32,
                                                                  device=dev)
    L.check(plan._lib.sop_bake(plan.handle, _ptr(probe_pos, torch.float32, "probe_pos"), P,
                               int(res), _ptr(tex, torch.float32, "texels"), _ptr(dep),
                               order_by.handle if order_by is not None else None,
                               _stream()), "sop_bake")
    return tex, dep


def sop_shade_traced(plan: BakePlan, env: torch.Tensor, pts: Points, n_dirs: int,
                     offset: float, seed: int = 0, rotate_per_point: bool = False,
                     irradiance: bool = False, order_by: Optional[Plan] = None,
                     samples: bool = False, ws: Optional[torch.Tensor] = None,
                     out: Optional[torch.Tensor] = None,
                     samples_out: Optional[torch.Tensor] = None):
    """Traced shading: rgb [N,3] with every sample's O and L_in from its own ray through
    the plan's Gaussians, starting at fmaf(offset, n, x). Returns rgb, or a tuple
    (rgb, irradiance [N,3] when asked, samples [N,S,4] when asked); order_by (a probe Plan)
    orders the points for ray coherence without changing the result."""
    dev = pts.pos.device
    n = pts.n
    pts.check()
    _env_shape(env)
    _shape(out, (n, 3), "out", torch.float32)
    _shape(samples_out, (n, int(n_dirs), 4), "samples_out", torch.float32)
    rgb = out if out is not None else torch.empty((n, 3), dtype=torch.float32, device=dev)
    irr = torch.empty((n, 3), dtype=torch.float32, device=dev) if irradiance else None
    smp = samples_out
    if samples and smp is None:
        smp = torch.empty((n, int(n_dirs), 4), dtype=torch.float32, device=dev)
    lib = plan._lib
    oh = order_by.handle if order_by is not None else None
    if ws is None:
        nbytes = lib.sop_shade_traced_workspace_size(oh, n, int(n_dirs), int(env.shape[0]),
                                                     int(env.shape[1]), int(smp is not None))
        ws = workspace(nbytes, dev)
    o = shade_opts(n_dirs, 1, seed, math.inf, rotate_per_point, irr)
    e, cp = _env(env), pts.c()
    L.check(lib.sop_shade_traced(plan.handle, oh, C.byref(e), C.byref(cp), C.byref(o),
                                 float(offset), _ptr(rgb, torch.float32, "rgb"), _ptr(smp),
                                 ws.data_ptr(), ws.numel(), _stream()), "sop_shade_traced")
    res = (rgb,) + ((irr,) if irradiance else ()) + ((smp,) if smp is not None else ())
    return res[0] if len(res) == 1 else res


def sop_shadow_ratio(plan: Plan, texels: torch.Tensor, env_oct: torch.Tensor, pts: Points,
                     n_dirs: int, k: int = 4, nb: Optional[Neighbors] = None, seed: int = 0,
                     radius: float = math.inf, rotate_per_point: bool = False,
                     sampler: int = L.SOP_SHADOW_HAMMERSLEY, irradiance: bool = False,
                     ws: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None):
    """Cast-shadow ratio [N,3] of the points under the octahedral environment env_oct
    [Re,Re,3], the object's occlusion read from channel 3 of the shadow-region probe maps
    texels [P,R,R,4]; with irradiance=True also the unshadowed estimate [N,3]."""
    dev = pts.pos.device
    n = pts.n
    _shape(pts.pos, (n, 3), "pos")
    _shape(pts.normal, (n, 3), "normal")
    _maps_shape(texels, plan)
    _shape(env_oct, (None, None, 3), "env_oct")
    _shape(out, (n, 3), "out", torch.float32)
    if nb is not None:
        nb.check(n)
    ratio = out if out is not None else torch.empty((n, 3), dtype=torch.float32, device=dev)
    irr = torch.empty((n, 3), dtype=torch.float32, device=dev) if irradiance else None
    kk = nb.k if nb is not None else k
    lib = plan._lib
    if ws is None:
        ws = workspace(lib.sop_shadow_workspace_size(plan.handle, n, kk, int(n_dirs),
                                                     int(env_oct.shape[0]), int(nb is not None)),
                       dev)
    o = L.sop_shadow_opts()
    o.n_dirs, o.k, o.radius, o.seed = int(n_dirs), int(kk), float(radius), int(seed) & 0xFFFFFFFF
    o.rotate_per_point, o.sampler = int(rotate_per_point), int(sampler)
    o.out_irradiance = _ptr(irr, torch.float32, "irradiance")
    e = L.sop_env_oct()
    e.res = int(env_oct.shape[0])
    e.texels = _ptr(env_oct, torch.float32, "env_oct")
    m = _maps(texels, plan)
    cp = L.sop_points()
    cp.count = n
    cp.pos = _ptr(pts.pos, torch.float32, "pos")
    cp.normal = _ptr(pts.normal, torch.float32, "normal")
    nbc = nb.c(n) if nb is not None else None
    L.check(lib.sop_shadow_ratio(plan.handle, C.byref(m), C.byref(e), C.byref(cp),
                                 C.byref(nbc) if nbc is not None else None, C.byref(o),
                                 _ptr(ratio, torch.float32, "ratio"), ws.data_ptr(), ws.numel(),
                                 _stream()), "sop_shadow_ratio")
    return (ratio, irr) if irradiance else ratio


def sop_place_probes(pts: torch.Tensor, normals: torch.Tensor, n_probes: int, start: int = 0,
                     offset: float = 0.0, ws: Optional[torch.Tensor] = None):
    """Farthest point sampling of n_probes of the surface points pts [M,3] (normals [M,3])
    from `start`, each pick raised by `offset` along its normal: (probe_pos [P,3],
    chosen [P] int32)."""
    _shape(pts, (None, 3), "pts")
    M, dev = int(pts.shape[0]), pts.device
    _shape(normals, (M, 3), "normals")
    lib = L.load()
    out = torch.empty((int(n_probes), 3), dtype=torch.float32, device=dev)
    chosen = torch.empty(int(n_probes), dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(lib.sop_place_workspace_size(M, int(n_probes)), dev)
    L.check(lib.sop_place_probes(_ptr(pts, torch.float32, "pts"),
                                 _ptr(normals, torch.float32, "normals"), M, int(n_probes),
                                 int(start), float(offset), _ptr(chosen, torch.int32, "chosen"),
                                 _ptr(out, torch.float32, "probe_pos"), ws.data_ptr(),
                                 ws.numel(), _stream()), "sop_place_probes")
    return out, chosen


def sop_sops_loss(tex: torch.Tensor, target: torch.Tensor, grad: bool = True,
                  ws: Optional[torch.Tensor] = None, loss_out: Optional[torch.Tensor] = None,
                  grad_out: Optional[torch.Tensor] = None):
    """L_sops of probe textures [...,4] against the traced ones: (loss [2] =
    (L1(L_in, L_tr), L1(O, O_tr)), gradient of their sum w.r.t. tex or None)."""
    if tex.dim() < 1 or tex.shape[-1] != 4:
        raise ValueError("probe textures must end in 4 channels")
    _shape(target, tuple(tex.shape), "target")
    _shape(grad_out, tuple(tex.shape), "grad_out", torch.float32)
    _shape(loss_out, (2,), "loss_out", torch.float32)
    lib = L.load()
    T, dev = int(tex.numel() // 4), tex.device
    loss = loss_out if loss_out is not None else torch.empty(2, dtype=torch.float32, device=dev)
    g = (grad_out if grad_out is not None else torch.empty_like(tex)) if grad else None
    if ws is None:
        ws = workspace(lib.sop_loss_workspace_size(T), dev)
    L.check(lib.sop_sops_loss(_ptr(tex, torch.float32, "tex"),
                              _ptr(target, torch.float32, "target"), T,
                              _ptr(loss, torch.float32, "loss"), _ptr(g), ws.data_ptr(),
                              ws.numel(), _stream()), "sop_sops_loss")
    return loss, g


def sop_lam_loss(rough: torch.Tensor, metal: torch.Tensor, grad: bool = True,
                 ws: Optional[torch.Tensor] = None):
    """L_lam of the materials: (loss [2] = (L1(R, 1), L1(M, 0)), g_rough, g_metal)."""
    _shape(rough, (None,), "rough")
    _shape(metal, (int(rough.shape[0]),), "metal")
    lib = L.load()
    N, dev = int(rough.numel()), rough.device
    loss = torch.empty(2, dtype=torch.float32, device=dev)
    gr = torch.empty_like(rough) if grad else None
    gm = torch.empty_like(metal) if grad else None
    if ws is None:
        ws = workspace(lib.sop_loss_workspace_size(N), dev)
    L.check(lib.sop_lam_loss(_ptr(rough, torch.float32, "rough"),
                             _ptr(metal, torch.float32, "metal"), N,
                             _ptr(loss, torch.float32, "loss"), _ptr(gr), _ptr(gm),
                             ws.data_ptr(), ws.numel(), _stream()), "sop_lam_loss")
    return loss, gr, gm
