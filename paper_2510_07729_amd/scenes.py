"""Seeded synthetic workloads for the SOP shading path.

Input generation only: this module draws positions, normals, materials, textures and
Gaussians with numpy and contains none of the method's arithmetic, so both the GPU
library's tests and the CPU oracle can take their inputs from it.

Every array comes from its own stream ``np.random.default_rng(SeedSequence([cfg, stream,
seed]))``, so two calls with the same arguments return byte-identical arrays.

Workloads (the shapes and distributions of the paper's reconstruction and rendering set-ups,
Sec. 4.1: 16x16 to 32x32 probe textures, 128-256 rays, thousands of probes near an object's
surface, object views of 800x800 and scene views up to 1920x1080):

* ``tiny_shade``      4096 points on the unit sphere, 64 probes on it, 16x16 f32 maps,
                      32x64 environment, S=64, K=4.
* ``object_scene``    sphere (r=0.5) and torus (R=0.9, r=0.2) covered by 100k 3D Gaussians,
                      4096 probes placed by farthest point sampling and offset along the
                      normal by 1% of the object's diagonal, 200k points, S=128, K=8,
                      256x512 environment.
* ``diff_step``       the tiny scene plus hidden materials for a reconstruction target.
* ``proposal_eval``   the tiny scene with 200k held-out points (learned proposal).
* ``mlp_init`` / ``bin_probs``  proposal network weights and bin distributions.
* ``gbuffer_frames``  8 pinhole cameras (1920x1080, f=3200 px) on a sphere of radius 3
                      looking at the unit sphere; 16,384 probes with 32x32 f16 maps.
* ``shadow_scene``    the object standing over a ground plane: 2048 shadow-region probes
                      placed by farthest point sampling on the plane around it (a square
                      twice the object's extent) and raised by 1% of its diagonal, 500k
                      ground points with normal +z, a 256x256 octahedral sky whose sun holds
                      about 70% of its energy and whose lower half is dimmed, S=64, K=8.
"""
from __future__ import annotations

import dataclasses
import functools
from typing import Optional

import numpy as np

F32 = np.float32

CFG_TINY, CFG_OBJECT, CFG_DIFF, CFG_FRAMES, CFG_PROPOSAL, CFG_SHADOW = 1, 2, 3, 4, 5, 6


def rng(cfg: int, stream: int, seed: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg, stream, seed]))


# ------------------------------------------------------------------------------------------
# elementary draws
# ------------------------------------------------------------------------------------------
def unit_vectors(g: np.random.Generator, n: int) -> np.ndarray:
    v = g.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def hemisphere_vectors(g: np.random.Generator, normals: np.ndarray) -> np.ndarray:
    """Uniform directions on the hemisphere around each normal (flip of a sphere draw)."""
    v = unit_vectors(g, normals.shape[0])
    s = np.sign(np.sum(v * normals, axis=1, keepdims=True))
    s[s == 0] = 1.0
    return v * s


def probe_textures(g: np.random.Generator, P: int, res: int, sigma: float = 1.0,
                   half: bool = False) -> np.ndarray:
    """RGB radiance ~ lognormal(0, sigma); occlusion stored as O = 1 - exp(-tau),
    tau ~ U(0, 2) (an optical depth turned into the occlusion fraction the texel holds)."""
    tex = np.empty((P, res, res, 4), dtype=np.float64)
    tex[..., :3] = g.lognormal(0.0, sigma, size=(P, res, res, 3))
    tau = g.uniform(0.0, 2.0, size=(P, res, res))
    tex[..., 3] = -np.expm1(-tau)
    return tex.astype(np.float16 if half else F32)


def env_map(g: np.random.Generator, H: int, W: int, sigma: float) -> np.ndarray:
    return g.lognormal(0.0, sigma, size=(H, W, 3)).astype(F32)


def materials(g: np.random.Generator, n: int):
    albedo = g.uniform(0.0, 1.0, size=(n, 3)).astype(F32)
    rough = g.uniform(0.05, 1.0, size=n).astype(F32)
    metal = g.uniform(0.0, 1.0, size=n).astype(F32)
    return albedo, rough, metal


# ------------------------------------------------------------------------------------------
# scene containers
# ------------------------------------------------------------------------------------------
@dataclasses.dataclass
class ShadeScene:
    """Everything a shading call needs, as float32/float16 numpy arrays."""
    name: str
    probe_pos: np.ndarray            # [P,3] f32
    bounds_lo: np.ndarray            # [3]   f32
    bounds_hi: np.ndarray            # [3]   f32
    texels: np.ndarray               # [P,R,R,4] f32 or f16
    env: np.ndarray                  # [H,W,3] f32
    pos: np.ndarray                  # [N,3] f32
    normal: np.ndarray               # [N,3] f32
    view: Optional[np.ndarray]       # [N,3] f32 or None (camera mode)
    cam_pos: Optional[np.ndarray]    # [F,3] f32
    points_per_frame: int
    albedo: np.ndarray               # [N,3]
    rough: np.ndarray                # [N]
    metal: np.ndarray                # [N]
    n_dirs: int
    k: int
    radius: float = float("inf")
    seed: int = 0
    env_oct: bool = False            # env is an octahedral map [R,R,3] (else equirect [H,W,3])

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def res(self) -> int:
        return int(self.texels.shape[1])

    def subset(self, rows: np.ndarray) -> "ShadeScene":
        """The same scene restricted to the given point rows (view mode only)."""
        assert self.view is not None
        return dataclasses.replace(
            self, pos=self.pos[rows].copy(), normal=self.normal[rows].copy(),
            view=self.view[rows].copy(), albedo=self.albedo[rows].copy(),
            rough=self.rough[rows].copy(), metal=self.metal[rows].copy())


@dataclasses.dataclass
class GaussianScene:
    mean: np.ndarray       # [G,3] f32
    scale: np.ndarray      # [G,3] f32
    rotation: np.ndarray   # [G,4] f32 (w,x,y,z)
    opacity: np.ndarray    # [G]   f32
    color: np.ndarray      # [G,3] f32

    @property
    def count(self) -> int:
        return int(self.mean.shape[0])


# ------------------------------------------------------------------------------------------
# tiny sphere scene (64 probes, 4096 points)
# ------------------------------------------------------------------------------------------
def tiny_shade(n_points: int = 4096, n_probes: int = 64, res: int = 16, H: int = 32,
               W: int = 64, n_dirs: int = 64, k: int = 4, seed: int = 0) -> ShadeScene:
    cfg = CFG_TINY
    ppos = unit_vectors(rng(cfg, 0, seed), n_probes).astype(F32)
    tex = probe_textures(rng(cfg, 1, seed), n_probes, res)
    pts = unit_vectors(rng(cfg, 2, seed), n_points)
    normal = pts.astype(F32)
    view = hemisphere_vectors(rng(cfg, 3, seed), pts).astype(F32)
    albedo, rough, metal = materials(rng(cfg, 4, seed), n_points)
    env = env_map(rng(cfg, 5, seed), H, W, 1.0)
    return ShadeScene("tiny_shade", ppos, np.full(3, -1.05, F32), np.full(3, 1.05, F32), tex,
                      env, pts.astype(F32), normal, view, None, 0, albedo, rough, metal,
                      n_dirs, k, seed=seed)


def proposal_eval(n_points: int = 200_000, seed: int = 0) -> ShadeScene:
    """The tiny scene (its probes, textures and environment, whatever the seed) with new
    shading points from the proposal workload's own streams (keyed by the seed): training
    pools and held-out sets of the learned proposal share one scene."""
    sc = tiny_shade(n_points=1, seed=0)
    cfg = CFG_PROPOSAL
    pts = unit_vectors(rng(cfg, 2, seed), n_points)
    view = hemisphere_vectors(rng(cfg, 3, seed), pts).astype(F32)
    albedo, rough, metal = materials(rng(cfg, 4, seed), n_points)
    return dataclasses.replace(sc, name="proposal_eval", pos=pts.astype(F32),
                               normal=pts.astype(F32), view=view, albedo=albedo, rough=rough,
                               metal=metal, seed=seed)


# learned direction proposal: parameter blob W1 [320,64], b1, W2 [64,64], b2, W3 [64,256], b3
MLP_SHAPES = ((320, 64), (64,), (64, 64), (64,), (64, 256), (256,))
MLP_PARAMS = sum(int(np.prod(s)) for s in MLP_SHAPES)


def mlp_init(seed: int = 0, gain: float = 1.0) -> np.ndarray:
    """He-normal weights (std = gain * sqrt(2 / fan_in)), zero biases, as one f32 blob."""
    g = rng(CFG_PROPOSAL, 10, seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            parts.append(g.standard_normal(shape).ravel() * gain * np.sqrt(2.0 / shape[0]))
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(F32)


def bin_probs(n: int, concentration: float = 0.3, seed: int = 0) -> np.ndarray:
    """Random distributions over the 256 proposal bins, Dirichlet(concentration), f32."""
    g = rng(CFG_PROPOSAL, 11, seed)
    return g.dirichlet(np.full(256, concentration), size=n).astype(F32)


def diff_step(seed: int = 0):
    """The tiny scene plus hidden materials (a separate stream) for the target image."""
    sc = tiny_shade(seed=seed)
    hidden = materials(rng(CFG_DIFF, 0, seed), sc.n)
    return sc, hidden


# ------------------------------------------------------------------------------------------
# object scene: sphere (r = 0.5) and torus (R = 0.9, r = 0.2) about z
# ------------------------------------------------------------------------------------------
SPHERE_R, TORUS_R, TORUS_r = 0.5, 0.9, 0.2


def object_surface(g: np.random.Generator, n: int):
    """Area-uniform points and outward normals on the sphere-and-torus object."""
    a_s = 4.0 * np.pi * SPHERE_R ** 2
    a_t = 4.0 * np.pi ** 2 * TORUS_R * TORUS_r
    on_sphere = g.uniform(size=n) < a_s / (a_s + a_t)
    pos = np.empty((n, 3))
    nrm = np.empty((n, 3))
    ns = int(on_sphere.sum())
    d = unit_vectors(g, ns)
    pos[on_sphere] = SPHERE_R * d
    nrm[on_sphere] = d
    nt = n - ns
    u = g.uniform(0.0, 2 * np.pi, size=nt)
    # tube angle with density proportional to (R + r cos v): rejection sampling
    v = np.empty(nt)
    filled = 0
    while filled < nt:
        cand = g.uniform(0.0, 2 * np.pi, size=2 * (nt - filled) + 16)
        acc = g.uniform(size=cand.size) * (TORUS_R + TORUS_r) < TORUS_R + TORUS_r * np.cos(cand)
        take = cand[acc][: nt - filled]
        v[filled: filled + take.size] = take
        filled += take.size
    ring = TORUS_R + TORUS_r * np.cos(v)
    pos[~on_sphere] = np.stack([ring * np.cos(u), ring * np.sin(u), TORUS_r * np.sin(v)], 1)
    nrm[~on_sphere] = np.stack([np.cos(v) * np.cos(u), np.cos(v) * np.sin(u), np.sin(v)], 1)
    return pos, nrm


def farthest_point_sampling(points: np.ndarray, m: int) -> np.ndarray:
    """Indices of m points chosen greedily by largest distance to the chosen set, starting
    at point 0 (the placement step of Sec. 3.1.2, run here on analytic surface samples)."""
    chosen = np.empty(m, dtype=np.int64)
    chosen[0] = 0
    dmin = np.sum((points - points[0]) ** 2, axis=1)
    for s in range(1, m):
        c = int(np.argmax(dmin))
        chosen[s] = c
        dmin = np.minimum(dmin, np.sum((points - points[c]) ** 2, axis=1))
    return chosen


OBJECT_DIAGONAL = float(np.sqrt((2 * (TORUS_R + TORUS_r)) ** 2 * 2 + (2 * SPHERE_R) ** 2))


@functools.lru_cache(maxsize=4)
def object_probes(n_probes: int = 4096, n_candidates: int = 65536, seed: int = 0):
    """Probe positions: FPS over surface samples, offset by 1% of the object's diagonal
    along the surface normal (Sec. 3.1.2 placement, Sec. 4.1 offset)."""
    pos, nrm = object_surface(rng(CFG_OBJECT, 10, seed), n_candidates)
    sel = farthest_point_sampling(pos, n_probes)
    out = pos[sel] + 0.01 * OBJECT_DIAGONAL * nrm[sel]
    return out.astype(F32)


def object_gaussians(n: int = 100_000, seed: int = 0) -> GaussianScene:
    g = rng(CFG_OBJECT, 11, seed)
    mean, _ = object_surface(g, n)
    scale = g.lognormal(-4.0, 0.5, size=(n, 3))
    q = g.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opacity = g.uniform(0.3, 1.0, size=n)
    color = g.uniform(0.0, 1.0, size=(n, 3))
    return GaussianScene(mean.astype(F32), scale.astype(F32), q.astype(F32),
                         opacity.astype(F32), color.astype(F32))


OBJECT_BOUNDS = (np.array([-1.2, -1.2, -0.6], F32), np.array([1.2, 1.2, 0.6], F32))


def object_scene(n_points: int = 200_000, n_probes: int = 4096, res: int = 32,
                 H: int = 256, W: int = 512, n_dirs: int = 128, k: int = 8,
                 textures: Optional[np.ndarray] = None, seed: int = 0) -> ShadeScene:
    """Shading workload on the object. ``textures`` are the probe maps to shade with (the
    bake's output in the full pipeline); by default synthetic maps with the tiny scene's
    distributions are drawn so that the scene stands on its own."""
    cfg = CFG_OBJECT
    ppos = object_probes(n_probes, seed=seed)
    if textures is None:
        textures = probe_textures(rng(cfg, 1, seed), n_probes, res)
    pos, nrm = object_surface(rng(cfg, 2, seed), n_points)
    view = hemisphere_vectors(rng(cfg, 3, seed), nrm).astype(F32)
    albedo, rough, metal = materials(rng(cfg, 4, seed), n_points)
    env = env_map(rng(cfg, 5, seed), H, W, 1.5)
    lo, hi = OBJECT_BOUNDS
    return ShadeScene("object_scene", ppos, lo.copy(), hi.copy(), textures, env,
                      pos.astype(F32), nrm.astype(F32), view, None, 0, albedo, rough, metal,
                      n_dirs, k, seed=seed)


# ------------------------------------------------------------------------------------------
# G-buffer frames: analytic ray-sphere hits of pinhole cameras
# ------------------------------------------------------------------------------------------
def camera_rays(cam: np.ndarray, width: int, height: int, focal: float, rows=None):
    """Unit ray directions of a pinhole camera at `cam` looking at the origin (up = +z, or
    +x near the poles). rows: optional pixel-row subset."""
    f = -cam / np.linalg.norm(cam)
    up = np.array([0.0, 0.0, 1.0]) if abs(f[2]) < 0.99 else np.array([1.0, 0.0, 0.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    up2 = np.cross(right, f)
    ys = np.arange(height) if rows is None else np.asarray(rows)
    px, py = np.meshgrid(np.arange(width) + 0.5 - width / 2, height / 2 - (ys + 0.5))
    d = f * focal + right * px[..., None] + up2 * py[..., None]
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return d.reshape(-1, 3)


def gbuffer_frames(n_frames: int = 8, width: int = 1920, height: int = 1080,
                   focal: float = 3200.0, n_probes: int = 16384, res: int = 32,
                   H: int = 256, W: int = 512, n_dirs: int = 64, k: int = 8,
                   rows=None, seed: int = 0) -> ShadeScene:
    """G-buffers of the unit sphere seen by n_frames cameras on a sphere of radius 3 (every
    pixel hits: the silhouette radius f*tan(asin(1/3)) = 1131 px exceeds the half diagonal
    1101 px). Points are frame-major; the view of a point is its frame's camera.
    rows: optional subset of pixel rows per frame (a smaller workload of the same kind)."""
    cfg = CFG_FRAMES
    cams = 3.0 * unit_vectors(rng(cfg, 0, seed), n_frames)
    pos_l = []
    for f in range(n_frames):
        d = camera_rays(cams[f], width, height, focal, rows)
        c = cams[f]
        b = d @ c
        disc = b * b - (c @ c - 1.0)
        assert np.all(disc > 0), "every pixel ray must hit the unit sphere"
        t = -b - np.sqrt(disc)
        pos_l.append(c + t[:, None] * d)
    pos = np.concatenate(pos_l, 0)
    nrm = pos / np.linalg.norm(pos, axis=1, keepdims=True)
    n = pos.shape[0]
    albedo, rough, metal = materials(rng(cfg, 4, seed), n)
    ppos = unit_vectors(rng(cfg, 1, seed), n_probes).astype(F32)
    tex = probe_textures(rng(cfg, 2, seed), n_probes, res, half=True)
    env = env_map(rng(CFG_OBJECT, 5, seed), H, W, 1.5)
    return ShadeScene("gbuffer_frames", ppos, np.full(3, -1.05, F32), np.full(3, 1.05, F32),
                      tex, env, pos.astype(F32), nrm.astype(F32), None,
                      cams.astype(F32), n // n_frames, albedo, rough, metal, n_dirs, k,
                      seed=seed)


# ------------------------------------------------------------------------------------------
# small helpers for tests
# ------------------------------------------------------------------------------------------
def random_gaussians(g: np.random.Generator, n: int, center=(0.0, 0.0, 0.0), spread=0.3,
                     log_scale=(-3.0, 0.4)) -> GaussianScene:
    mean = np.asarray(center) + spread * g.standard_normal((n, 3))
    scale = g.lognormal(log_scale[0], log_scale[1], size=(n, 3))
    q = g.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return GaussianScene(mean.astype(F32), scale.astype(F32), q.astype(F32),
                         g.uniform(0.3, 1.0, size=n).astype(F32),
                         g.uniform(0.0, 1.0, size=(n, 3)).astype(F32))


# ------------------------------------------------------------------------------------------
# cast shadows: the object over a ground plane, probes of the shadow region, octahedral sky
# ------------------------------------------------------------------------------------------
SHADOW_PLANE_Z = -0.55      # just below the object (its lowest point is at z = -0.5)
SHADOW_HALF = 2.2           # half side of the shadow region: twice the object's extent
SHADOW_BOUNDS = (np.array([-2.4, -2.4, -0.8], F32), np.array([2.4, 2.4, 0.8], F32))


@dataclasses.dataclass
class ShadowScene:
    probe_pos: np.ndarray            # [P,3] f32, the shadow-region probes
    bounds_lo: np.ndarray
    bounds_hi: np.ndarray
    texels: np.ndarray               # [P,R,R,4] f32 (channel 3: the object's occlusion O')
    env: np.ndarray                  # [Re,Re,3] f32 octahedral sky
    pos: np.ndarray                  # [N,3] f32 ground points
    normal: np.ndarray               # [N,3] f32
    n_dirs: int
    k: int
    seed: int = 0

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def subset(self, rows: np.ndarray) -> "ShadowScene":
        return dataclasses.replace(self, pos=self.pos[rows].copy(),
                                   normal=self.normal[rows].copy())


def octahedral_sky(g: np.random.Generator, res: int, sigma: float = 1.0,
                   sun=(0.3, 0.35), gain: float = 1000.0, width: float = 0.02,
                   ground: float = 0.2) -> np.ndarray:
    """Octahedral sky [res,res,3] shaped like an outdoor HDR map: lognormal(0, sigma)
    texels, those outside the square's central diamond (the lower hemisphere of the map)
    dimmed by ``ground``, plus a warm sun blob of peak ``gain`` centred at the fraction
    ``sun`` of the square (texel space, x then y; inside the diamond). With the defaults the
    sun holds about 70% of the energy at res 256."""
    base = g.lognormal(0.0, sigma, size=(res, res, 3))
    c = (np.arange(res) + 0.5) / res
    lower = (np.abs(c[None, :] - 0.5) + np.abs(c[:, None] - 0.5)) > 0.5
    base[lower] *= ground
    d2 = (c[None, :] - sun[0]) ** 2 + (c[:, None] - sun[1]) ** 2
    blob = gain * np.exp(-d2 / (2.0 * width * width))
    return (base + blob[..., None] * np.array([1.0, 0.9, 0.7])).astype(F32)


@functools.lru_cache(maxsize=4)
def shadow_probes(n_probes: int = 2048, n_candidates: int = 65536, seed: int = 0):
    """Probes of the shadow region: FPS over uniform samples of the ground square, raised
    along the plane's normal by 1% of the object's diagonal (the placement of the object's
    own probes)."""
    g = rng(CFG_SHADOW, 1, seed)
    xy = g.uniform(-SHADOW_HALF, SHADOW_HALF, size=(n_candidates, 2))
    pts = np.column_stack([xy, np.full(n_candidates, SHADOW_PLANE_Z)])
    sel = farthest_point_sampling(pts, n_probes)
    out = pts[sel] + np.array([0.0, 0.0, 0.01 * OBJECT_DIAGONAL])
    return out.astype(F32)


def shadow_scene(n_points: int = 500_000, n_probes: int = 2048, res: int = 32,
                 env_res: int = 256, n_dirs: int = 64, k: int = 8,
                 textures: Optional[np.ndarray] = None, seed: int = 0) -> ShadowScene:
    """Shadow workload. ``textures`` are the shadow probes' maps (the bake of the object's
    Gaussians in the full pipeline); by default synthetic maps with the tiny scene's
    distributions (O' = 1 - exp(-tau), tau ~ U(0, 2)) so that the scene stands on its own."""
    ppos = shadow_probes(n_probes, seed=seed)
    if textures is None:
        textures = probe_textures(rng(CFG_SHADOW, 2, seed), n_probes, res)
    g = rng(CFG_SHADOW, 3, seed)
    xy = g.uniform(-SHADOW_HALF, SHADOW_HALF, size=(n_points, 2))
    pos = np.column_stack([xy, np.full(n_points, SHADOW_PLANE_Z)]).astype(F32)
    nrm = np.tile(np.array([0.0, 0.0, 1.0], F32), (n_points, 1))
    env = octahedral_sky(rng(CFG_SHADOW, 4, seed), env_res)
    lo, hi = SHADOW_BOUNDS
    return ShadowScene(ppos, lo.copy(), hi.copy(), textures, env, pos, nrm, n_dirs, k,
                       seed=seed)
