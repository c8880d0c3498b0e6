"""torch.autograd.Function around sop_shade / sop_shade_backward.

Gradients flow to per-point albedo, roughness and metallic, to the environment texels and
to the probe texels (radiance and occlusion channels). Geometry (positions, normals, views)
and the neighbour weights are constants of the step, as in the paper's material and
lighting decomposition (Sec. 3.1.2, step 2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import torch

from .sop import Neighbors, OctEnv, Plan, Points, sop_knn, sop_shade, sop_shade_backward


@dataclasses.dataclass
class Geometry:
    pos: torch.Tensor
    normal: torch.Tensor
    view: Optional[torch.Tensor] = None
    cam_pos: Optional[torch.Tensor] = None
    points_per_frame: int = 0

    def points(self, albedo, rough, metal) -> Points:
        return Points(self.pos, self.normal, albedo, rough, metal, view=self.view,
                      cam_pos=self.cam_pos, points_per_frame=self.points_per_frame)


class SopShade(torch.autograd.Function):
    """rgb = SopShade.apply(albedo, rough, metal, env, texels, plan, geometry, nb, n_dirs,
    seed, env_oct). nb may be None (the search then runs inside each call with k = 4);
    env_oct: env is an octahedral map [R,R,3] (else equirectangular [H,W,3])."""

    @staticmethod
    def forward(ctx, albedo, rough, metal, env, texels, plan: Plan, geom: Geometry,
                nb: Optional[Neighbors], n_dirs: int, seed: int = 0, env_oct: bool = False):
        albedo, rough, metal = albedo.contiguous(), rough.contiguous(), metal.contiguous()
        env, texels = env.contiguous(), texels.contiguous()
        pts = geom.points(albedo, rough, metal)
        rgb = sop_shade(plan, texels, OctEnv(env) if env_oct else env, pts, n_dirs, nb=nb,
                        seed=seed, k=nb.k if nb is not None else 4)
        ctx.save_for_backward(albedo, rough, metal, env, texels)
        ctx.plan, ctx.geom, ctx.nb, ctx.n_dirs, ctx.seed = plan, geom, nb, n_dirs, seed
        ctx.env_oct = env_oct
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        albedo, rough, metal, env, texels = ctx.saved_tensors
        need = ctx.needs_input_grad
        want = [name for name, flag in zip(("albedo", "rough", "metal", "env", "tex"), need[:5])
                if flag]
        if not want:
            return (None,) * 11
        pts = ctx.geom.points(albedo, rough, metal)
        g = sop_shade_backward(ctx.plan, texels, OctEnv(env) if ctx.env_oct else env, pts,
                               grad_rgb.contiguous(), ctx.n_dirs,
                               nb=ctx.nb, seed=ctx.seed,
                               k=ctx.nb.k if ctx.nb is not None else 4, want=tuple(want))
        g_tex = g.get("tex")
        if g_tex is not None and g_tex.dtype != texels.dtype:
            g_tex = g_tex.to(texels.dtype)
        return (g.get("albedo"), g.get("rough"), g.get("metal"), g.get("env"), g_tex,
                None, None, None, None, None, None)


def shade(albedo, rough, metal, env, texels, plan: Plan, geom: Geometry, n_dirs: int, k: int,
          seed: int = 0, radius: float = math.inf, nb: Optional[Neighbors] = None,
          env_oct: bool = False):
    """Differentiable shading; searches the neighbours once when nb is not given. env_oct:
    env is an octahedral map [R,R,3]."""
    if nb is None:
        nb = sop_knn(plan, geom.points(albedo, rough, metal), k, radius)
    return SopShade.apply(albedo, rough, metal, env, texels, plan, geom, nb, n_dirs, seed,
                          env_oct)
