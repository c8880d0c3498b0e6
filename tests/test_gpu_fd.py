"""Finite differences of the GPU shading forward against the GPU adjoint, on the L2
reconstruction step of the tiny scene (4096 points with their own materials, a target
shaded with hidden materials, grad_rgb = 2 (rgb - target), S = 64, K = 4). The adjoint
gives J^T g for the upstream gradient g, so each entry is compared with the central
difference of the linear functional L = sum_i g_i . rgb_i (g fixed, sums in FP64 on the
host) under a perturbation of that entry: every point's roughness, metallic and albedo
(one perturbation of all points at once: a point's rgb depends on its own materials only),
64 probe texel channels and 64 environment texel channels. rgb is affine in the texels
and linear in the environment, so those differences are exact up to FP32 rounding; the
material ones carry the O(h^2) truncation of the BRDF's curvature."""
import numpy as np
import pytest

from paper_2510_07729_amd import scenes
from tests.gpu_util import dev, gpu_plan, gpu_points, log

pytestmark = pytest.mark.gpu

S, K = 64, 4


@pytest.fixture(scope="module")
def fd_case():
    import torch
    from paper_2510_07729_amd import sop
    assert torch.cuda.is_available()
    sc, (ha, hr, hm) = scenes.diff_step()
    plan = gpu_plan(sc)
    tex, env = dev(sc.texels), dev(sc.env)
    pts = gpu_points(sc)
    nb = sop.sop_knn(plan, pts, K)
    target = sop.sop_shade(plan, tex, env, gpu_points(sc, ha, hr, hm), S, nb=nb)
    rgb = sop.sop_shade(plan, tex, env, pts, S, nb=nb)
    g = (2.0 * (rgb - target)).contiguous()
    ad = {k: v.cpu().numpy().astype(np.float64)
          for k, v in sop.sop_shade_backward(plan, tex, env, pts, g, S, k=K, nb=nb).items()}
    return sc, plan, tex, env, nb, g.cpu().numpy().astype(np.float64), ad


def shade(sc, plan, tex, env, nb, albedo=None, rough=None, metal=None):
    from paper_2510_07729_amd import sop
    pts = gpu_points(sc, albedo, rough, metal)
    return sop.sop_shade(plan, tex, env, pts, S, nb=nb).cpu().numpy().astype(np.float64)


def rel_err(fd, ad):
    return np.abs(fd - ad) / (np.abs(ad) + 1e-2 * np.mean(np.abs(ad)) + 1e-6)


def test_material_gradients_match_central_differences(fd_case):
    sc, plan, tex, env, nb, g, ad = fd_case
    h = 1e-2
    for key in ("rough", "metal"):
        x = getattr(sc, key).astype(np.float32)
        # roughness enters through alpha = r^2 and the GGX lobe: a step relative to r keeps
        # the truncation error small at r = 0.05 (rgb is linear in metallic and albedo)
        hk = (0.02 * x if key == "rough" else np.full_like(x, h)).astype(np.float32)
        xp, xm = x + hk, x - hk
        lp = np.sum(g * shade(sc, plan, tex, env, nb, **{key: xp}), axis=1)
        lm = np.sum(g * shade(sc, plan, tex, env, nb, **{key: xm}), axis=1)
        e = rel_err((lp - lm) / (xp.astype(np.float64) - xm), ad[key])
        log(f"FD {key}: p99 {np.percentile(e, 99):.2e} max {e.max():.2e} over {e.size} points")
        assert np.percentile(e, 99) <= 1e-2 and e.max() <= 5e-2
    for c in range(3):
        a = sc.albedo.astype(np.float32).copy()
        ap, am = a.copy(), a.copy()
        ap[:, c] += h
        am[:, c] -= h
        lp = np.sum(g * shade(sc, plan, tex, env, nb, albedo=ap), axis=1)
        lm = np.sum(g * shade(sc, plan, tex, env, nb, albedo=am), axis=1)
        e = rel_err((lp - lm) / (ap[:, c].astype(np.float64) - am[:, c]), ad["albedo"][:, c])
        log(f"FD albedo[{c}]: p99 {np.percentile(e, 99):.2e} max {e.max():.2e}")
        assert np.percentile(e, 99) <= 1e-2 and e.max() <= 5e-2


@pytest.mark.parametrize("which", ["tex", "env"])
def test_texture_gradients_match_central_differences(fd_case, which):
    import torch
    sc, plan, tex, env, nb, g, ad = fd_case
    base = (tex if which == "tex" else env).clone()
    grad = ad[which].ravel()
    scale = np.abs(grad).max()
    cand = np.flatnonzero(np.abs(grad) > 1e-3 * scale)
    picks = np.random.default_rng(61).choice(cand, 64, replace=False)
    h = 1e-2
    fd = np.empty(64)
    flat = base.view(-1)
    for n, f in enumerate(picks):
        out = []
        for sgn in (1.0, -1.0):
            pert = base.clone()
            pert.view(-1)[int(f)] = flat[int(f)] + sgn * h
            t, e = (pert, env) if which == "tex" else (tex, pert)
            out.append((np.sum(g * shade(sc, plan, t, e, nb)),
                        float(pert.view(-1)[int(f)].item())))
        fd[n] = (out[0][0] - out[1][0]) / (out[0][1] - out[1][1])
    e = np.abs(fd - grad[picks]) / (np.abs(grad[picks]) + 1e-3 * scale)
    log(f"FD {which}: 64 entries, max {e.max():.2e}")
    torch.cuda.synchronize()
    assert e.max() <= 1e-2
