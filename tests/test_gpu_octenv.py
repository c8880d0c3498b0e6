"""GPU parity of shading with an octahedral environment map (the paper's representation of
the lighting) against the oracle: forward with irradiance, the adjoint (environment
gradient included), the object workload sampled, traced shading, and the calls that take
an equirectangular map only."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2510_07729_amd import scenes
from tests.gpu_util import (TOL, dev, gpu_plan, gpu_points, log, oracle_knn, parity_err,
                            report, sum_err)

pytestmark = pytest.mark.gpu

F32 = np.float32


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


def with_oct_sky(sc, R, seed=0, sigma=1.0):
    env = np.random.default_rng(seed).lognormal(0.0, sigma, (R, R, 3)).astype(F32)
    return dataclasses.replace(sc, env=env, env_oct=True)


def gpu_shade(sc, nb=None, per_point=False):
    from paper_2510_07729_amd import sop
    plan = gpu_plan(sc)
    rgb, irr = sop.sop_shade(plan, dev(sc.texels), sop.OctEnv(dev(sc.env)), gpu_points(sc),
                             sc.n_dirs, k=sc.k, seed=sc.seed, rotate_per_point=per_point,
                             irradiance=True)
    return rgb.cpu().numpy(), irr.cpu().numpy()


@pytest.mark.parametrize("R,per_point", [(16, False), (33, True)])
def test_octahedral_sky_forward(torch_gpu, R, per_point):
    log(f"octahedral sky {R}x{R}: tiny scene forward (1000 points, S=64, K=4)")
    sc = with_oct_sky(scenes.tiny_shade(n_points=1000), R)
    rgb, irr = gpu_shade(sc, per_point=per_point)
    idx, w = oracle_knn(sc)
    ref, rirr = oracle.shade(sc, idx, w, per_point=per_point, irradiance=True)
    assert report("oct rgb", parity_err(rgb, ref)) <= TOL
    assert report("oct irradiance", parity_err(irr, rirr)) <= TOL


def test_octahedral_sky_backward(torch_gpu):
    from paper_2510_07729_amd import sop
    log("octahedral sky 16x16: adjoint on the tiny scene (777 points, S=64, K=4)")
    sc = with_oct_sky(scenes.tiny_shade(n_points=777), 16, seed=3)
    grad = np.random.default_rng(4).standard_normal((sc.n, 3)).astype(F32)
    g = sop.sop_shade_backward(gpu_plan(sc), dev(sc.texels), sop.OctEnv(dev(sc.env)),
                               gpu_points(sc), dev(grad), sc.n_dirs, k=sc.k, seed=sc.seed)
    g = {k: v.cpu().numpy() for k, v in g.items()}
    idx, w = oracle_knn(sc)
    ref = oracle.shade_backward(sc, idx, w, grad.astype(np.float64), mass=True)
    for key in ("albedo", "rough", "metal", "env", "tex"):
        assert report(f"oct {key}", sum_err(g[key], ref["g_" + key], ref["m_" + key])) <= TOL


def test_octahedral_sky_object_sampled(torch_gpu):
    """The object workload (200k points, S=128, K=8) under a 256x256 octahedral sky in one
    launch; 300 sampled points on the oracle."""
    log("octahedral sky 256x256: object workload forward, 300 points on the oracle")
    sc = with_oct_sky(scenes.object_scene(), 256, seed=5, sigma=1.5)
    rgb, irr = gpu_shade(sc)
    rows = np.sort(np.random.default_rng(6).choice(sc.n, 300, replace=False))
    sub = sc.subset(rows)
    idx, w = oracle_knn(sub)
    ref, rirr = oracle.shade(sub, idx, w, irradiance=True)
    assert report("oct object rgb", parity_err(rgb[rows], ref)) <= TOL
    assert report("oct object irradiance", parity_err(irr[rows], rirr)) <= TOL


def test_octahedral_sky_traced_and_rejections(torch_gpu):
    from paper_2510_07729_amd import _lib as L
    from paper_2510_07729_amd import sop
    log("octahedral sky: traced shading; proposal sampler and integrand dump rejected")
    g = np.random.default_rng(8)
    gs = scenes.random_gaussians(g, 200)
    sc = with_oct_sky(scenes.tiny_shade(n_points=120, n_dirs=16), 16, seed=9)
    sc = dataclasses.replace(sc, pos=(0.4 * sc.pos).astype(F32))
    plan = sop.BakePlan(dev(gs.mean), dev(gs.scale), dev(gs.rotation), dev(gs.opacity),
                        dev(gs.color))
    rgb, smp = sop.sop_shade_traced(plan, sop.OctEnv(dev(sc.env)), gpu_points(sc), 16, 0.02,
                                    samples=True)
    ref = oracle.shade_traced(gs, sc, 0.02)
    ok = ~ref["amb"]
    assert ok.mean() > 0.8
    assert report("oct traced rgb", parity_err(rgb.cpu().numpy()[ok], ref["rgb"][ok])) <= TOL
    pplan = gpu_plan(sc)
    probs = dev(scenes.bin_probs(sc.n, seed=1))
    with pytest.raises(L.SopError) as e:
        sop.sop_shade(pplan, dev(sc.texels), sop.OctEnv(dev(sc.env)), gpu_points(sc), 16,
                      k=sc.k, probs=probs)
    assert e.value.status == L.SOP_ERR_UNSUPPORTED
    with pytest.raises(L.SopError) as e:
        sop.sop_dump_integrand(pplan, dev(sc.texels), sop.OctEnv(dev(sc.env)), gpu_points(sc),
                               1, k=sc.k)
    assert e.value.status == L.SOP_ERR_UNSUPPORTED


def test_octahedral_sky_through_autograd(torch_gpu):
    import torch
    from paper_2510_07729_amd import sop
    from paper_2510_07729_amd.autograd import Geometry, shade
    log("octahedral sky: autograd.shade against the direct calls")
    sc = with_oct_sky(scenes.tiny_shade(n_points=300), 16, seed=11)
    plan = gpu_plan(sc)
    geom = Geometry(dev(sc.pos), dev(sc.normal), view=dev(sc.view))
    albedo = dev(sc.albedo).requires_grad_(True)
    env = dev(sc.env).requires_grad_(True)
    rough, metal, tex = dev(sc.rough), dev(sc.metal), dev(sc.texels)
    rgb = shade(albedo, rough, metal, env, tex, plan, geom, sc.n_dirs, sc.k, seed=sc.seed,
                env_oct=True)
    grad = torch.randn_like(rgb)
    rgb.backward(grad)
    pts = gpu_points(sc)
    direct = sop.sop_shade(plan, tex, sop.OctEnv(dev(sc.env)), pts, sc.n_dirs, k=sc.k,
                           seed=sc.seed)
    g = sop.sop_shade_backward(plan, tex, sop.OctEnv(dev(sc.env)), pts, grad, sc.n_dirs,
                               k=sc.k, seed=sc.seed, want=("albedo", "env"))
    assert torch.equal(rgb.detach(), direct)
    assert torch.allclose(albedo.grad, g["albedo"], rtol=1e-6, atol=1e-7)
    assert torch.allclose(env.grad, g["env"], rtol=1e-5, atol=1e-6)
