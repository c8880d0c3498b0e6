"""GPU parity of the shading adjoint (sop_shade_backward) against the oracle's analytic
adjoint, and the autograd.Function around it (the differentiable reconstruction step)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2510_07729_amd import scenes
from tests.gpu_util import (TOL, dev, gpu_plan, gpu_points, log, oracle_knn, parity_err,
                            report, sum_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


def diff_step_inputs():
    """The tiny scene, a target rendered by the oracle with hidden materials and the L2
    loss gradient 2 (rgb - target), all computed on the CPU."""
    sc, (ha, hr, hm) = scenes.diff_step()
    idx, w = oracle_knn(sc)
    target = oracle.shade(sc, idx, w, albedo=ha, rough=hr, metal=hm)
    rgb = oracle.shade(sc, idx, w)
    grad = (2.0 * (rgb - target)).astype(np.float32)
    return sc, idx, w, grad


def run_backward(sc, grad, k=None, per_point=False, n_dirs=None):
    from paper_2510_07729_amd import sop
    plan = gpu_plan(sc)
    g = sop.sop_shade_backward(plan, dev(sc.texels), dev(sc.env), gpu_points(sc), dev(grad),
                               sc.n_dirs if n_dirs is None else n_dirs,
                               k=sc.k if k is None else k, seed=sc.seed,
                               rotate_per_point=per_point)
    return {k2: v.cpu().numpy() for k2, v in g.items()}


def check_all(g, ref, label):
    """Every gradient is a sum over samples (and probes/taps) of signed terms: compared
    relative to max(|sum|, sum of |terms|) from the oracle (asserted). The plain relative
    error with the 1e-3 * mean floor of the forward's metric is logged next to it: where
    the terms cancel, it measures the rounding of the sum against a smaller scale."""
    ok = True
    for key in ("albedo", "rough", "metal", "env", "tex"):
        ok &= report(f"{label} {key}", sum_err(g[key], ref["g_" + key], ref["m_" + key])) <= TOL
        pe = parity_err(g[key], ref["g_" + key])
        if pe.size:
            log(f"{label} {key} (floored relative error): max {pe.max():.3e} "
                f"p99.99 {np.percentile(pe, 99.99):.3e}")
    return ok


def test_backward_diff_step_parity(torch_gpu):
    log("backward: tiny scene L2 step (4096 points, S=64, K=4)")
    sc, idx, w, grad = diff_step_inputs()
    g = run_backward(sc, grad)
    ref = oracle.shade_backward(sc, idx, w, grad.astype(np.float64), mass=True)
    assert check_all(g, ref, "diff step")


@pytest.mark.parametrize("k,n_dirs,per_point,n", [(8, 128, False, 700), (3, 37, True, 333)])
def test_backward_variants(torch_gpu, k, n_dirs, per_point, n):
    log(f"backward variant K={k} S={n_dirs} per_point={per_point} N={n}")
    sc = scenes.tiny_shade(n_points=n, seed=7)
    grad = np.random.default_rng(8).standard_normal((n, 3)).astype(np.float32)
    g = run_backward(sc, grad, k=k, n_dirs=n_dirs, per_point=per_point)
    idx, w = oracle_knn(sc, k)
    ref = oracle.shade_backward(sc, idx, w, grad.astype(np.float64), n_dirs=n_dirs,
                                per_point=per_point, mass=True)
    assert check_all(g, ref, f"K={k} S={n_dirs}")


def test_backward_half_texels(torch_gpu):
    log("backward with f16 textures (gradient f32)")
    sc = scenes.tiny_shade(n_points=500, seed=9)
    sc.texels = sc.texels.astype(np.float16)
    grad = np.random.default_rng(10).standard_normal((sc.n, 3)).astype(np.float32)
    g = run_backward(sc, grad)
    idx, w = oracle_knn(sc)
    ref = oracle.shade_backward(sc, idx, w, grad.astype(np.float64), mass=True)
    assert check_all(g, ref, "f16")


def test_backward_accumulates_into_texture_gradients(torch_gpu):
    log("backward accumulates (+=) into g_env / g_tex")
    import torch
    from paper_2510_07729_amd import sop
    sc = scenes.tiny_shade(n_points=300, seed=12)
    grad = np.random.default_rng(13).standard_normal((sc.n, 3)).astype(np.float32)
    plan = gpu_plan(sc)
    pts = gpu_points(sc)
    g_env = torch.full(sc.env.shape, 0.5, device="cuda")
    g_tex = torch.full(sc.texels.shape, -0.25, device="cuda")
    sop.sop_shade_backward(plan, dev(sc.texels), dev(sc.env), pts, dev(grad), 64, k=4,
                           g_env=g_env, g_tex=g_tex)
    fresh = sop.sop_shade_backward(plan, dev(sc.texels), dev(sc.env), pts, dev(grad), 64, k=4)
    assert torch.allclose(g_env - 0.5, fresh["env"], rtol=1e-5, atol=1e-6)
    assert torch.allclose(g_tex + 0.25, fresh["tex"], rtol=1e-5, atol=1e-6)


def test_autograd_function_matches_direct_call_and_descends(torch_gpu):
    log("SopShade autograd: gradients and a few Adam steps")
    import torch
    from paper_2510_07729_amd import sop
    from paper_2510_07729_amd.autograd import Geometry, shade
    sc, (ha, hr, hm) = scenes.diff_step()
    plan = gpu_plan(sc)
    geom = Geometry(dev(sc.pos), dev(sc.normal), view=dev(sc.view))
    pts_h = gpu_points(sc, ha, hr, hm)
    nb = sop.sop_knn(plan, pts_h, 4)
    target = sop.sop_shade(plan, dev(sc.texels), dev(sc.env), pts_h, 64, nb=nb)
    albedo = dev(sc.albedo).requires_grad_(True)
    rough = dev(sc.rough).requires_grad_(True)
    metal = dev(sc.metal).requires_grad_(True)
    env = dev(sc.env).requires_grad_(True)
    tex = dev(sc.texels).requires_grad_(True)
    rgb = shade(albedo, rough, metal, env, tex, plan, geom, 64, 4, nb=nb)
    loss = ((rgb - target) ** 2).sum()
    loss.backward()
    direct = sop.sop_shade_backward(plan, tex.detach(), env.detach(),
                                    gpu_points(sc), (2 * (rgb - target)).detach(), 64, nb=nb)
    assert torch.allclose(albedo.grad, direct["albedo"], rtol=1e-6, atol=1e-7)
    assert torch.allclose(rough.grad, direct["rough"], rtol=1e-6, atol=1e-7)
    assert torch.allclose(tex.grad, direct["tex"], rtol=1e-4, atol=1e-6)
    # learning rates of the paper's step 2 (0.01 materials and env, 0.001 textures)
    opt = torch.optim.Adam([{"params": [albedo, rough, metal, env], "lr": 0.01},
                            {"params": [tex], "lr": 0.001}])
    losses = [float(loss)]
    for _ in range(5):
        opt.zero_grad()
        with torch.no_grad():
            rough.clamp_(0.05, 1.0)
            metal.clamp_(0.0, 1.0)
            albedo.clamp_(0.0, 1.0)
        rgb = shade(albedo, rough, metal, env, tex, plan, geom, 64, 4, nb=nb)
        loss = ((rgb - target) ** 2).sum()
        loss.backward()
        opt.step()
        losses.append(float(loss))
    log(f"losses {losses}")
    assert losses[-1] < 0.8 * losses[0]


@pytest.fixture(scope="module")
def object_subset():
    """1000 points of the object workload with all its 4096 probes (32x32 maps), K = 8,
    S = 128 and the 256x512 environment."""
    sc = scenes.object_scene()
    rows = np.random.default_rng(31).choice(sc.n, 1000, replace=False)
    return sc.subset(np.sort(rows))


@pytest.mark.parametrize("fmt", ["f32", "f16"])
def test_backward_object_scale_batched(torch_gpu, object_subset, fmt):
    """The benchmark's instantiation of the batched adjoint: 32x32 maps (every thread owns
    8 values of a map, ~154 KB of dynamic LDS), K = 8, S = 128, 256x512 environment."""
    sc = object_subset
    if fmt == "f16":
        sc = dataclasses.replace(sc, texels=sc.texels.astype(np.float16))
    log(f"backward object scale ({fmt} maps 32x32, 4096 probes, 1000 points, S=128, K=8)")
    grad = np.random.default_rng(32).standard_normal((sc.n, 3)).astype(np.float32)
    g = run_backward(sc, grad)
    idx, w = oracle_knn(sc)
    ref = oracle.shade_backward(sc, idx, w, grad.astype(np.float64), mass=True)
    assert check_all(g, ref, f"object {fmt}")


@pytest.mark.parametrize("fmt,k,n_dirs", [("f32", 8, 128), ("f16", 4, 64)])
def test_backward_large_maps_general_kernel(torch_gpu, fmt, k, n_dirs):
    """64x64 maps do not fit the batched kernel's LDS: the one-wavefront-per-point adjoint
    with scattered atomics takes them."""
    log(f"backward 64x64 maps ({fmt}, K={k}, S={n_dirs}): general kernel")
    sc = scenes.tiny_shade(n_points=400, res=64, seed=21)
    if fmt == "f16":
        sc.texels = sc.texels.astype(np.float16)
    grad = np.random.default_rng(22).standard_normal((sc.n, 3)).astype(np.float32)
    g = run_backward(sc, grad, k=k, n_dirs=n_dirs)
    idx, w = oracle_knn(sc, k)
    ref = oracle.shade_backward(sc, idx, w, grad.astype(np.float64), n_dirs=n_dirs, mass=True)
    assert check_all(g, ref, f"R=64 {fmt}")


def test_backward_list_naming_a_probe_twice(torch_gpu):
    """Caller-given neighbour lists may name a probe twice: forward and adjoint count both
    entries, as Eq. 9 read literally does."""
    log("neighbour lists with a repeated probe")
    import torch
    from paper_2510_07729_amd import sop
    sc = scenes.tiny_shade(n_points=300, seed=23)
    idx, w = oracle_knn(sc)
    idx = idx.copy()
    w = w.copy()
    idx[::3, 2] = idx[::3, 0]              # every third point lists its nearest probe twice
    w = w / w.sum(axis=1, keepdims=True)
    nb = sop.Neighbors(None, dev(idx.astype(np.int32)), dev(w.astype(np.float32)))
    grad = np.random.default_rng(24).standard_normal((sc.n, 3)).astype(np.float32)
    plan = gpu_plan(sc)
    pts = gpu_points(sc)
    rgb = sop.sop_shade(plan, dev(sc.texels), dev(sc.env), pts, sc.n_dirs, nb=nb, seed=sc.seed)
    g = sop.sop_shade_backward(plan, dev(sc.texels), dev(sc.env), pts, dev(grad), sc.n_dirs,
                               nb=nb, seed=sc.seed)
    torch.cuda.synchronize()
    wf = w.astype(np.float32).astype(np.float64)
    ro = oracle.shade(sc, idx, wf)
    assert report("repeated probe forward", parity_err(rgb.cpu().numpy(), ro)) <= TOL
    ref = oracle.shade_backward(sc, idx, wf, grad.astype(np.float64), mass=True)
    assert check_all({k2: v.cpu().numpy() for k2, v in g.items()}, ref, "repeated probe")


@pytest.mark.parametrize("hw,oct_sky", [((1, 1), False), ((1, 2), False), ((2, 1), False),
                                         ((3, 5), False), ((4, 3), False), ((2, 2), True),
                                         ((3, 3), True)])
def test_backward_small_environments(torch_gpu, hw, oct_sky):
    """Environments of a few texels: every bilinear footprint wraps (columns) and clamps
    (rows), or mirrors (octahedral), so the environment adjoint's 2x2 blocks fold back onto
    few texels, each from several block offsets."""
    from paper_2510_07729_amd import sop
    log(f"backward with a {hw[0]}x{hw[1]} {'octahedral' if oct_sky else 'equirectangular'} sky")
    sc = scenes.tiny_shade(n_points=300, seed=41)
    sky = np.random.default_rng(42).lognormal(0.0, 0.7, (*hw, 3)).astype(np.float32)
    sc = dataclasses.replace(sc, env=sky, env_oct=oct_sky)
    grad = np.random.default_rng(43).standard_normal((sc.n, 3)).astype(np.float32)
    plan = gpu_plan(sc)
    env = sop.OctEnv(dev(sky)) if oct_sky else dev(sky)
    g = sop.sop_shade_backward(plan, dev(sc.texels), env, gpu_points(sc), dev(grad),
                               sc.n_dirs, k=sc.k, seed=sc.seed)
    g = {k2: v.cpu().numpy() for k2, v in g.items()}
    idx, w = oracle_knn(sc)
    ref = oracle.shade_backward(sc, idx, w, grad.astype(np.float64), mass=True)
    assert check_all(g, ref, f"sky {hw} oct={oct_sky}")


def test_backward_sky_beyond_the_block_limit(torch_gpu):
    """A 2050x4100 sky (8.4M texels, above the 4096x2048 limit of the environment blocks):
    the float adjoint adds its environment gradient as runs straight into g_env, and the
    workspace holds no blocks."""
    from paper_2510_07729_amd import _lib as L
    from paper_2510_07729_amd import sop
    log("backward under a 2050x4100 sky: environment runs instead of blocks")
    sc = scenes.tiny_shade(n_points=120, seed=51)
    H, W = 2050, 4100
    sky = np.random.default_rng(52).lognormal(0.0, 0.5, (H, W, 3)).astype(np.float32)
    sc = dataclasses.replace(sc, env=sky)
    grad = np.random.default_rng(53).standard_normal((sc.n, 3)).astype(np.float32)
    plan = gpu_plan(sc)
    small = plan.workspace_size(L.SOP_OP_SHADE_BACKWARD, sc.n, sc.k, sc.n_dirs, (H, W - 8))
    large = plan.workspace_size(L.SOP_OP_SHADE_BACKWARD, sc.n, sc.k, sc.n_dirs, (H, W))
    assert large < small          # 4092 columns still take blocks, 4100 do not
    g = sop.sop_shade_backward(plan, dev(sc.texels), dev(sky), gpu_points(sc), dev(grad),
                               sc.n_dirs, k=sc.k, seed=sc.seed)
    g = {k2: v.cpu().numpy() for k2, v in g.items()}
    idx, w = oracle_knn(sc)
    ref = oracle.shade_backward(sc, idx, w, grad.astype(np.float64), mass=True)
    assert check_all(g, ref, "sky 2050x4100")
