"""The deterministic adjoint (sop_shade_backward_deterministic): g_env and g_tex are exact
sums of their contributions rounded once, so two runs give the same bits; every gradient
matches the oracle's analytic adjoint (Sec. 3.1.2, Eq. 6-11) as the float-atomic adjoint
does, on the batched kernel (32x32 maps, the benchmark's instantiation), on the general
kernel (64x64 maps) and on the octahedral environment."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2510_07729_amd import scenes
from tests.gpu_util import TOL, dev, gpu_plan, gpu_points, log, oracle_knn, report, sum_err

pytestmark = pytest.mark.gpu

KEYS = ("albedo", "rough", "metal", "env", "tex")


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


def run(sc, grad, deterministic, k=None, n_dirs=None, env=None, g_env=None, g_tex=None):
    from paper_2510_07729_amd import sop
    plan = gpu_plan(sc)
    g = sop.sop_shade_backward(plan, dev(sc.texels), env if env is not None else dev(sc.env),
                               gpu_points(sc), dev(grad), sc.n_dirs if n_dirs is None else n_dirs,
                               k=sc.k if k is None else k, seed=sc.seed, g_env=g_env,
                               g_tex=g_tex, deterministic=deterministic)
    return {key: v.cpu().numpy() for key, v in g.items()}


def check(g, ref, label):
    ok = True
    for key in KEYS:
        ok &= report(f"{label} {key}", sum_err(g[key], ref["g_" + key], ref["m_" + key])) <= TOL
    return ok


def same_bits(a, b):
    return all(np.array_equal(a[key].view(np.uint32), b[key].view(np.uint32)) for key in KEYS)


def test_deterministic_tiny_scene(torch_gpu):
    log("deterministic adjoint: tiny scene (2048 points, S=64, K=4), two runs + oracle")
    sc = scenes.tiny_shade(n_points=2048, seed=41)
    grad = np.random.default_rng(42).standard_normal((sc.n, 3)).astype(np.float32)
    a = run(sc, grad, True)
    b = run(sc, grad, True)
    assert same_bits(a, b)
    idx, w = oracle_knn(sc)
    ref = oracle.shade_backward(sc, idx, w, grad.astype(np.float64), mass=True)
    assert check(a, ref, "det tiny")
    f = run(sc, grad, False)
    assert check(f, ref, "atomic tiny")


@pytest.fixture(scope="module")
def object_subset():
    sc = scenes.object_scene()
    rows = np.random.default_rng(43).choice(sc.n, 1000, replace=False)
    return sc.subset(np.sort(rows))


@pytest.mark.parametrize("fmt", ["f32", "f16"])
def test_deterministic_object_scale_batched(torch_gpu, object_subset, fmt):
    sc = object_subset
    if fmt == "f16":
        sc = dataclasses.replace(sc, texels=sc.texels.astype(np.float16))
    log(f"deterministic adjoint: object scale ({fmt} 32x32 maps, 4096 probes, 1000 points, "
        "S=128, K=8, 256x512 env)")
    grad = np.random.default_rng(44).standard_normal((sc.n, 3)).astype(np.float32)
    a = run(sc, grad, True)
    b = run(sc, grad, True)
    assert same_bits(a, b)
    idx, w = oracle_knn(sc)
    ref = oracle.shade_backward(sc, idx, w, grad.astype(np.float64), mass=True)
    assert check(a, ref, f"det object {fmt}")


def test_deterministic_general_kernel_large_maps(torch_gpu):
    log("deterministic adjoint: 64x64 maps (general kernel), K=8, S=128")
    sc = scenes.tiny_shade(n_points=400, res=64, seed=45)
    grad = np.random.default_rng(46).standard_normal((sc.n, 3)).astype(np.float32)
    a = run(sc, grad, True, k=8, n_dirs=128)
    b = run(sc, grad, True, k=8, n_dirs=128)
    assert same_bits(a, b)
    idx, w = oracle_knn(sc, 8)
    ref = oracle.shade_backward(sc, idx, w, grad.astype(np.float64), n_dirs=128, mass=True)
    assert check(a, ref, "det R=64")


def test_deterministic_octahedral_env(torch_gpu):
    log("deterministic adjoint: octahedral 33x33 sky")
    from paper_2510_07729_amd import sop
    sc = scenes.tiny_shade(n_points=600, seed=47)
    sky = scenes.octahedral_sky(np.random.default_rng(48), 33)
    sc = dataclasses.replace(sc, env=sky, env_oct=True)
    grad = np.random.default_rng(49).standard_normal((sc.n, 3)).astype(np.float32)
    env = sop.OctEnv(dev(sky))
    a = run(sc, grad, True, env=env)
    b = run(sc, grad, True, env=env)
    assert same_bits(a, b)
    idx, w = oracle_knn(sc)
    ref = oracle.shade_backward(sc, idx, w, grad.astype(np.float64), mass=True)
    assert check(a, ref, "det octahedral")


def test_deterministic_accumulates(torch_gpu):
    log("deterministic adjoint accumulates (+=) into g_env / g_tex")
    import torch
    sc = scenes.tiny_shade(n_points=300, seed=50)
    grad = np.random.default_rng(51).standard_normal((sc.n, 3)).astype(np.float32)
    g_env = torch.full(sc.env.shape, 0.5, device="cuda")
    g_tex = torch.full(sc.texels.shape, -0.25, device="cuda")
    run(sc, grad, True, g_env=g_env, g_tex=g_tex)
    fresh = run(sc, grad, True)
    # the exact sum is rounded once and then added to the previous value
    assert np.array_equal(g_env.cpu().numpy(), (np.float32(0.5) + fresh["env"]))
    assert np.array_equal(g_tex.cpu().numpy(), (np.float32(-0.25) + fresh["tex"]))


def test_deterministic_flags_unrepresentable(torch_gpu):
    """A contribution that is not finite turns every g_env and g_tex value of the call into
    NaN (the host forces it through an infinite upstream gradient)."""
    log("deterministic adjoint: an infinite upstream gradient")
    sc = scenes.tiny_shade(n_points=64, seed=52)
    grad = np.random.default_rng(53).standard_normal((sc.n, 3)).astype(np.float32)
    grad[5, 1] = np.inf
    a = run(sc, grad, True)
    assert np.isnan(a["env"]).all() and np.isnan(a["tex"]).all()
