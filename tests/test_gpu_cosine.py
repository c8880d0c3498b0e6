"""GPU parity of the cosine-weighted direction set (SOP_SAMPLER_COSINE) against the
oracle's orc_shade_cosine: the estimate of Eq. 7 with the density cos/pi, rgb and
irradiance within 1e-4, on the tiny scene (per-call and per-point rotations, S from 1 to
128, f16 maps, an octahedral sky) and on the object workload; the adjoint refuses it."""
import ctypes as C
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2510_07729_amd import scenes
from tests.gpu_util import TOL, dev, gpu_plan, gpu_points, log, oracle_knn, parity_err, report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


def gpu_cos(sc, S=None, per_point=False, env=None):
    from paper_2510_07729_amd import sop
    plan = gpu_plan(sc)
    rgb, irr = sop.sop_shade(plan, dev(sc.texels), env if env is not None else dev(sc.env),
                             gpu_points(sc), sc.n_dirs if S is None else S, k=sc.k,
                             seed=sc.seed, rotate_per_point=per_point, irradiance=True,
                             cosine=True)
    return rgb.cpu().numpy(), irr.cpu().numpy()


@pytest.mark.parametrize("S,per_point", [(64, False), (128, True), (1, False), (37, True)])
def test_cosine_tiny(torch_gpu, S, per_point):
    log(f"cosine set: tiny scene, S={S}, per_point={per_point}")
    sc = scenes.tiny_shade(n_points=1000, seed=71)
    rgb, irr = gpu_cos(sc, S, per_point)
    idx, w = oracle_knn(sc)
    ref, rirr = oracle.shade(sc, idx, w, n_dirs=S, per_point=per_point, irradiance=True,
                             cosine=True)
    assert report("cosine rgb", parity_err(rgb, ref)) <= TOL
    assert report("cosine irradiance", parity_err(irr, rirr)) <= TOL


def test_cosine_half_texels_and_octahedral_sky(torch_gpu):
    from paper_2510_07729_amd import sop
    log("cosine set: f16 maps under a 33x33 octahedral sky")
    sc = scenes.tiny_shade(n_points=500, seed=72)
    sky = np.random.default_rng(73).lognormal(0.0, 1.0, (33, 33, 3)).astype(np.float32)
    sc = dataclasses.replace(sc, texels=sc.texels.astype(np.float16), env=sky, env_oct=True)
    rgb, irr = gpu_cos(sc, env=sop.OctEnv(dev(sky)))
    idx, w = oracle_knn(sc)
    ref, rirr = oracle.shade(sc, idx, w, irradiance=True, cosine=True)
    assert report("cosine f16/oct rgb", parity_err(rgb, ref)) <= TOL
    assert report("cosine f16/oct irradiance", parity_err(irr, rirr)) <= TOL


def test_cosine_object_scale_sampled(torch_gpu):
    log("cosine set: object workload (200k points, S=128, K=8) in one launch, 300 on oracle")
    sc = scenes.object_scene()
    rgb, irr = gpu_cos(sc)
    rows = np.sort(np.random.default_rng(74).choice(sc.n, 300, replace=False))
    sub = sc.subset(rows)
    idx, w = oracle_knn(sub)
    ref, rirr = oracle.shade(sub, idx, w, irradiance=True, cosine=True)
    assert report("cosine object rgb", parity_err(rgb[rows], ref)) <= TOL
    assert report("cosine object irradiance", parity_err(irr[rows], rirr)) <= TOL


def test_cosine_refused_by_the_adjoint(torch_gpu):
    import torch
    from paper_2510_07729_amd import _lib as L
    from paper_2510_07729_amd import sop
    sc = scenes.tiny_shade(n_points=16, seed=75)
    plan = gpu_plan(sc)
    o = sop.shade_opts(16, 4, cosine=True)
    assert o.sampler == L.SOP_SAMPLER_COSINE
    m, e, cp = sop._maps(dev(sc.texels)), sop._env(dev(sc.env)), gpu_points(sc).c()
    grad = torch.zeros((sc.n, 3), device="cuda")
    ga = torch.empty((sc.n, 3), device="cuda")
    st = plan._lib.sop_shade_backward(plan.handle, C.byref(m), C.byref(e), C.byref(cp), None,
                                      C.byref(o), grad.data_ptr(), ga.data_ptr(), None, None,
                                      None, None, None, 0, None)
    assert st == L.SOP_ERR_UNSUPPORTED
    assert b"cosine" in plan._lib.sop_last_error()
