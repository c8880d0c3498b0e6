"""Pins of the oracle's shading with an octahedral environment map (the paper's own
representation of the lighting): a constant sky integrates to pi L; the sky map read as
the environment shades exactly like the same map handed to every probe as its indirect
light with zero occlusion (so the environment lookup is the probe lookup, whose octahedral
convention is pinned elsewhere); and the environment adjoint satisfies the dot-product
identity of a linear map."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2510_07729_amd import scenes

F32 = np.float32


def oct_scene(R=8, n_points=60, P=16, S=64, seed=0):
    sc = scenes.tiny_shade(n_points=n_points, n_probes=P, res=R, H=R, W=R, n_dirs=S)
    g = np.random.default_rng(seed)
    env = g.lognormal(0.0, 1.0, (R, R, 3)).astype(F32)
    return dataclasses.replace(sc, env=env, env_oct=True)


@pytest.mark.parametrize("S", [16, 64, 256])
def test_constant_octahedral_sky_gives_pi_L(S):
    sc = oct_scene(S=S)
    sc = dataclasses.replace(sc, env=np.full_like(sc.env, 1.5))
    tex = np.zeros(sc.texels.shape)                     # no occlusion, no indirect light
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    _, irr = oracle.shade(sc, idx, w, texels=tex, irradiance=True)
    assert np.allclose(irr, np.pi * 1.5, rtol=1e-12)


@pytest.mark.parametrize("per_point", [False, True])
def test_octahedral_sky_reads_like_a_probe_map(per_point):
    sc = oct_scene(R=8)
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    # the sky as the environment, probes empty
    a = oracle.shade(sc, idx, w, texels=np.zeros(sc.texels.shape), per_point=per_point)
    # a black environment, every probe carrying the sky as L_in with O = 0 (weights sum to 1)
    tex = np.zeros(sc.texels.shape)
    tex[..., :3] = sc.env.astype(np.float64)[None]
    b = oracle.shade(sc, idx, w, texels=tex, env=np.zeros_like(sc.env), per_point=per_point)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-15)


def test_octahedral_environment_adjoint_dot_product():
    sc = oct_scene(R=6, n_points=40, S=32)
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    rng = np.random.default_rng(7)
    g = rng.standard_normal((sc.n, 3))
    env = sc.env.astype(np.float64)
    ad = oracle.shade_backward(sc, idx, w, g)
    de = rng.standard_normal(env.shape)
    je = oracle.shade(sc, idx, w, env=env + de) - oracle.shade(sc, idx, w)
    assert np.sum(g * je) == pytest.approx(np.sum(ad["g_env"] * de), rel=1e-9)
