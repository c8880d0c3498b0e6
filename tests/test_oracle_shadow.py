"""Pins of the oracle's cast-shadow ratio (Eq. 15-17) and environment importance sampling
(Eq. 18) against facts that do not go through its code: integer masses in closed form,
the stratification of the draws over the mass line, every draw inside its texel, the
ratio of an object that occludes nothing (1) or a fixed fraction c of every direction
(1 - c) under both samplers, and the irradiance of a constant sky (pi L)."""
import math

import numpy as np
import pytest

import oracle
from paper_2510_07729_amd import scenes

F32 = np.float32


def setup(n_points=40, P=12, R=8, O=None, seed=0):
    g = np.random.default_rng(seed)
    probes = g.uniform(-1, 1, (P, 3)).astype(F32)
    pts = g.uniform(-1, 1, (n_points, 3)).astype(F32)
    nrm = scenes.unit_vectors(g, n_points).astype(F32)
    tex = np.zeros((P, R, R, 4), F32)
    tex[..., :3] = g.uniform(0, 1, (P, R, R, 3))
    tex[..., 3] = g.uniform(0, 1, (P, R, R)) if O is None else O
    lo, hi = np.full(3, -1.2, F32), np.full(3, 1.2, F32)
    idx, w = oracle.knn(probes, lo, hi, pts, nrm, 4)
    return nrm, tex, idx, w


def oct_env(R, seed=1, sigma=1.0):
    return np.random.default_rng(seed).lognormal(0.0, sigma, (R, R, 3)).astype(F32)


def test_masses_closed_form_and_degenerate_maps():
    env = np.zeros((2, 2, 3), F32)
    env[..., 0] = [[0, 1], [2, 4]]          # I_max = 4: 2^14/4 = 4096 exactly
    mass, prefix = oracle.env_masses(env)
    assert mass.tolist() == [1, 1 + 4096, 1 + 8192, 1 + 16384]
    assert prefix.tolist() == [0, 1, 4098, 12291, 28676]
    # black, negative and NaN texels all keep the unit mass
    env = np.array([[[0, 0, 0], [-1, 0, 0]], [[np.nan, 0, 0], [0, 0, 0]]], F32)
    mass, prefix = oracle.env_masses(env)
    assert mass.tolist() == [1, 1, 1, 1] and int(prefix[-1]) == 4


@pytest.mark.parametrize("R,S", [(4, 64), (8, 256), (8, 7)])
def test_draws_are_stratified_over_the_mass_line(R, S):
    """Draw j lies in the j-th of S equal slices of the mass line, so texel t receives
    S m_t / C draws up to one slice at each end of its stretch."""
    env = oct_env(R, seed=R + S)
    mass, prefix = oracle.env_masses(env)
    C = int(prefix[-1])
    for i in (0, 5):
        counts = np.zeros(R * R)
        for j in range(S):
            t, _, _ = oracle.env_draw(mass, prefix, R, S, j, 3, i)
            counts[t] += 1
        assert np.all(np.abs(counts - S * mass / C) < 2.0)


def test_draws_land_in_their_texel_with_the_eq18_density():
    R, S = 8, 128
    env = oct_env(R, seed=4, sigma=1.5)
    mass, prefix = oracle.env_masses(env)
    C = int(prefix[-1])
    for j in range(S):
        t, w, pdf = oracle.env_draw(mass, prefix, R, S, j, 11, 2)
        assert abs(np.linalg.norm(w) - 1.0) < 1e-12
        u, v = oracle.oct_encode(w, R)
        assert t % R - 1e-9 <= u <= t % R + 1 + 1e-9 and t // R - 1e-9 <= v <= t // R + 1 + 1e-9
        assert pdf == pytest.approx(mass[t] / C * R * R / (4 * math.pi), rel=1e-14)


@pytest.mark.parametrize("sampler", [0, 1, 2])
def test_no_occlusion_gives_ratio_one(sampler):
    nrm, tex, idx, w = setup(O=0.0)
    r = oracle.shadow_ratio(nrm, tex, idx, w, oct_env(16), 64, seed=5, sampler=sampler)
    assert np.all(r["ratio"] == 1.0)


@pytest.mark.parametrize("sampler", [0, 1, 2])
@pytest.mark.parametrize("c", [0.25, 0.9])
def test_uniform_occlusion_gives_one_minus_c(sampler, c):
    nrm, tex, idx, w = setup(O=c)
    r = oracle.shadow_ratio(nrm, tex, idx, w, oct_env(16, sigma=1.5), 32, seed=9,
                            per_point=True, sampler=sampler)
    assert np.allclose(r["ratio"], 1.0 - float(F32(c)), rtol=1e-12)   # c as stored (float32)


def test_constant_sky_irradiance_is_pi_L_with_the_hemisphere_set():
    nrm, tex, idx, w = setup()
    L = np.array([0.5, 1.0, 2.0], F32)
    env = np.tile(L, (8, 8, 1))
    r = oracle.shadow_ratio(nrm, tex, idx, w, env, 64, sampler=0)
    assert np.allclose(r["irr"], np.pi * L.astype(np.float64), rtol=1e-12)


def test_black_sky_casts_no_shadow():
    nrm, tex, idx, w = setup()
    env = np.zeros((8, 8, 3), F32)
    for sampler in (0, 1, 2):
        r = oracle.shadow_ratio(nrm, tex, idx, w, env, 16, sampler=sampler)
        assert np.all(r["ratio"] == 1.0) and np.all(r["irr"] == 0.0)


def test_importance_and_hemisphere_estimates_agree_at_many_samples():
    """Not an exact pin: Eq. 18 gives every texel the mean solid angle, so the importance
    estimate weighs directions by the octahedral map's texel-area distortion; for the ratio
    that weighting largely cancels. At 4096 samples the two agree to a few percent."""
    nrm, tex, idx, w = setup(n_points=12)
    env = oct_env(32, seed=6, sigma=0.5)
    a = oracle.shadow_ratio(nrm, tex, idx, w, env, 4096, sampler=0)["ratio"]
    b = oracle.shadow_ratio(nrm, tex, idx, w, env, 4096, sampler=1)["ratio"]
    assert np.max(np.abs(a - b)) < 0.03


def test_importance_irradiance_of_a_constant_sky_matches_quadrature():
    """With a constant sky every texel has the same mass, so Eq. 18 gives pdf = 1/(4 pi)
    and the stratified estimate tends to 4 pi L times the mean of cos+ over the octahedral
    square (uniform in (u, v)); the mean is taken here by a fine midpoint rule over the
    square with its own decode of the map."""
    L = np.array([0.5, 1.0, 2.0], F32)
    R, S = 8, 4096
    env = np.tile(L, (R, R, 1))
    g = np.random.default_rng(2)
    nrm = scenes.unit_vectors(g, 3).astype(F32)
    tex = np.zeros((1, 4, 4, 4), F32)
    idx = np.zeros((3, 1), np.int32)
    w = np.ones((3, 1))
    r = oracle.shadow_ratio(nrm, tex, idx, w, env, S, sampler=1)
    m = 1000
    c = (np.arange(m) + 0.5) / m
    px, py = np.meshgrid(2 * c - 1, 2 * c - 1, indexing="xy")
    z = 1 - np.abs(px) - np.abs(py)
    fx = np.where(z < 0, (1 - np.abs(py)) * np.where(px < 0, -1, 1), px)
    fy = np.where(z < 0, (1 - np.abs(px)) * np.where(py < 0, -1, 1), py)
    d = np.stack([fx, fy, z], -1)
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    for i in range(3):
        mean_cos = np.mean(np.maximum(d @ nrm[i].astype(np.float64), 0.0))
        expect = 4 * np.pi * mean_cos * L.astype(np.float64)
        assert np.allclose(r["irr"][i], expect, rtol=5e-3)


def test_exact_density_importance_ratio_agrees_with_the_hemisphere_set():
    """With the draws' exact density (sampler 2) the importance estimate is unbiased: at
    4096 samples its ratio and irradiance agree with the Hammersley ones to the Monte Carlo
    error, closer than the Eq. 18 density does for the irradiance."""
    nrm, tex, idx, w = setup(n_points=12)
    env = oct_env(32, seed=6, sigma=0.5)
    a = oracle.shadow_ratio(nrm, tex, idx, w, env, 4096, sampler=0)
    b = oracle.shadow_ratio(nrm, tex, idx, w, env, 4096, sampler=1)
    c = oracle.shadow_ratio(nrm, tex, idx, w, env, 4096, sampler=2)
    assert np.max(np.abs(a["ratio"] - c["ratio"])) < 0.03
    err_b = np.max(np.abs(b["irr"] / a["irr"] - 1.0))
    err_c = np.max(np.abs(c["irr"] / a["irr"] - 1.0))
    assert err_c < 0.03 and err_c < err_b
