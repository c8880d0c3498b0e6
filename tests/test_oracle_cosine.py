"""Pins of the oracle's cosine-weighted direction set (orc_direction_cos, orc_shade_cosine):
the uniform estimate of Eq. 7 with the density cos(theta)/pi in place of 1/(2 pi), the
cosine-weighted alternative to the uniform set. Checked against closed forms (a
constant sky, the Lambert part, full occlusion), properties of the set itself (the disk
radius, the azimuths of the uniform set, the first moment 2/3 of the cosine density), and
agreement with the uniform set's estimate at many directions."""
import numpy as np
import pytest

import oracle
from paper_2510_07729_amd import scenes


def const_scene(n=64, L=1.5, O=0.0, Lin=0.0, S=64, seed=0):
    sc = scenes.tiny_shade(n_points=n, n_dirs=S, seed=seed)
    tex = np.zeros(sc.texels.shape)
    tex[..., :3] = Lin
    tex[..., 3] = O
    env = np.full(sc.env.shape, L)
    return sc, tex, env


def direction_cos(j, S, rho, n):
    import ctypes as C
    n = np.ascontiguousarray(n, np.float64)
    w = np.zeros(3)
    dp = C.POINTER(C.c_double)
    ct = oracle.lib().orc_direction_cos(j, S, rho, n.ctypes.data_as(dp), w.ctypes.data_as(dp))
    return w, ct


@pytest.mark.parametrize("S", [1, 5, 64, 128])
@pytest.mark.parametrize("per_point", [False, True])
def test_cosine_irradiance_of_constant_sky_is_pi_L(S, per_point):
    sc, tex, env = const_scene(S=S, L=1.5)
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    _, irr = oracle.shade(sc, idx, w, texels=tex, env=env, irradiance=True, cosine=True,
                          per_point=per_point)
    assert np.allclose(irr, np.pi * 1.5, rtol=1e-12)


def test_cosine_irradiance_of_full_occlusion_is_pi_Lin():
    sc, tex, env = const_scene(O=1.0, Lin=0.7, S=7)
    env = np.random.default_rng(61).lognormal(0, 1, env.shape)   # must not matter
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    _, irr = oracle.shade(sc, idx, w, texels=tex, env=env, irradiance=True, cosine=True)
    assert np.allclose(irr, np.pi * 0.7, rtol=1e-12)


@pytest.mark.parametrize("S", [1, 3, 64])
def test_cosine_lambert_part_is_albedo_times_L(S):
    # (pi/S) sum_j (a/pi) L = a L for any S: the density cancels the Lambert cosine exactly
    sc, tex, env = const_scene(L=2.0, S=S)
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    m0 = np.zeros(sc.n)
    a = sc.albedo.astype(np.float64)
    c1 = oracle.shade(sc, idx, w, albedo=a, metal=m0, texels=tex, env=env, cosine=True)
    c0 = oracle.shade(sc, idx, w, albedo=np.zeros_like(a), metal=m0, texels=tex, env=env,
                      cosine=True)
    assert np.allclose(c1 - c0, a * 2.0, rtol=1e-11, atol=1e-13)


def test_cosine_set_geometry():
    rng = np.random.default_rng(62)
    for _ in range(5):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        S = int(rng.integers(1, 300))
        rho = int(rng.integers(0, 1 << 24))
        t, b = oracle.frame(n)
        for j in range(S):
            w, ct = direction_cos(j, S, rho, n)
            u, _ = oracle.direction(j, S, rho, n)
            assert abs(np.linalg.norm(w) - 1.0) < 1e-13
            assert abs(float(w @ n) - ct) < 1e-13 and ct > 0.0
            # squared radius on the unit disk is (j + 0.5) / S
            assert abs((1.0 - ct * ct) - (j + 0.5) / S) < 1e-13
            # the same azimuth as the uniform set's direction j
            az_c = np.arctan2(w @ b, w @ t)
            az_u = np.arctan2(u @ b, u @ t)
            assert abs(np.angle(np.exp(1j * (az_c - az_u)))) < 1e-9


def test_cosine_set_first_moment_is_two_thirds():
    # E[cos theta] under the density cos/pi is 2/3; the set's midpoint rule in the squared
    # radius converges to it (a uniform-in-cos set would give 1/2)
    S = 4096
    n = np.array([0.0, 0.0, 1.0])
    m = np.mean([direction_cos(j, S, 0, n)[1] for j in range(S)])
    assert abs(m - 2.0 / 3.0) < 1e-4


def test_cosine_and_uniform_sets_agree_at_many_directions():
    sc = scenes.tiny_shade(n_points=200, seed=63)
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    _, e_u = oracle.shade(sc, idx, w, n_dirs=4096, irradiance=True)
    _, e_c = oracle.shade(sc, idx, w, n_dirs=4096, irradiance=True, cosine=True)
    rel = np.abs(e_c - e_u) / np.abs(e_u)
    assert np.median(rel) < 2e-3 and np.max(rel) < 1e-2
