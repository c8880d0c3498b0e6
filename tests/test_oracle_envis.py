"""Pins of the oracle's relighting with environment importance sampling (Sec. 3.3: object
relighting is estimated with the draws and density of Eq. 18, the draws being those of the
cast-shadow ratio, pinned in test_oracle_shadow.py). The estimate weights every draw by
1/pdf with pdf = (m_t / C) R^2 / (4 pi), so with S = R^2 q draws, which the stratified mass
line spreads q to a texel when the masses are equal, it converges to 4 pi times the mean of
the integrand over the octahedral square. These tests compare with that mean taken by an
independent midpoint quadrature (its own octahedral decode, written out here), for a
constant sky in closed form and for a full scene point."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2510_07729_amd import scenes

F32 = np.float32


def decode(u, v, R):
    """Octahedral decode of texel coordinates (u, v) in [0, R]^2 (+z at the centre)."""
    px, py = 2.0 * u / R - 1.0, 2.0 * v / R - 1.0
    z = 1.0 - np.abs(px) - np.abs(py)
    lower = z < 0.0
    fx = (1.0 - np.abs(py)) * np.where(px < 0.0, -1.0, 1.0)
    fy = (1.0 - np.abs(px)) * np.where(py < 0.0, -1.0, 1.0)
    px, py = np.where(lower, fx, px), np.where(lower, fy, py)
    w = np.stack([px, py, z], axis=-1)
    return w / np.linalg.norm(w, axis=-1, keepdims=True)


def square_dirs(R, sub):
    """Midpoints of a sub x sub grid inside every texel of an R x R square: [R*R*sub^2, 3]."""
    g = (np.arange(R * sub) + 0.5) / sub
    u, v = np.meshgrid(g, g)
    return decode(u.ravel(), v.ravel(), R)


def one_point(n, seed=0, R=8, P=6):
    """A point with normal n, view on its hemisphere, random material, P probes with random
    maps (occlusion in [0,1]) and its four neighbours."""
    g = np.random.default_rng(seed)
    n = np.asarray(n, np.float64)
    n = (n / np.linalg.norm(n)).astype(F32)
    v = g.standard_normal(3)
    v -= 2.0 * min(0.0, float(v @ n)) * n
    v = (v / np.linalg.norm(v)).astype(F32)
    probes = g.uniform(-0.5, 0.5, (P, 3)).astype(F32)
    tex = np.zeros((P, R, R, 4), F32)
    tex[..., :3] = g.uniform(0, 1, (P, R, R, 3))
    tex[..., 3] = g.uniform(0, 1, (P, R, R))
    lo, hi = np.full(3, -1.0, F32), np.full(3, 1.0, F32)
    pos = np.zeros((1, 3), F32)
    sc = scenes.ShadeScene("one", probes, lo, hi, tex, None, pos, n[None], v[None], None, 0,
                           g.uniform(0, 1, (1, 3)).astype(F32),
                           np.array([g.uniform(0.3, 1.0)], F32),
                           np.array([g.uniform(0, 1)], F32), 64, 4)
    idx, w = oracle.knn(probes, lo, hi, pos, sc.normal, 4)
    return sc, idx, w


@pytest.mark.parametrize("n", [(0, 0, 1), (0, 0, -1), (0.3, -0.5, 0.81), (1, 0, 0)])
def test_constant_sky_irradiance_is_four_pi_times_the_square_mean_of_the_cosine(n):
    Re, L = 8, 1.7
    sc, idx, w = one_point(n, seed=1)
    sc = dataclasses.replace(sc, texels=np.zeros_like(sc.texels),
                             env=np.full((Re, Re, 3), L, F32), env_oct=True)
    S = Re * Re * 256                                  # equal masses: 256 draws per texel
    _, irr, tx = oracle.shade_envis(sc, idx, w, n_dirs=S, seed=3, irradiance=True,
                                    texels_out=True)
    assert np.array_equal(np.bincount(tx[0], minlength=Re * Re), np.full(Re * Re, 256))
    d = square_dirs(Re, 32)
    ref = 4.0 * np.pi * L * np.mean(np.maximum(d @ sc.normal[0].astype(np.float64), 0.0))
    # the draws sit at hashed places inside their texels: Monte Carlo error ~1e-3
    assert irr[0] == pytest.approx(np.full(3, ref), rel=5e-3)


def test_importance_estimate_converges_to_the_square_mean_of_the_integrand():
    """A full point (GGX/Lambert BRDF, probes, octahedral sky): the estimate at q draws per
    texel of a sky with equal masses against 4 pi times the midpoint mean of f L_i cos+ over
    the square; L_i = (1 - O) L_env + L_in from the oracle's own pinned lookups."""
    Re = 8
    sc, idx, w = one_point((0.2, 0.4, 0.89), seed=2)
    env = np.full((Re, Re, 3), 1.0, F32)
    env[..., 0] += np.random.default_rng(5).uniform(-1e-3, 1e-3, (Re, Re))   # masses stay equal
    sc = dataclasses.replace(sc, env=env, env_oct=True)
    rgb, irr = oracle.shade_envis(sc, idx, w, n_dirs=Re * Re * 256, seed=4, irradiance=True)
    d = square_dirs(Re, 16)
    n, v = sc.normal[0].astype(np.float64), sc.view[0].astype(np.float64)
    ct = d @ n
    keep = ct > 0
    dk = d[keep]
    Lin, O = oracle.query(sc.texels.astype(np.float64), idx, w, dk[None])
    E = np.array([oracle.oct_fetch(env.astype(np.float64), x) for x in dk])
    Li = (1.0 - O[0][:, None]) * E + Lin[0]
    f = np.array([oracle.brdf(n, v, x, sc.albedo[0].astype(np.float64), float(sc.rough[0]),
                              float(sc.metal[0])) for x in dk])
    ref_rgb = 4.0 * np.pi * np.sum(f * Li * ct[keep][:, None], axis=0) / d.shape[0]
    ref_irr = 4.0 * np.pi * np.sum(Li * ct[keep][:, None], axis=0) / d.shape[0]
    assert irr[0] == pytest.approx(ref_irr, rel=3e-3)
    assert rgb[0] == pytest.approx(ref_rgb, rel=3e-3)


def test_bright_texel_takes_its_share_of_the_draws_and_the_weights_undo_it():
    """A sky whose one texel is 1000x brighter: that texel takes its mass share of the draws
    (stratified), and the irradiance still converges to the same square mean as with equal
    masses, because 1/pdf undoes the choice (dropping the 1/pdf weight would inflate the
    bright texel's share ~100x)."""
    Re = 8
    sc, idx, w = one_point((0, 0, 1), seed=3)
    env = np.full((Re, Re, 3), 1.0, F32)
    t_hot = 3 * Re + 4                                 # upper hemisphere, near the centre
    env.reshape(-1, 3)[t_hot] = 1000.0
    sc = dataclasses.replace(sc, texels=np.zeros_like(sc.texels), env=env, env_oct=True)
    S = 1 << 15
    _, irr, tx = oracle.shade_envis(sc, idx, w, n_dirs=S, seed=6, irradiance=True,
                                    texels_out=True)
    mass, prefix = oracle.env_masses(env)
    share = np.mean(tx[0] == t_hot)
    assert share == pytest.approx(mass[t_hot] / float(prefix[-1]), abs=2.0 / S)
    d = square_dirs(Re, 32)
    L = np.array([oracle.oct_fetch(env.astype(np.float64), x)[0] for x in d])
    ref = 4.0 * np.pi * np.mean(L * np.maximum(d @ sc.normal[0].astype(np.float64), 0.0))
    assert irr[0, 0] == pytest.approx(ref, rel=2e-2)


# ------------------------------------------------------------------------------------------
# the same draws weighted by their exact density (m_t / C) (R^2 / 4) / s^3
# ------------------------------------------------------------------------------------------
def encode(w, R):
    """Texel coordinates (u, v) in [0, R]^2 of a unit direction (inverse of decode)."""
    w = np.asarray(w, np.float64)
    p = w / np.sum(np.abs(w))
    px, py = p[0], p[1]
    if p[2] < 0.0:
        px, py = (1.0 - abs(p[1])) * (1.0 if p[0] >= 0 else -1.0), \
                 (1.0 - abs(p[0])) * (1.0 if p[1] >= 0 else -1.0)
    return (px + 1.0) * R / 2.0, (py + 1.0) * R / 2.0


def test_exact_density_is_the_mass_over_the_numerical_area_element():
    """pdf of a draw = (m_t / C) / |dw/du x dw/dv| with the Jacobian of this file's own
    decode taken by central differences (texel units: a texel has area 1), independent of
    the s^3 formula."""
    Re = 8
    env = np.random.default_rng(7).lognormal(0.0, 1.0, (Re, Re, 3)).astype(F32)
    mass, prefix = oracle.env_masses(env)
    C = float(prefix[-1])
    h = 1e-5
    for j in range(0, 256, 7):
        t, w, pdf = oracle.env_draw(mass, prefix, Re, 256, j, 5, 3, exact=True)
        u, v = encode(w, Re)
        assert np.allclose(decode(u, v, Re), w, atol=1e-12)
        du = (decode(u + h, v, Re) - decode(u - h, v, Re)) / (2 * h)
        dv = (decode(u, v + h, Re) - decode(u, v - h, Re)) / (2 * h)
        area = np.linalg.norm(np.cross(du, dv))
        assert pdf == pytest.approx(mass[t] / C / area, rel=1e-6)
        _, w2, pdf_paper = oracle.env_draw(mass, prefix, Re, 256, j, 5, 3)
        assert np.array_equal(w, w2)               # the same draw, only the density differs
        assert pdf_paper == pytest.approx(mass[t] / C * Re * Re / (4 * np.pi), rel=1e-12)


@pytest.mark.parametrize("n", [(0, 0, 1), (0, 0, -1), (0.3, -0.5, 0.81), (1, 0, 0)])
def test_exact_density_constant_sky_irradiance_is_pi_L(n):
    """With the exact density the estimate is unbiased: a constant sky L gives pi L for
    every normal (the biased density of Eq. 18 gives 4 pi L times the square mean of cos+
    instead, pinned above)."""
    Re, L = 8, 1.7
    sc, idx, w = one_point(n, seed=1)
    sc = dataclasses.replace(sc, texels=np.zeros_like(sc.texels),
                             env=np.full((Re, Re, 3), L, F32), env_oct=True)
    # 4096 draws per texel: the in-texel spread of 4 s^3 cos+ leaves a Monte Carlo error of
    # ~1e-3 (relative standard deviation, from a quadrature of its per-texel variance)
    _, irr = oracle.shade_envis(sc, idx, w, n_dirs=Re * Re * 4096, seed=3, irradiance=True,
                                exact=True)
    assert irr[0] == pytest.approx(np.full(3, np.pi * L), rel=5e-3)


def test_exact_density_bright_texel_converges_to_the_solid_angle_integral():
    """A sky with one texel 1000x brighter, normal +z: the exact-density irradiance against
    the integral of L cos over the hemisphere by a midpoint rule in spherical coordinates
    (L from the oracle's pinned octahedral lookup)."""
    Re = 8
    sc, idx, w = one_point((0, 0, 1), seed=3)
    env = np.full((Re, Re, 3), 1.0, F32)
    env.reshape(-1, 3)[3 * Re + 4] = 1000.0
    sc = dataclasses.replace(sc, texels=np.zeros_like(sc.texels), env=env, env_oct=True)
    # 2^19 draws: the texels next to the bright one take its bilinear spill-over with few
    # draws (their masses are small), which leaves ~4% of scatter at 2^15 draws
    _, irr = oracle.shade_envis(sc, idx, w, n_dirs=1 << 19, seed=6, irradiance=True,
                                exact=True)
    nt, nph = 192, 384
    th = (np.arange(nt) + 0.5) * (np.pi / 2) / nt
    ph = (np.arange(nph) + 0.5) * 2 * np.pi / nph
    T, P = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    env64 = env.astype(np.float64)
    Lr = np.array([oracle.oct_fetch(env64, x)[0] for x in d])
    wq = (np.cos(T) * np.sin(T)).ravel() * (np.pi / 2 / nt) * (2 * np.pi / nph)
    ref = float(np.sum(Lr * wq))
    assert irr[0, 0] == pytest.approx(ref, rel=2e-2)
