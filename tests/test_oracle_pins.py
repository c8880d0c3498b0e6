"""Pins of the CPU oracle against what the paper and mathematics fix (no GPU needed).

Each test checks an oracle function against a closed form, an invariant, a library routine
or a brute force that does not share the oracle's formula, so that a dropped term, a wrong
sign or index or a transposed operand in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate
from scipy.spatial import cKDTree

import oracle
from paper_2510_07729_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_dirs(n, seed=0):
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# ------------------------------------------------------------------------------------------
# direction set (Eq. 7: Hammersley set)
# ------------------------------------------------------------------------------------------
def test_bitreverse_against_string_reversal():
    rng = np.random.default_rng(1)
    for x in [0, 1, 2, 3, 0xFFFF, 0x12345678, 0xFFFFFFFF] + list(rng.integers(0, 2**32, 200)):
        x = int(x)
        assert oracle.bitreverse32(x) == int(format(x, "032b")[::-1], 2)


def test_pcg_hash_bits_are_uniform():
    # a hash used as a rotation must spread its top 8 bits evenly (chi-square, 255 dof)
    h = np.array([oracle.pcg_hash(i) for i in range(1 << 15)], dtype=np.uint64)
    counts = np.bincount((h >> 24).astype(np.int64), minlength=256)
    e = h.size / 256
    chi2 = float(np.sum((counts - e) ** 2 / e))
    assert chi2 < 340.0   # p ~ 3e-4 upper tail for 255 dof
    assert len(set(h.tolist())) > 0.999 * h.size


@pytest.mark.parametrize("S", [1, 3, 7, 64, 128, 1000, 4096])
def test_hammersley_cosine_sum_is_half(S):
    # cos(theta_j) = 1 - (j+0.5)/S sums to S/2 exactly: the reason the constant-light
    # irradiance is exactly pi*L for every S
    n = np.array([0.0, 0.0, 1.0])
    cs = [oracle.direction(j, S, 0, n)[1] for j in range(S)]
    assert math.fsum(cs) == pytest.approx(S / 2, abs=1e-12)


def test_directions_on_hemisphere_with_given_cosine():
    for n in list(rand_dirs(20, 3)) + [np.array([0, 0, 1.0]), np.array([0, 0, -1.0]),
                                        np.array([1.0, 0, 0])]:
        for j in range(0, 128, 7):
            w, ct = oracle.direction(j, 128, 12345, n)
            assert np.linalg.norm(w) == pytest.approx(1.0, abs=1e-14)
            assert float(w @ n) == pytest.approx(ct, abs=1e-14)
            assert ct > 0


def test_hammersley_azimuths_are_evenly_spaced():
    # for S a power of two the 24-bit azimuth codes of j < S are a rotated lattice k*2^24/S
    S, rho = 64, 0xABCDE
    n = np.array([0.0, 0.0, 1.0])
    phis = []
    for j in range(S):
        w, _ = oracle.direction(j, S, rho, n)
        phis.append(math.atan2(w[1], w[0]))
    t, b = oracle.frame(n)
    # azimuth measured in the frame (t,b): phi_frame = atan2(w.b, w.t)
    ph = np.sort(np.array([math.atan2(oracle.direction(j, S, rho, n)[0] @ b,
                                      oracle.direction(j, S, rho, n)[0] @ t) for j in range(S)]))
    gaps = np.diff(ph)
    assert np.allclose(gaps, 2 * np.pi / S, atol=1e-12)


def test_frame_is_right_handed_orthonormal():
    for n in list(rand_dirs(200, 4)) + [np.array([0, 0, 1.0]), np.array([0, 0, -1.0]),
                                         np.array([0, 1e-9, -1.0]) / np.linalg.norm([0, 1e-9, -1])]:
        t, b = oracle.frame(n)
        M = np.stack([t, b, n])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-14)
        assert np.allclose(np.cross(t, b), n, atol=1e-14)


# ------------------------------------------------------------------------------------------
# octahedral map (Sec. 3.1.2, probe textures)
# ------------------------------------------------------------------------------------------
def test_oct_special_directions_golden():
    g = json.load(open(os.path.join(GOLDEN, "oct_special.json")))
    R = g["R"]
    for case in g["cases"]:
        uv = oracle.oct_encode(np.array(case["dir"], float), R)
        assert any(np.allclose(uv, c, atol=1e-12) for c in case["uv"]), (case, uv)
        back = oracle.oct_decode(uv[0], uv[1], R)
        assert np.allclose(back, np.array(case["dir"]) / np.linalg.norm(case["dir"]), atol=1e-12)


@pytest.mark.parametrize("R", [2, 16, 32])
def test_oct_round_trip(R):
    for w in rand_dirs(2000, R):
        uv = oracle.oct_encode(w, R)
        assert 0 <= uv[0] <= R and 0 <= uv[1] <= R
        assert np.allclose(oracle.oct_decode(uv[0], uv[1], R), w, atol=1e-14)


def test_oct_texel_centres_round_trip():
    R = 16
    for j in range(R):
        for i in range(R):
            w = oracle.oct_decode(i + 0.5, j + 0.5, R)
            assert np.allclose(oracle.oct_encode(w, R), [i + 0.5, j + 0.5], atol=1e-12)


def test_oct_fetch_constant_and_centres():
    R = 8
    rng = np.random.default_rng(5)
    const = np.full((R, R, 4), 2.5)
    for w in rand_dirs(300, 6):
        assert np.allclose(oracle.oct_fetch(const, w), 2.5, atol=1e-14)
    tex = rng.standard_normal((R, R, 4))
    for j in range(R):
        for i in range(R):
            w = oracle.oct_decode(i + 0.5, j + 0.5, R)
            assert np.allclose(oracle.oct_fetch(tex, w), tex[j, i], atol=1e-12)


def test_oct_fetch_is_bilinear_in_the_interior():
    # texture value = column index: inside the square the fetch returns u - 0.5
    R = 16
    tex = np.tile(np.arange(R, dtype=float)[None, :, None], (R, 1, 1))
    rng = np.random.default_rng(7)
    for _ in range(200):
        u, v = rng.uniform(1.0, R - 1.0, 2)
        w = oracle.oct_decode(u, v, R)
        assert oracle.oct_fetch(tex, w)[0] == pytest.approx(u - 0.5, abs=1e-12)
    tex2 = np.tile(np.arange(R, dtype=float)[:, None, None], (1, R, 1))
    for _ in range(200):
        u, v = rng.uniform(1.0, R - 1.0, 2)
        w = oracle.oct_decode(u, v, R)
        assert oracle.oct_fetch(tex2, w)[0] == pytest.approx(v - 0.5, abs=1e-12)


def test_oct_fetch_is_continuous_across_every_seam():
    # the mirror wrap makes the fetch continuous on the sphere: across the equator fold,
    # across the x=0 / y=0 folds of the lower hemisphere and around -z
    R = 16
    tex = np.random.default_rng(8).standard_normal((R, R, 4))
    rng = np.random.default_rng(9)
    eps = 1e-7
    worst = 0.0
    for _ in range(3000):
        w = rng.standard_normal(3)
        kind = rng.integers(0, 4)
        if kind == 0:
            w[2] = 0.0            # equator: the border of the square
        elif kind == 1:
            w[0] = 0.0; w[2] = -abs(w[2])   # lower-hemisphere fold x = 0
        elif kind == 2:
            w[1] = 0.0; w[2] = -abs(w[2])   # lower-hemisphere fold y = 0
        else:
            w = np.array([rng.normal() * 1e-3, rng.normal() * 1e-3, -1.0])  # around -z
        w /= np.linalg.norm(w)
        d = rng.standard_normal(3)
        d -= (d @ w) * w
        d /= np.linalg.norm(d)
        a = oracle.oct_fetch(tex, (w + eps * d) / np.linalg.norm(w + eps * d))
        b = oracle.oct_fetch(tex, (w - eps * d) / np.linalg.norm(w - eps * d))
        worst = max(worst, float(np.max(np.abs(a - b))))
    # Lipschitz bound: derivative of the fetch <= max|texel diff| * R * O(1) per radian
    assert worst < 1e-4


def test_oct_taps_weights_sum_to_one_and_wrap_in_range():
    R = 16
    rng = np.random.default_rng(10)
    for _ in range(2000):
        u, v = rng.uniform(0, R, 2)
        tap, wt = oracle.oct_taps(u, v, R)
        assert wt.sum() == pytest.approx(1.0, abs=1e-14)
        assert np.all((tap >= 0) & (tap < R * R))
    # a tap just outside the right border at row j reads column R-1, row R-1-j
    tap, wt = oracle.oct_taps(R - 0.25, 3.5, R)
    assert tap[1] == (R - 1 - 3) * R + (R - 1)


# ------------------------------------------------------------------------------------------
# environment map (Eq. 8, L_dir)
# ------------------------------------------------------------------------------------------
def test_env_constant_and_row_column_mapping():
    H, W = 32, 64
    const = np.full((H, W, 3), 1.75)
    for w in rand_dirs(200, 11):
        assert np.allclose(oracle.env_fetch(const, w), 1.75, atol=1e-14)
    cols = np.tile(np.arange(W, dtype=float)[None, :, None], (H, 1, 3))
    rows = np.tile(np.arange(H, dtype=float)[:, None, None], (1, W, 3))
    rng = np.random.default_rng(12)
    for _ in range(300):
        theta = rng.uniform(0.2, np.pi - 0.2)
        phi = rng.uniform(-np.pi + 0.2, np.pi - 0.2)
        w = np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
        u = (phi + np.pi) / (2 * np.pi) * W
        v = theta / np.pi * H
        assert oracle.env_fetch(cols, w)[0] == pytest.approx(u - 0.5, abs=1e-9)
        assert oracle.env_fetch(rows, w)[0] == pytest.approx(v - 0.5, abs=1e-9)


def test_env_azimuth_seam_is_continuous():
    H, W = 16, 32
    env = np.random.default_rng(13).lognormal(0, 1, (H, W, 3))
    for theta in np.linspace(0.1, 3.0, 15):
        a = oracle.env_fetch(env, [np.sin(theta) * np.cos(np.pi - 1e-9),
                                   np.sin(theta) * np.sin(np.pi - 1e-9), np.cos(theta)])
        b = oracle.env_fetch(env, [np.sin(theta) * np.cos(-np.pi + 1e-9),
                                   np.sin(theta) * np.sin(-np.pi + 1e-9), np.cos(theta)])
        assert np.allclose(a, b, rtol=1e-6)


# ------------------------------------------------------------------------------------------
# neighbour search (Eq. 9-11)
# ------------------------------------------------------------------------------------------
def numpy_quantize(x, lo, hi):
    x = np.asarray(x, np.float32)
    lo = np.asarray(lo, np.float32)
    ext = np.max(np.asarray(hi, np.float32) - lo)
    sc = np.float32(32768.0) / np.float32(ext)
    q = np.floor((x - lo) * sc)       # float32 numpy arithmetic
    return np.clip(q, 0, 32767).astype(np.int64), sc


def test_lattice_matches_numpy_single_precision():
    rng = np.random.default_rng(14)
    lo, hi = np.array([-1.05, -1.05, -1.05], np.float32), np.array([1.05, 1.05, 1.05], np.float32)
    x = rng.uniform(-1.2, 1.2, (3000, 3)).astype(np.float32)
    qn, sc = numpy_quantize(x, lo, hi)
    assert oracle.lattice_scale(lo, hi) == float(sc)
    for i in range(0, 3000, 3):
        assert np.array_equal(oracle.quantize(x[i], lo, sc), qn[i])


@pytest.mark.parametrize("P,K,radius", [(64, 4, float("inf")), (300, 8, float("inf")),
                                        (300, 8, 0.35), (5, 8, float("inf")), (0, 4, float("inf"))])
def test_knn_matches_kdtree_on_lattice(P, K, radius):
    rng = np.random.default_rng(P * 31 + K)
    lo, hi = np.full(3, -1.05, np.float32), np.full(3, 1.05, np.float32)
    probes = scenes.unit_vectors(rng, P).astype(np.float32) if P else np.zeros((0, 3), np.float32)
    pts = scenes.unit_vectors(rng, 500).astype(np.float32)
    idx, w = oracle.knn(probes, lo, hi, pts, pts, K, radius)
    if P == 0:
        assert np.all(idx == -1) and np.all(w == 0)
        return
    qp, sc = numpy_quantize(probes, lo, hi)
    qx, _ = numpy_quantize(pts, lo, hi)
    lim = oracle.radius_limit(radius, float(sc))
    tree = cKDTree(qp.astype(np.float64))
    kk = min(K, P)
    dist, nn = tree.query(qx.astype(np.float64), k=kk)
    dist = np.asarray(dist).reshape(len(pts), kk)
    d2_tree = np.rint(dist ** 2).astype(np.int64)
    for i in range(len(pts)):
        sel = idx[i][idx[i] >= 0]
        d2 = np.sum((qp[sel] - qx[i]) ** 2, axis=1)
        if len(sel) and d2[0] == 0:            # exact-hit rule
            assert len(sel) == 1
            continue
        want = d2_tree[i][d2_tree[i] <= lim]
        assert np.array_equal(np.sort(d2), want), i      # same distances as the KD-tree
        # ties broken by the lowest index: every excluded probe at the K-th distance has a
        # larger index than the selected ones at that distance
        all_d2 = np.sum((qp - qx[i]) ** 2, axis=1)
        if len(sel) == kk and len(sel):
            dk = d2[-1]
            tied = np.where(all_d2 == dk)[0]
            chosen = set(sel[d2 == dk].tolist())
            assert chosen == set(sorted(tied.tolist())[:len(chosen)])
        assert abs(w[i][: len(sel)].sum() - 1.0) < 1e-12
        assert np.all(w[i][len(sel):] == 0) and np.all(idx[i][len(sel):] == -1)


def test_knn_back_face_weight_closed_form():
    # two probes at distance a on either side of x along n: w_s equal, w_b = 1.01 and 0.01
    lo, hi = np.full(3, -1.0, np.float32), np.full(3, 1.0, np.float32)
    x = np.array([[0.125, 0.25, 0.0]], np.float32)
    n = np.array([[0.0, 0.0, 1.0]], np.float32)
    probes = np.array([[0.125, 0.25, 0.25], [0.125, 0.25, -0.25]], np.float32)
    idx, w = oracle.knn(probes, lo, hi, x, n, 2)
    assert list(idx[0]) == [0, 1]
    assert w[0][0] == pytest.approx(1.01 / 1.02, abs=1e-15)
    assert w[0][1] == pytest.approx(0.01 / 1.02, abs=1e-15)


def test_knn_inverse_distance_closed_form():
    # probes in the tangent plane (d . n = 0): w_b = 0.51 for all, w ~ 1/|d|
    lo, hi = np.full(3, -1.0, np.float32), np.full(3, 1.0, np.float32)
    x = np.zeros((1, 3), np.float32)
    n = np.array([[0.0, 0.0, 1.0]], np.float32)
    probes = np.array([[0.5, 0, 0], [0, 0.25, 0], [-0.125, 0, 0]], np.float32)
    idx, w = oracle.knn(probes, lo, hi, x, n, 3)
    inv = np.array([8.0, 4.0, 2.0])
    assert list(idx[0]) == [2, 1, 0]
    assert np.allclose(w[0], inv / inv.sum(), atol=1e-15)


def test_exact_probe_value_at_probe_position():
    sc = scenes.tiny_shade(n_points=16)
    pts = sc.probe_pos[:10].copy()
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, pts, pts, 4)
    assert np.all(idx[:, 0] == np.arange(10)) and np.all(idx[:, 1:] == -1)
    tex = sc.texels.astype(np.float64)
    dirs = rand_dirs(10 * 5, 15).reshape(10, 5, 3)
    Lin, O = oracle.query(tex, idx, w, dirs)
    for i in range(10):
        for j in range(5):
            f = oracle.oct_fetch(tex[i], dirs[i, j])
            assert np.allclose(Lin[i, j], f[:3], atol=1e-14) and O[i, j] == pytest.approx(f[3])


def test_query_with_identical_probes_equals_one_probe():
    sc = scenes.tiny_shade(n_points=32)
    tex = np.repeat(sc.texels[:1].astype(np.float64), sc.texels.shape[0], axis=0)
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    dirs = rand_dirs(32 * 3, 16).reshape(32, 3, 3)
    Lin, O = oracle.query(tex, idx, w, dirs)
    for i in range(32):
        for j in range(3):
            f = oracle.oct_fetch(tex[0], dirs[i, j])
            assert np.allclose(Lin[i, j], f[:3], atol=1e-12) and abs(O[i, j] - f[3]) < 1e-12


# ------------------------------------------------------------------------------------------
# BRDF (Eq. 6, the simplified Disney model read as Lambert + GGX)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("alpha", [0.0025, 0.04, 0.3, 1.0])
def test_ggx_ndf_is_normalised(alpha):
    # the microfacet distribution projected onto the macro surface integrates to 1
    val, _ = integrate.quad(lambda th: oracle.ggx_D(math.cos(th), alpha) * math.cos(th) *
                            math.sin(th) * 2 * math.pi, 0, math.pi / 2,
                            points=[min(alpha, 1.0) * 0.5, alpha], limit=400, epsabs=1e-12)
    assert val == pytest.approx(1.0, rel=1e-6)


def test_smith_and_schlick_limits():
    for k in [0.01, 0.2, 0.5]:
        assert oracle.smith_G1(1.0, k) == pytest.approx(1.0)
        assert oracle.smith_G1(0.0, k) == 0.0
    for F0 in [0.04, 0.5, 0.9]:
        assert oracle.schlick_F(F0, 1.0) == pytest.approx(F0)
        assert oracle.schlick_F(F0, 0.0) == pytest.approx(1.0)


def test_brdf_reciprocity_and_lambert_part():
    rng = np.random.default_rng(17)
    n = np.array([0.0, 0.0, 1.0])
    for _ in range(100):
        v, l = rand_dirs(2, int(rng.integers(1 << 30)))
        v[2], l[2] = abs(v[2]) + 0.05, abs(l[2]) + 0.05
        v /= np.linalg.norm(v)
        l /= np.linalg.norm(l)
        a = rng.uniform(0, 1, 3)
        r, m = rng.uniform(0.05, 1), rng.uniform(0, 1)
        assert np.allclose(oracle.brdf(n, v, l, a, r, m), oracle.brdf(n, l, v, a, r, m),
                           rtol=1e-12)
        # metallic = 0: F0 = 0.04 for every channel, so f(a) - f(0) is the Lambert term a/pi
        d = oracle.brdf(n, v, l, a, r, 0.0) - oracle.brdf(n, v, l, np.zeros(3), r, 0.0)
        assert np.allclose(d, a / np.pi, rtol=1e-12)


# ------------------------------------------------------------------------------------------
# shading estimator (Eq. 6-8)
# ------------------------------------------------------------------------------------------
def const_scene(n=64, L=1.5, O=0.0, Lin=0.0, S=64, seed=0):
    sc = scenes.tiny_shade(n_points=n, n_dirs=S, seed=seed)
    tex = np.zeros(sc.texels.shape)
    tex[..., :3] = Lin
    tex[..., 3] = O
    env = np.full(sc.env.shape, L)
    return sc, tex, env


@pytest.mark.parametrize("S", [1, 5, 64, 128])
def test_irradiance_of_constant_sky_is_pi_L(S):
    sc, tex, env = const_scene(S=S, L=1.5)
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    rgb, irr = oracle.shade(sc, idx, w, texels=tex, env=env, irradiance=True)
    assert np.allclose(irr, np.pi * 1.5, rtol=1e-12)


def test_irradiance_of_full_occlusion_is_pi_Lin():
    sc, tex, env = const_scene(O=1.0, Lin=0.7)
    env = np.random.default_rng(18).lognormal(0, 1, env.shape)   # must not matter
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    _, irr = oracle.shade(sc, idx, w, texels=tex, env=env, irradiance=True)
    assert np.allclose(irr, np.pi * 0.7, rtol=1e-12)


def test_lambert_part_of_constant_sky_is_albedo_times_L():
    sc, tex, env = const_scene(L=2.0)
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    m0 = np.zeros(sc.n)
    a = sc.albedo.astype(np.float64)
    c1 = oracle.shade(sc, idx, w, albedo=a, metal=m0, texels=tex, env=env)
    c0 = oracle.shade(sc, idx, w, albedo=np.zeros_like(a), metal=m0, texels=tex, env=env)
    assert np.allclose(c1 - c0, a * 2.0, rtol=1e-11, atol=1e-13)


def test_white_furnace_metal_conserves_energy():
    # metallic = 1, albedo = 1: F = 1 and sum f cos / pdf estimates the GGX directional
    # albedo, which single-scattering Smith microfacets keep in (0, 1]
    sc, tex, env = const_scene(n=64, L=1.0, S=2048)
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    ones = np.ones((sc.n, 3))
    r = np.linspace(0.3, 1.0, sc.n)
    rgb = oracle.shade(sc, idx, w, albedo=ones, metal=np.ones(sc.n), rough=r, texels=tex, env=env)
    assert np.all(rgb > 0.3) and np.all(rgb <= 1.0 + 1e-3)


def test_estimator_converges_in_S():
    sc = scenes.tiny_shade(n_points=48)
    tex = sc.texels.astype(np.float64)
    env = np.full(sc.env.shape, 1.0) + 0.5 * np.sin(np.arange(sc.env.shape[1]))[None, :, None]
    rough = np.full(sc.n, 0.9)
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    ref = oracle.shade(sc, idx, w, rough=rough, texels=tex, env=env, n_dirs=8192)
    errs = [np.sqrt(np.mean((oracle.shade(sc, idx, w, rough=rough, texels=tex, env=env,
                                          n_dirs=S) - ref) ** 2)) for S in (16, 64, 256, 1024)]
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 0.2 * errs[0]


# ------------------------------------------------------------------------------------------
# adjoint (gradients through Eq. 6-9)
# ------------------------------------------------------------------------------------------
def small_diff_scene(n=12):
    sc = scenes.tiny_shade(n_points=n, res=8, H=8, W=16, n_dirs=16)
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, 4)
    return sc, idx, w


def test_adjoint_matches_central_differences_materials():
    sc, idx, w = small_diff_scene()
    g = np.random.default_rng(20).standard_normal((sc.n, 3))
    ad = oracle.shade_backward(sc, idx, w, g)
    base = dict(albedo=sc.albedo.astype(np.float64), rough=sc.rough.astype(np.float64),
                metal=sc.metal.astype(np.float64))

    def L(**kw):
        args = dict(base)
        args.update(kw)
        return float(np.sum(g * oracle.shade(sc, idx, w, **args)))

    for i in range(sc.n):
        for key, gk in (("rough", "g_rough"), ("metal", "g_metal")):
            x = base[key].copy()
            h = 1e-6 * max(1.0, abs(x[i]))
            xp, xm = x.copy(), x.copy()
            xp[i] += h
            xm[i] -= h
            fd = (L(**{key: xp}) - L(**{key: xm})) / (2 * h)
            assert ad[gk][i] == pytest.approx(fd, rel=1e-6, abs=1e-9), (key, i)
        for c in range(3):
            a = base["albedo"].copy()
            h = 1e-6
            ap, am = a.copy(), a.copy()
            ap[i, c] += h
            am[i, c] -= h
            fd = (L(albedo=ap) - L(albedo=am)) / (2 * h)
            assert ad["g_albedo"][i, c] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_adjoint_dot_product_textures_and_env():
    # rgb is linear in the env texels and affine in the probe texels (O enters as (1-O));
    # <g, J d> = <J^T g, d> for random perturbations d
    sc, idx, w = small_diff_scene()
    rng = np.random.default_rng(21)
    g = rng.standard_normal((sc.n, 3))
    tex = sc.texels.astype(np.float64)
    env = sc.env.astype(np.float64)
    ad = oracle.shade_backward(sc, idx, w, g)
    dt = rng.standard_normal(tex.shape)
    de = rng.standard_normal(env.shape)
    base = oracle.shade(sc, idx, w)
    jt = oracle.shade(sc, idx, w, texels=tex + dt) - base
    je = oracle.shade(sc, idx, w, env=env + de) - base
    assert np.sum(g * jt) == pytest.approx(np.sum(ad["g_tex"] * dt), rel=1e-9)
    assert np.sum(g * je) == pytest.approx(np.sum(ad["g_env"] * de), rel=1e-9)


def test_adjoint_single_texel_finite_difference():
    sc, idx, w = small_diff_scene()
    g = np.random.default_rng(22).standard_normal((sc.n, 3))
    ad = oracle.shade_backward(sc, idx, w, g)
    tex = sc.texels.astype(np.float64)
    flat = np.argsort(-np.abs(ad["g_tex"]).ravel())[:6]
    for f in flat:
        tp, tm = tex.copy().ravel(), tex.copy().ravel()
        tp[f] += 1e-3
        tm[f] -= 1e-3
        fd = (np.sum(g * oracle.shade(sc, idx, w, texels=tp.reshape(tex.shape))) -
              np.sum(g * oracle.shade(sc, idx, w, texels=tm.reshape(tex.shape)))) / 2e-3
        assert ad["g_tex"].ravel()[f] == pytest.approx(fd, rel=1e-8)


# ------------------------------------------------------------------------------------------
# bake (ray tracing through 3D Gaussians)
# ------------------------------------------------------------------------------------------
def one_ray_scene(means, scales, opac, colors, quats=None):
    n = len(means)
    q = np.tile([1.0, 0, 0, 0], (n, 1)) if quats is None else np.asarray(quats, float)
    return scenes.GaussianScene(np.asarray(means, np.float32), np.asarray(scales, np.float32),
                                np.asarray(q, np.float32), np.asarray(opac, np.float32),
                                np.asarray(colors, np.float32))


R_BAKE = 4
Z_TEXEL = (R_BAKE // 2) * R_BAKE + R_BAKE // 2   # texel whose centre decodes near +z


def ray_dir():
    return oracle.oct_decode(R_BAKE // 2 + 0.5, R_BAKE // 2 + 0.5, R_BAKE)


def test_bake_empty_scene_is_zero():
    gs = one_ray_scene(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3)))
    out, amb = oracle.bake_rays(gs, np.zeros((1, 3)), R_BAKE, [0], [Z_TEXEL])
    assert np.all(out == 0) and not amb[0]


def test_bake_single_gaussian_on_the_ray():
    d = ray_dir()
    gs = one_ray_scene([0.7 * d], [[0.05, 0.05, 0.05]], [0.6], [[0.2, 0.4, 0.8]])
    out, amb = oracle.bake_rays(gs, np.zeros((1, 3)), R_BAKE, [0], [Z_TEXEL])
    assert np.allclose(out[0, :3], 0.6 * np.array([0.2, 0.4, 0.8]), rtol=1e-6)
    assert out[0, 3] == pytest.approx(0.6, rel=1e-6)       # alpha = opacity at m = 0
    assert out[0, 4] == pytest.approx(0.7, rel=1e-6)       # depth = t*


def test_bake_off_axis_isotropic_gaussian_closed_form():
    d = ray_dir()
    perp = np.cross(d, [1.0, 0, 0])
    perp /= np.linalg.norm(perp)
    s, off, t0 = 0.08, 0.1, 0.9
    gs = one_ray_scene([t0 * d + off * perp], [[s, s, s]], [0.8], [[1.0, 1.0, 1.0]])
    out, _ = oracle.bake_rays(gs, np.zeros((1, 3)), R_BAKE, [0], [Z_TEXEL])
    mean32 = gs.mean[0].astype(np.float64)
    t_star = mean32 @ d
    m2 = (np.linalg.norm(mean32 - t_star * d) / float(np.float32(s))) ** 2
    alpha = 0.8 * math.exp(-m2 / 2)
    assert out[0, 3] == pytest.approx(alpha, rel=1e-6)
    assert out[0, 4] == pytest.approx(t_star, rel=1e-6)


def test_bake_anisotropic_gaussian_through_its_centre():
    d = ray_dir()
    q = np.array([0.9, 0.3, -0.2, 0.25])
    q /= np.linalg.norm(q)
    gs = one_ray_scene([0.5 * d], [[0.2, 0.01, 0.05]], [0.5], [[1, 0, 0]], quats=[q])
    out, _ = oracle.bake_rays(gs, np.zeros((1, 3)), R_BAKE, [0], [Z_TEXEL])
    assert out[0, 3] == pytest.approx(0.5, rel=1e-5)
    assert out[0, 4] == pytest.approx(0.5, rel=1e-5)


def test_bake_two_gaussians_composite_front_to_back():
    d = ray_dir()
    gs = one_ray_scene([0.9 * d, 0.4 * d], [[0.03] * 3, [0.03] * 3], [0.5, 0.7],
                       [[0, 1, 0], [1, 0, 0]])
    out, _ = oracle.bake_rays(gs, np.zeros((1, 3)), R_BAKE, [0], [Z_TEXEL])
    # the nearer one (index 1, t=0.4) first
    assert np.allclose(out[0, :3], [0.7, 0.3 * 0.5, 0.0], rtol=1e-6)
    assert out[0, 3] == pytest.approx(1 - 0.3 * 0.5, rel=1e-6)
    assert out[0, 4] == pytest.approx((0.7 * 0.4 + 0.15 * 0.9) / 0.85, rel=1e-6)


def test_bake_alpha_clamp_cutoff_and_stop():
    d = ray_dir()
    # opacity 1 is clamped to 0.99
    gs = one_ray_scene([0.5 * d], [[0.03] * 3], [1.0], [[1, 1, 1]])
    out, _ = oracle.bake_rays(gs, np.zeros((1, 3)), R_BAKE, [0], [Z_TEXEL])
    assert out[0, 3] == pytest.approx(0.99, rel=1e-6)
    # behind the origin (t* < 0): skipped
    gs = one_ray_scene([-0.5 * d], [[0.03] * 3], [0.9], [[1, 1, 1]])
    out, _ = oracle.bake_rays(gs, np.zeros((1, 3)), R_BAKE, [0], [Z_TEXEL])
    assert out[0, 3] == 0.0
    # far off the ray: alpha < 1/255, skipped
    perp = np.cross(d, [1.0, 0, 0])
    perp /= np.linalg.norm(perp)
    gs = one_ray_scene([0.5 * d + 0.2 * perp], [[0.03] * 3], [0.9], [[1, 1, 1]])
    out, _ = oracle.bake_rays(gs, np.zeros((1, 3)), R_BAKE, [0], [Z_TEXEL])
    assert out[0, 3] == 0.0
    # five opacity-0.95 Gaussians: T = 0.05, 0.0025, 1.25e-4, then 6.25e-6 < 1e-4 stops
    gs = one_ray_scene([(0.2 + 0.1 * i) * d for i in range(5)], [[0.01] * 3] * 5, [0.95] * 5,
                       [[1, 1, 1]] * 5)
    out, amb = oracle.bake_rays(gs, np.zeros((1, 3)), R_BAKE, [0], [Z_TEXEL])
    assert out[0, 3] == pytest.approx(1 - 1.25e-4, rel=1e-9) and not amb[0]


def test_adjoint_summation_scale():
    # the m_* outputs hold sum |term|: never below |gradient|, and equal to it when no term
    # can be negative (albedo gradient with a non-negative upstream gradient and metallic 0)
    sc, idx, w = small_diff_scene()
    g = np.abs(np.random.default_rng(23).standard_normal((sc.n, 3)))
    ad = oracle.shade_backward(sc, idx, w, g, metal=np.zeros(sc.n), mass=True)
    for k in ("albedo", "rough", "metal", "tex", "env"):
        assert np.all(ad["m_" + k] >= np.abs(ad["g_" + k]) * (1 - 1e-12))
    assert np.allclose(ad["m_albedo"], ad["g_albedo"], rtol=1e-12)
    ad2 = oracle.shade_backward(sc, idx, w, g, metal=np.zeros(sc.n))
    assert np.array_equal(ad2["g_tex"], ad["g_tex"]) or np.allclose(ad2["g_tex"], ad["g_tex"],
                                                                       rtol=1e-12, atol=1e-15)
