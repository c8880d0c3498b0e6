"""Pins of the oracle's learned direction proposal (features, network, training, bin
sampler, proposal shading and training targets) against closed forms, an independent
rounding route, finite differences, independent quadrature of the sampling density and
statistical agreement with the fixed-direction estimate of Eq. 7."""
import math

import numpy as np
import pytest

import oracle
from paper_2510_07729_amd import scenes

OFF = oracle.mlp_offsets()


# ---------------------------------------------------------------------------- bfloat16
def bf16_by_bits(x32: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even of float32 values to bfloat16 by integer bit arithmetic."""
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_rounding_matches_bit_route():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(2000) * 10.0 ** rng.uniform(-20, 20, 2000),
        np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 2 ** -130, 3 * 2 ** -134,
                  65504.0, 1e-39, -7e-40], np.float64)]).astype(np.float32)
    want = bf16_by_bits(x)
    got = np.array([oracle.bf16(float(v)) for v in x])
    assert np.array_equal(got, want)
    assert oracle.bf16(1 + 2 ** -8) == 1.0                  # tie to even (down)
    assert oracle.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6      # tie to even (up)


# ---------------------------------------------------------------------------- features
def test_feature_layout_closed_forms():
    lo, hi = np.full(3, -1.0), np.full(3, 1.0)
    s2 = 1.0 / math.sqrt(2.0)
    f = oracle.pe_features(np.array([-1.0, 0.0, 1.0]), np.array([0.0, 0.0, 1.0]),
                           np.array([s2, s2, 0.0]), 0.5, lo, hi)
    sin = lambda c, l: f[32 * c + 2 * l]          # noqa: E731
    cos = lambda c, l: f[32 * c + 2 * l + 1]      # noqa: E731
    # scalar 1 (y position 0): sin 0 = 0, cos 0 = 1 at every frequency
    for l in range(16):
        assert sin(1, l) == 0.0 and cos(1, l) == 1.0
    # scalar 0 (x = -1) and scalar 5 (n_z = 1): even l has integer f = 2^(l/2)
    assert abs(cos(0, 0) + 1.0) < 1e-15 and abs(cos(5, 0) + 1.0) < 1e-15
    for l in range(2, 16, 2):
        assert abs(sin(0, l)) < 1e-12 and abs(cos(0, l) - 1.0) < 1e-15
    # scalar 6 (v_x = 1/sqrt 2): l = 1 has f = sqrt 2, so the argument is pi
    assert abs(sin(6, 1)) < 1e-15 and abs(cos(6, 1) + 1.0) < 1e-15
    # scalar 9 (roughness 0.5): pi/2, pi, 2 pi at l = 0, 2, 4
    assert abs(sin(9, 0) - 1.0) < 1e-15 and abs(cos(9, 0)) < 1e-15
    assert abs(cos(9, 2) + 1.0) < 1e-15 and abs(cos(9, 4) - 1.0) < 1e-15
    # every pair lies on the unit circle
    assert np.allclose(f[0::2] ** 2 + f[1::2] ** 2, 1.0, atol=1e-14)


# ---------------------------------------------------------------------------- network
def feat0():
    rng = np.random.default_rng(3)
    return oracle.pe_features(rng.uniform(-1, 1, 3), np.array([0, 0, 1.0]),
                              np.array([0, 1.0, 0]), 0.3, np.full(3, -1.0), np.full(3, 1.0))


def test_zero_network_is_uniform():
    P = np.zeros(oracle.mlp_param_count())
    out = oracle.mlp_forward(P, feat0())
    assert np.all(out["z3"] == 0.0) and np.allclose(out["q"], 1.0 / 256, rtol=1e-15)
    rng = np.random.default_rng(0)
    B = 5
    pos, n = rng.uniform(-1, 1, (B, 3)), rng.standard_normal((B, 3))
    T = rng.uniform(0, 1, (B, 256))
    loss, g = oracle.mlp_loss_grad(P, pos, n, n, rng.uniform(0, 1, B), -np.ones(3),
                                   np.ones(3), T)
    assert abs(loss - math.log(256.0)) < 1e-13
    t = T / T.sum(1, keepdims=True)
    assert np.allclose(g[OFF["b3"]], (1.0 / 256 - t).mean(0), atol=1e-15)
    assert np.all(g[OFF["W1"]] == 0.0)       # no signal reaches the first layer


def test_biases_only_network():
    rng = np.random.default_rng(1)
    P = np.zeros(oracle.mlp_param_count())
    P[OFF["b3"]] = rng.standard_normal(256)
    P[OFF["b1"]] = rng.standard_normal(64)
    out = oracle.mlp_forward(P, feat0(), emulate_bf16=False)
    e = np.exp(P[OFF["b3"]] - P[OFF["b3"]].max())
    assert np.allclose(out["q"], e / e.sum(), rtol=1e-14)
    assert np.allclose(out["h1"], np.maximum(P[OFF["b1"]], 0.0))


def test_single_path_routes_through_weight_layout():
    """W[in][out] layout: feature k0 -> hidden 0 -> hidden 0 -> logit 5."""
    P = np.zeros(oracle.mlp_param_count())
    k0 = 32 * 1 + 1                       # cos of scalar 1 (y position) at l = 0
    W1 = P[OFF["W1"]].reshape(320, 64)
    W2 = P[OFF["W2"]].reshape(64, 64)
    W3 = P[OFF["W3"]].reshape(64, 256)
    W1[k0, 0], W2[0, 0], W3[0, 5] = 2.0, 3.0, 0.5
    f = oracle.pe_features(np.array([0.3, 0.0, 0.1]), np.array([0, 0, 1.0]),
                           np.array([0, 1.0, 0]), 0.5, np.full(3, -1.0), np.full(3, 1.0))
    assert f[k0] == 1.0
    out = oracle.mlp_forward(P, f, emulate_bf16=False)
    assert out["z3"][5] == 3.0 and np.count_nonzero(out["z3"]) == 1
    assert abs(out["q"][5] - math.exp(3) / (255 + math.exp(3))) < 1e-15


def random_batch(B=6, seed=2):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-1, 1, (B, 3))
    n = rng.standard_normal((B, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    v = rng.standard_normal((B, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return pos, n, v, rng.uniform(0.05, 1, B), rng.uniform(0, 1, (B, 256)) ** 3


def test_gradient_matches_central_differences():
    """FP64 network without rounding: analytic gradient vs central differences."""
    P = scenes.mlp_init(seed=1, gain=0.7).astype(np.float64)
    P[OFF["b1"]] = 0.05
    P[OFF["b2"]] = 0.05
    pos, n, v, r, T = random_batch()
    args = (pos, n, v, r, -np.ones(3), np.ones(3), T)
    loss, g = oracle.mlp_loss_grad(P, *args, emulate_bf16=False)
    rng = np.random.default_rng(5)
    picks = np.concatenate([rng.choice(np.arange(s.start, s.stop), 12, replace=False)
                            for s in OFF.values()])
    for i in picks:
        h = 1e-6 * max(1.0, abs(P[i]))
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (oracle.mlp_loss_grad(Pp, *args, emulate_bf16=False)[0] -
              oracle.mlp_loss_grad(Pm, *args, emulate_bf16=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_rounded_gradient_stays_close():
    P = scenes.mlp_init(seed=1).astype(np.float64)
    pos, n, v, r, T = random_batch(B=32)
    args = (pos, n, v, r, -np.ones(3), np.ones(3), T)
    _, g0 = oracle.mlp_loss_grad(P, *args, emulate_bf16=False)
    _, g1 = oracle.mlp_loss_grad(P, *args, emulate_bf16=True)
    assert np.linalg.norm(g1 - g0) < 0.1 * np.linalg.norm(g0)     # BF16 operands: ~2^-9 each


def test_adam_closed_form_two_steps():
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, -1.0, 0.25, 3.0])
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    oracle.adam(p, m, v, g, lr, b1, b2, eps, 1)
    assert np.allclose(p, p0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    oracle.adam(p, m, v, g, lr, b1, b2, eps, 2)
    assert np.allclose(p, p0 - 2 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------- sampler
def test_bin_masses_special_cases():
    c, tot = oracle.prop_masses(np.full(256, 0.37, np.float32), 1.0)
    assert tot == 1 << 24 and np.all(c == 65536)
    p = np.zeros(256, np.float32)
    p[7] = 1.0
    c, tot = oracle.prop_masses(p, 0.0)
    assert tot == 1 << 24 and c[7] == 1 << 24 and c.sum() == c[7]
    c, tot = oracle.prop_masses(np.full(256, np.nan, np.float32), 0.0)
    assert tot == 256 and np.all(c == 1)               # nothing to sample: one unit per bin
    probs = scenes.bin_probs(4)
    for row in probs:
        c, tot = oracle.prop_masses(row, 0.1)
        approx = (0.9 * row.astype(np.float64) + 0.1 / 256) * 2 ** 24
        assert np.all(np.abs(c - approx) <= 1.0) and tot == c.sum()


@pytest.mark.parametrize("w,b", [((0, 0, 1), 8 * 16 + 8), ((1, 0, 0), 255), ((0, 1, 0), 15),
                                 ((-1, 0, 0), 0), ((0, -1, 0), 240)])
def test_bin_of_axis_directions(w, b):
    got, uv = oracle.prop_bin(np.array(w, np.float64))
    assert got == b


def decode_uv(u, v):
    px, py = 0.5 * (u + v), 0.5 * (u - v)
    z = 1.0 - np.abs(px) - np.abs(py)
    w = np.stack([px, py, z], -1)
    return w / np.linalg.norm(w, axis=-1, keepdims=True)


@pytest.mark.parametrize("b", [8 * 16 + 8, 0, 15, 3 * 16 + 12])
def test_bin_density_integrates_to_one_with_numerical_jacobian(b):
    """One-hot proposal on bin b: its density times the numerically differentiated area
    element of the (u,v) -> direction map integrates to 1 over the bin."""
    p = np.zeros(256, np.float32)
    p[b] = 1.0
    n = 48
    bu, bv = b % 16, b // 16
    uu = -1 + (bu + (np.arange(n) + 0.5) / n) / 8
    vv = -1 + (bv + (np.arange(n) + 0.5) / n) / 8
    U, V = np.meshgrid(uu, vv, indexing="ij")
    h = 1e-7
    du = (decode_uv(U + h, V) - decode_uv(U - h, V)) / (2 * h)
    dv = (decode_uv(U, V + h) - decode_uv(U, V - h)) / (2 * h)
    J = np.linalg.norm(np.cross(du, dv), axis=-1)
    W = decode_uv(U, V)
    pdf = np.array([oracle.prop_pdf(p, 0.0, w) for w in W.reshape(-1, 3)]).reshape(n, n)
    total = np.sum(pdf * J) * (1 / (8 * n)) ** 2
    assert abs(total - 1.0) < 2e-4


def test_uniform_density_integrates_to_one_in_spherical_coordinates():
    p = np.full(256, 1.0 / 256, np.float32)
    nt, nf = 180, 360
    th = (np.arange(nt) + 0.5) * (np.pi / 2) / nt
    ph = (np.arange(nf) + 0.5) * 2 * np.pi / nf
    T, F = np.meshgrid(th, ph, indexing="ij")
    W = np.stack([np.sin(T) * np.cos(F), np.sin(T) * np.sin(F), np.cos(T)], -1).reshape(-1, 3)
    pdf = np.array([oracle.prop_pdf(p, 0.1, w) for w in W]).reshape(nt, nf)
    total = np.sum(pdf * np.sin(T)) * (np.pi / 2 / nt) * (2 * np.pi / nf)
    assert abs(total - 1.0) < 1e-4


def test_draws_are_stratified_and_consistent():
    probs = scenes.bin_probs(3, seed=4)
    S = 1000
    for i, row in enumerate(probs):
        c, tot = oracle.prop_masses(row, 0.1)
        bins, wl, pdf = oracle.prop_samples(row, 0.1, S, 99, i)
        counts = np.bincount(bins, minlength=256)
        # one draw per slice of the mass line: at most the two partly covered end slices
        # of a bin's interval differ from its expected count
        assert np.all(np.abs(counts - S * c / tot) < 2.0)
        assert np.mean(np.abs(counts - S * c / tot)) < 0.6
        for j in range(0, S, 37):
            assert abs(np.linalg.norm(wl[j]) - 1.0) < 1e-14 and wl[j, 2] > 0
            assert oracle.prop_bin(wl[j])[0] == bins[j]
            assert abs(oracle.prop_pdf(row, 0.1, wl[j]) - pdf[j]) <= 1e-12 * pdf[j]


@pytest.fixture(scope="module")
def small_scene():
    sc = scenes.tiny_shade(n_points=48)
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, sc.k)
    return sc, idx, w


def test_proposal_estimate_is_unbiased(small_scene):
    """Mean over seeds of the proposal estimate = the fixed-direction estimate at S=4096."""
    sc, idx, w = small_scene
    # rough surfaces only: a lobe of roughness 0.05 (alpha^2 ~ 6e-6) is far too narrow for
    # any of these sample counts, so neither estimate would have converged
    rough = np.linspace(0.4, 1.0, sc.n).astype(np.float32)
    ref = oracle.shade(sc, idx, w, n_dirs=4096, rough=rough)
    probs = scenes.bin_probs(sc.n, concentration=0.5, seed=7)
    est = np.stack([oracle.prop_shade(sc, idx, w, probs, 0.1, 64, seed, rough=rough)
                    for seed in range(48)])
    mean, se = est.mean(0), est.std(0, ddof=1) / np.sqrt(est.shape[0])
    z = (mean - ref) / np.sqrt(se ** 2 + (2e-3 * np.abs(ref)) ** 2)
    assert np.max(np.abs(z)) < 5.0
    assert np.mean(np.abs(z)) < 1.2


def test_uniform_bins_irradiance_of_constant_environment(small_scene):
    """Constant environment, no occlusion, no probe light: E = pi L in expectation."""
    sc, idx, w = small_scene
    env = np.full_like(sc.env, 2.0)
    tex = np.zeros(sc.texels.shape)
    probs = np.full((sc.n, 256), 1.0 / 256, np.float32)
    est = np.stack([oracle.prop_shade(sc, idx, w, probs, 0.0, 256, seed, texels=tex, env=env,
                                      irradiance=True)[1] for seed in range(8)])
    assert abs(est.mean() / (2.0 * np.pi) - 1.0) < 3e-3


def test_training_targets_sum_to_the_shading_luminance(small_scene):
    sc, idx, w = small_scene
    rough = np.linspace(0.4, 1.0, sc.n).astype(np.float32)     # lobes both estimates resolve
    T = oracle.dump_integrand(sc, idx, w, 16, 11, rough=rough)
    assert T.shape == (sc.n, 256) and np.all(T >= 0)
    ref = oracle.shade(sc, idx, w, n_dirs=4096, rough=rough)
    lum = ref @ np.array([0.2126, 0.7152, 0.0722])
    ratio = T.sum(1) / lum
    assert abs(ratio.mean() - 1.0) < 0.01 and np.max(np.abs(ratio - 1.0)) < 0.08
    zero = oracle.dump_integrand(sc, idx, w, 2, 11, env=np.zeros_like(sc.env),
                                 texels=np.zeros(sc.texels.shape))
    assert np.all(zero == 0.0)


def test_gradient_mass_bounds_the_gradient():
    """The sum of |terms| of each gradient entry: never below |gradient| (triangle
    inequality, so a sign slip in the chain fails), and for the output biases it sums to
    exactly 2 over the bins (sum over points of sum_b (q_b + t_b) / B, both rows normalised)."""
    P = scenes.mlp_init(seed=1).astype(np.float64)
    P[OFF["b1"]] = 0.05
    pos, n, v, r, T = random_batch(B=48)
    T[5] = 0.0                                   # an empty row counts as uniform
    args = (pos, n, v, r, -np.ones(3), np.ones(3), T)
    for emu in (False, True):
        loss, g, m = oracle.mlp_loss_grad(P, *args, emulate_bf16=emu, mass=True)
        _, g2 = oracle.mlp_loss_grad(P, *args, emulate_bf16=emu)
        assert np.array_equal(g, g2)
        if not emu:
            assert np.all(m >= np.abs(g) * (1 - 1e-12))
        assert m[OFF["b3"]].sum() == pytest.approx(2.0, rel=1e-12)
        assert np.all(m >= 0)
    # first-layer units all off: no mass reaches the first layer or the weights after it
    P0 = P.copy()
    P0[OFF["b1"]] = -100.0
    _, g0, m0 = oracle.mlp_loss_grad(P0, *args, emulate_bf16=False, mass=True)
    for name in ("W1", "b1", "W2"):
        assert np.all(m0[OFF[name]] == 0) and np.all(g0[OFF[name]] == 0)
