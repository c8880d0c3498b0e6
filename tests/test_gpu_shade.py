"""GPU parity of the neighbour search, the Eq. 9 query and the shading forward pass against
the CPU oracle, called through the C ABI (libsop.so)."""
import math

import numpy as np
import pytest

import oracle
from paper_2510_07729_amd import scenes
from tests.gpu_util import (TOL, dev, gpu_plan, gpu_points, log, oracle_knn, parity_err,
                            report, subset_frames)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def sop():
    from paper_2510_07729_amd import sop as s
    return s


# ------------------------------------------------------------------------------------------
# neighbour search: indices bit-exact
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("k,radius", [(4, math.inf), (1, math.inf), (3, math.inf),
                                      (8, math.inf), (16, math.inf), (4, 0.3), (8, 0.05)])
def test_knn_tiny_bit_exact(torch_gpu, k, radius):
    log(f"knn tiny k={k} radius={radius}")
    sc = scenes.tiny_shade()
    plan = gpu_plan(sc)
    nb = sop().sop_knn(plan, gpu_points(sc), k, radius)
    torch_gpu.cuda.synchronize()
    idx_o, w_o = oracle_knn(sc, k, radius)
    idx_g = nb.idx.cpu().numpy()
    assert np.array_equal(idx_g, idx_o)
    w_g = nb.w.cpu().numpy()
    assert np.max(np.abs(w_g - w_o)) < 1e-6
    order = np.sort(nb.order.cpu().numpy())
    assert np.array_equal(order, np.arange(sc.n))


def test_knn_object_scene_bit_exact(torch_gpu):
    log("knn object scene 200k points, 4096 probes, k=8")
    sc = scenes.object_scene()
    plan = gpu_plan(sc)
    nb = sop().sop_knn(plan, gpu_points(sc), 8)
    torch_gpu.cuda.synchronize()
    idx_o, w_o = oracle_knn(sc, 8)
    assert np.array_equal(nb.idx.cpu().numpy(), idx_o)
    assert np.max(np.abs(nb.w.cpu().numpy() - w_o)) < 1e-5


def test_knn_frames_bit_exact(torch_gpu):
    log("knn g-buffer frames subset (16384 probes, k=8)")
    sc = scenes.gbuffer_frames(rows=np.arange(0, 1080, 90))
    plan = gpu_plan(sc)
    nb = sop().sop_knn(plan, gpu_points(sc), 8)
    torch_gpu.cuda.synchronize()
    idx_o, _ = oracle_knn(sc, 8)
    assert np.array_equal(nb.idx.cpu().numpy(), idx_o)


def test_knn_exact_hit_and_empty_plan(torch_gpu):
    log("knn exact hit / empty probe set")
    sc = scenes.tiny_shade(n_points=64)
    s2 = sc.subset(np.arange(64))
    s2.pos = sc.probe_pos.copy()
    s2.normal = sc.probe_pos.copy()
    plan = gpu_plan(s2)
    nb = sop().sop_knn(plan, gpu_points(s2), 4)
    idx = nb.idx.cpu().numpy()
    assert np.array_equal(idx[:, 0], np.arange(64)) and np.all(idx[:, 1:] == -1)
    assert np.all(nb.w.cpu().numpy()[:, 0] == 1.0)
    s3 = s2.subset(np.arange(64))
    s3.probe_pos = np.zeros((0, 3), np.float32)
    s3.texels = np.zeros((0, 16, 16, 4), np.float32)
    plan0 = sop().Plan(dev(np.zeros((1, 3), np.float32))[:0], s3.bounds_lo, s3.bounds_hi)
    nb0 = sop().sop_knn(plan0, gpu_points(s3), 4)
    assert np.all(nb0.idx.cpu().numpy() == -1) and np.all(nb0.w.cpu().numpy() == 0)


# ------------------------------------------------------------------------------------------
# Eq. 9 query
# ------------------------------------------------------------------------------------------
def test_query_matches_oracle(torch_gpu):
    log("query tiny D=7")
    sc = scenes.tiny_shade(n_points=1000)
    rng = np.random.default_rng(3)
    dirs = rng.standard_normal((sc.n, 7, 3))
    dirs /= np.linalg.norm(dirs, axis=-1, keepdims=True)
    dirs = dirs.astype(np.float32)
    plan = gpu_plan(sc)
    pts = gpu_points(sc)
    Lin, O = sop().sop_query(plan, dev(sc.texels), pts, dev(dirs), k=4)
    idx, w = oracle_knn(sc, 4)
    Lo, Oo = oracle.query(sc.texels.astype(np.float64), idx, w, dirs.astype(np.float64))
    assert report("query Lin", parity_err(Lin.cpu().numpy(), Lo)) <= TOL
    assert report("query O", parity_err(O.cpu().numpy(), Oo)) <= TOL


# ------------------------------------------------------------------------------------------
# shading forward
# ------------------------------------------------------------------------------------------
def run_shade(sc, n_dirs=None, k=None, per_point=False, irradiance=False, seed=None):
    s = sop()
    plan = gpu_plan(sc)
    out = s.sop_shade(plan, dev(sc.texels), dev(sc.env), gpu_points(sc),
                      sc.n_dirs if n_dirs is None else n_dirs, k=sc.k if k is None else k,
                      seed=sc.seed if seed is None else seed, rotate_per_point=per_point,
                      irradiance=irradiance)
    if irradiance:
        return out[0].cpu().numpy(), out[1].cpu().numpy()
    return out.cpu().numpy()


def test_shade_tiny_full_parity(torch_gpu):
    log("shade tiny (4096 points, S=64, K=4) + irradiance")
    sc = scenes.tiny_shade()
    rgb, irr = run_shade(sc, irradiance=True)
    idx, w = oracle_knn(sc)
    ro, io = oracle.shade(sc, idx, w, irradiance=True)
    assert report("shade tiny rgb", parity_err(rgb, ro)) <= TOL
    assert report("shade tiny irradiance", parity_err(irr, io)) <= TOL


@pytest.mark.parametrize("n_dirs,k,per_point,n", [(1, 4, False, 257), (5, 3, False, 1001),
                                                   (100, 8, True, 999), (128, 16, False, 512),
                                                   (64, 1, True, 64), (200, 2, False, 130),
                                                   (32, 4, True, 1003), (16, 8, False, 77),
                                                   (17, 5, False, 3)])
def test_shade_variants(torch_gpu, n_dirs, k, per_point, n):
    log(f"shade variant S={n_dirs} K={k} per_point={per_point} N={n}")
    sc = scenes.tiny_shade(n_points=n, seed=5)
    rgb = run_shade(sc, n_dirs=n_dirs, k=k, per_point=per_point)
    idx, w = oracle_knn(sc, k)
    ro = oracle.shade(sc, idx, w, n_dirs=n_dirs, per_point=per_point)
    assert report(f"shade S={n_dirs} K={k}", parity_err(rgb, ro)) <= TOL


def test_shade_is_deterministic(torch_gpu):
    log("shade repeat bitwise")
    sc = scenes.tiny_shade()
    a = run_shade(sc)
    b = run_shade(sc)
    assert np.array_equal(a, b)


def test_shade_constant_sky_irradiance_is_pi_L(torch_gpu):
    log("shade constant sky")
    sc = scenes.tiny_shade()
    sc.texels = np.zeros_like(sc.texels)
    sc.env = np.full_like(sc.env, 1.5)
    _, irr = run_shade(sc, irradiance=True)
    assert np.max(np.abs(irr / (np.pi * 1.5) - 1.0)) < 2e-6


def test_shade_object_scene_sampled(torch_gpu):
    log("shade object scene: 200k points on GPU, 3000 sampled on the oracle (S=128, K=8)")
    sc = scenes.object_scene()
    rgb = run_shade(sc)
    rows = np.random.default_rng(11).choice(sc.n, 3000, replace=False)
    sub = sc.subset(rows)
    idx, w = oracle_knn(sub)
    ro = oracle.shade(sub, idx, w)
    err = parity_err(rgb[rows], ro)
    assert report("shade object sampled", err) <= TOL


def test_shade_frames_half_texels_camera_views(torch_gpu):
    log("shade g-buffer frames: f16 textures, camera views, 8 frames x 1920 x 12 rows")
    sc = scenes.gbuffer_frames(rows=np.arange(0, 1080, 90))
    rgb = run_shade(sc)
    sub, rows = subset_frames(sc, 250)
    idx, w = oracle_knn(sub)
    ro = oracle.shade(sub, idx, w)
    assert report("shade frames sampled", parity_err(rgb[rows], ro)) <= TOL


def test_shade_frames_full_size_sampled(torch_gpu):
    # the G-buffer configuration at its full size (8 frames x 1920 x 1080 = 16.6M points,
    # 16,384 probes with f16 maps, 64 directions, K = 8) in one call; 40 pixels per frame
    # checked against the oracle
    log("shade g-buffer frames at full size: 16.6M points, 16384 f16 probes, S=64, K=8")
    sc = scenes.gbuffer_frames()
    rgb = run_shade(sc)
    assert rgb.shape == (sc.n, 3) and np.all(np.isfinite(rgb))
    sub, rows = subset_frames(sc, 40, seed=3)
    idx, w = oracle_knn(sub)
    ro = oracle.shade(sub, idx, w)
    assert report("shade frames full size sampled", parity_err(rgb[rows], ro)) <= TOL


def test_shade_empty_and_no_probes(torch_gpu):
    log("shade N=0 and P=0")
    s = sop()
    sc = scenes.tiny_shade(n_points=100)
    plan = gpu_plan(sc)
    e = sc.subset(np.arange(0))
    out = s.sop_shade(plan, dev(sc.texels), dev(sc.env), gpu_points(e), 64, k=4)
    assert out.shape == (0, 3)
    plan0 = s.Plan(dev(np.zeros((1, 3), np.float32))[:0], sc.bounds_lo, sc.bounds_hi)
    rgb = s.sop_shade(plan0, dev(sc.texels[:0]), dev(sc.env), gpu_points(sc), 64, k=4)
    idx = -np.ones((sc.n, 4), np.int32)
    w = np.zeros((sc.n, 4))
    ro = oracle.shade(sc, idx, w, texels=np.zeros((1, 16, 16, 4)))
    assert report("shade P=0", parity_err(rgb.cpu().numpy(), ro)) <= TOL


def test_shade_with_precomputed_neighbors(torch_gpu):
    log("shade with sop_knn neighbours passed in")
    s = sop()
    sc = scenes.tiny_shade(n_points=2000, seed=2)
    plan = gpu_plan(sc)
    pts = gpu_points(sc)
    nb = s.sop_knn(plan, pts, 4)
    a = s.sop_shade(plan, dev(sc.texels), dev(sc.env), pts, 64, nb=nb).cpu().numpy()
    b = s.sop_shade(plan, dev(sc.texels), dev(sc.env), pts, 64, k=4).cpu().numpy()
    assert np.array_equal(a, b)


def test_shade_reference_direction_count(torch_gpu):
    """The 4096-direction Hammersley estimate that judges the proposal's error, on the
    proposal workload's geometry: 1000 points against the oracle."""
    log("shade at S=4096 (the reference estimate) on 1000 points")
    sc = scenes.proposal_eval(n_points=1000, seed=0)
    rgb = run_shade(sc, n_dirs=4096, seed=123)
    idx, w = oracle_knn(sc)
    ro = oracle.shade(sc, idx, w, n_dirs=4096, seed=123)
    assert report("shade S=4096", parity_err(rgb, ro)) <= TOL


@pytest.mark.parametrize("hw", [(1, 2), (2, 3), (3, 5), (5, 7)])
def test_shade_small_equirect_environments(torch_gpu, hw):
    """Equirectangular skies whose texels span more than a right angle (W < 8 or H < 4):
    the lookup's FP64 fraction then comes from the full arctangent, not the small-angle
    series."""
    import dataclasses
    from paper_2510_07729_amd import sop
    log(f"forward with a {hw[0]}x{hw[1]} equirectangular sky")
    sc = scenes.tiny_shade(n_points=400, seed=44)
    sky = np.random.default_rng(45).lognormal(0.0, 0.7, (*hw, 3)).astype(np.float32)
    sc = dataclasses.replace(sc, env=sky)
    rgb, irr = sop.sop_shade(gpu_plan(sc), dev(sc.texels), dev(sky), gpu_points(sc),
                             sc.n_dirs, k=sc.k, seed=sc.seed, irradiance=True)
    idx, w = oracle_knn(sc)
    ref, rirr = oracle.shade(sc, idx, w, irradiance=True)
    assert report(f"sky {hw} rgb", parity_err(rgb.cpu().numpy(), ref)) <= TOL
    assert report(f"sky {hw} irradiance", parity_err(irr.cpu().numpy(), rirr)) <= TOL
