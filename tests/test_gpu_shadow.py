"""GPU parity of the cast-shadow ratio (Eq. 15-17) with the Hammersley set and with
environment importance sampling (Eq. 18) against the oracle. Texel choices of the
importance sampler are integer decisions taken identically on both sides."""
import numpy as np
import pytest

import oracle
from paper_2510_07729_amd import scenes
from tests.gpu_util import TOL, dev, log, parity_err, report

pytestmark = pytest.mark.gpu

F32 = np.float32


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


def small_scene(n_points=333, seed=0, **kw):
    args = dict(n_points=n_points, n_probes=48, res=8, env_res=16, n_dirs=64, k=4, seed=seed)
    args.update(kw)
    return scenes.shadow_scene(**args)


def gpu_shadow(sc, sampler, texels=None, env=None, per_point=False, k=None, half=False,
               use_nb=False):
    from paper_2510_07729_amd import sop
    plan = sop.Plan(dev(sc.probe_pos), sc.bounds_lo, sc.bounds_hi)
    tex = sc.texels if texels is None else texels
    tex_t = dev(tex.astype(np.float16) if half else tex)
    pts = sop.Points(dev(sc.pos), dev(sc.normal), None, None, None)
    kk = sc.k if k is None else k
    nb = sop.sop_knn(plan, sop.Points(dev(sc.pos), dev(sc.normal), None, None, None), kk) \
        if use_nb else None
    ratio, irr = sop.sop_shadow_ratio(plan, tex_t, dev(sc.env if env is None else env), pts,
                                      sc.n_dirs, k=kk, nb=nb, seed=sc.seed,
                                      rotate_per_point=per_point, sampler=sampler,
                                      irradiance=True)
    return ratio.cpu().numpy(), irr.cpu().numpy()


def ref_shadow(sc, sampler, texels=None, env=None, per_point=False, k=None):
    kk = sc.k if k is None else k
    idx, w = oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal, kk)
    tex = sc.texels if texels is None else texels
    return oracle.shadow_ratio(sc.normal, tex.astype(np.float64), idx, w,
                               sc.env if env is None else env, sc.n_dirs, seed=sc.seed,
                               per_point=per_point, sampler=sampler)


def compare(label, got, ref):
    e = report(f"{label} ratio", parity_err(got[0], ref["ratio"]))
    return max(e, report(f"{label} irradiance", parity_err(got[1], ref["irr"])))


@pytest.mark.parametrize("sampler", [0, 1, 2])
def test_shadow_small_scene(torch_gpu, sampler):
    log(f"shadow: 48 probes 8x8, 333 ground points, 16x16 sky, S=64, K=4, sampler {sampler}")
    sc = small_scene()
    assert compare(f"small s{sampler}", gpu_shadow(sc, sampler), ref_shadow(sc, sampler)) <= TOL


@pytest.mark.parametrize("S", [16, 32])
@pytest.mark.parametrize("sampler", [0, 1, 2])
def test_shadow_lane_groups(torch_gpu, S, sampler):
    """S <= 32 runs 64/S-ish points per wavefront (16 or 32 lanes each); 333 points leave a
    ragged last wavefront."""
    log(f"shadow: 333 points, S={S} (lane groups), sampler {sampler}")
    sc = small_scene(n_dirs=S, seed=8)
    assert compare(f"S={S} s{sampler}", gpu_shadow(sc, sampler), ref_shadow(sc, sampler)) <= TOL


def test_shadow_rotation_per_point_runtime_k_and_half_maps(torch_gpu):
    log("shadow: per-point rotation; K=3 (run-time K); f16 maps; given neighbour lists")
    sc = small_scene(n_points=200, seed=3)
    assert compare("per point", gpu_shadow(sc, 0, per_point=True),
                   ref_shadow(sc, 0, per_point=True)) <= TOL
    assert compare("K=3", gpu_shadow(sc, 1, k=3), ref_shadow(sc, 1, k=3)) <= TOL
    half = sc.texels.astype(np.float16)
    assert compare("f16", gpu_shadow(sc, 1, half=True),
                   ref_shadow(sc, 1, texels=half.astype(F32))) <= TOL
    a = gpu_shadow(sc, 1)
    b = gpu_shadow(sc, 1, use_nb=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_shadow_edge_cases(torch_gpu):
    from paper_2510_07729_amd import sop
    log("shadow: black sky, S=1, 2x2 sky, no points")
    sc = small_scene(n_points=40, seed=5)
    black = np.zeros_like(sc.env)
    for sampler in (0, 1, 2):
        r, irr = gpu_shadow(sc, sampler, env=black)
        assert np.all(r == 1.0) and np.all(irr == 0.0)
    for sampler in (0, 1):
        sc1 = scenes.shadow_scene(n_points=37, n_probes=48, res=8, env_res=2, n_dirs=1, k=4,
                                  seed=6)
        assert compare(f"S=1 2x2 s{sampler}", gpu_shadow(sc1, sampler),
                       ref_shadow(sc1, sampler)) <= TOL
    empty = sc.subset(np.arange(0))
    plan = sop.Plan(dev(sc.probe_pos), sc.bounds_lo, sc.bounds_hi)
    pts = sop.Points(dev(empty.pos), dev(empty.normal), None, None, None)
    r = sop.sop_shadow_ratio(plan, dev(sc.texels), dev(sc.env), pts, 16, k=4, sampler=1)
    assert r.shape == (0, 3)


@pytest.mark.parametrize("sampler", [0, 1, 2])
def test_shadow_full_size_sampled(torch_gpu, sampler):
    """The full workload in one launch (500k ground points, 2048 probes of 32x32, 256x256
    sky, S=64, K=8) as the benchmark runs it; 64 sampled points on the oracle."""
    log(f"shadow: 500k points, 2048 probes 32x32, 256x256 sky, S=64, K=8, sampler {sampler}")
    sc = scenes.shadow_scene()
    r, irr = gpu_shadow(sc, sampler)
    assert np.all(np.isfinite(r)) and np.all(np.isfinite(irr))
    rows = np.sort(np.random.default_rng(7).choice(sc.n, 64, replace=False))
    # the importance draws are keyed by the point index: the oracle gets the same indices
    sub = sc.subset(rows)
    idx, w = oracle.knn(sub.probe_pos, sub.bounds_lo, sub.bounds_hi, sub.pos, sub.normal, sc.k)
    ref = oracle.shadow_ratio(sub.normal, sc.texels.astype(np.float64), idx, w, sc.env,
                              sc.n_dirs, seed=sc.seed, sampler=sampler, ids=rows)
    assert compare(f"full s{sampler}", (r[rows], irr[rows]), ref) <= TOL
