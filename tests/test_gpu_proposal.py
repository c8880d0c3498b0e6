"""GPU parity of the learned direction proposal against the oracle, through the C ABI:
network inference (BF16 matrix cores, FP32 accumulation) against the oracle's network that
rounds the same operands to bfloat16, the training step's loss and gradient, Adam, the
proposal-sampled shading (bin choices are exact integer decisions on both sides) and the
training-target dump."""
import numpy as np
import pytest

import oracle
from paper_2510_07729_amd import scenes
from tests.gpu_util import (TOL, dev, gpu_plan, gpu_points, log, oracle_knn, parity_err,
                            report, sum_err)

pytestmark = pytest.mark.gpu

OFF = oracle.mlp_offsets()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def sop():
    from paper_2510_07729_amd import sop as s
    return s


def eval_scene(n, seed=0):
    return scenes.proposal_eval(n_points=n, seed=seed)


def gpu_mlp(params, sc):
    return sop().Mlp(dev(params), sc.bounds_lo, sc.bounds_hi)


def logit_mass(params, sc, rows):
    """sum_k |h2_k W3_kb| + |b3_b| per logit (oracle activations): the scale of a logit's
    rounding error."""
    W3 = params[OFF["W3"]].astype(np.float64)
    W3r = np.abs(np.array([oracle.bf16(x) for x in W3])).reshape(64, 256)
    b3 = np.abs(params[OFF["b3"]].astype(np.float64))
    P64 = params.astype(np.float64)
    out = []
    for i in rows:
        f = oracle.pe_features(sc.pos[i], sc.normal[i], sc.view[i], sc.rough[i], sc.bounds_lo,
                               sc.bounds_hi)
        out.append(np.abs(oracle.mlp_forward(P64, f)["h2"]) @ W3r + b3)
    return np.array(out)


@pytest.mark.parametrize("n", [1000, 1, 17])
def test_infer_matches_bf16_oracle(torch_gpu, n):
    log(f"proposal inference: {n} points")
    sc = eval_scene(max(n, 1))
    params = scenes.mlp_init(seed=3)
    params[OFF["b1"]] = 0.1
    params[OFF["b3"]] = np.linspace(-1, 1, 256)
    mlp = gpu_mlp(params, sc)
    probs, logits = sop().sop_proposal_infer(mlp, gpu_points(sc), logits=True)
    torch_gpu.cuda.synchronize()
    lg, pg = logits.cpu().numpy(), probs.cpu().numpy()
    lo, po = oracle.mlp_infer(params.astype(np.float64), sc.pos, sc.normal, sc.view, sc.rough,
                              sc.bounds_lo, sc.bounds_hi, emulate_bf16=True)
    rows = np.arange(n)                      # every row
    mass = logit_mass(params, sc, rows)
    rel = np.abs(lg[rows] - lo[rows]) / mass
    log(f"logits ({n} rows): max |d|/mass {rel.max():.3e}  p99.9 "
        f"{np.percentile(rel, 99.9):.3e}; max |d| {np.abs(lg - lo).max():.3e}")
    # one bfloat16 step (2^-8 relative) of an operand moves a logit by far less than its
    # mass; FP32 vs FP64 accumulation adds ~1e-7 of it
    assert np.percentile(rel, 99.9) <= 2.0 ** -8 and rel.max() <= 2.0 ** -6
    dq = np.abs(pg - po)
    bound = 2.0 * po * np.abs(lg - lo).max(axis=1, keepdims=True) + 1e-7
    assert np.all(dq <= bound)
    assert np.allclose(pg.sum(1), 1.0, atol=1e-5)


def test_infer_empty(torch_gpu):
    sc = eval_scene(4)
    mlp = gpu_mlp(scenes.mlp_init(), sc)
    pts = gpu_points(sc)
    import dataclasses
    pts0 = dataclasses.replace(pts, pos=pts.pos[:0], normal=pts.normal[:0],
                               albedo=pts.albedo[:0], rough=pts.rough[:0], metal=pts.metal[:0],
                               view=pts.view[:0])
    out = sop().sop_proposal_infer(mlp, pts0)
    assert out.shape == (0, 256)


def batch(B, seed=2):
    sc = eval_scene(B, seed=seed)
    rng = np.random.default_rng(seed)
    T = (rng.uniform(0, 1, (B, 256)) ** 3).astype(np.float32)
    T[::7] = 0.0                                  # rows without signal count as uniform
    return sc, T


@pytest.mark.parametrize("B", [300, 4096])
def test_train_gradient_matches_oracle(torch_gpu, B):
    log(f"proposal training gradient: batch {B}")
    import torch
    sc, T = batch(B)
    params = scenes.mlp_init(seed=4)
    params[OFF["b1"]] = 0.05
    params[OFF["b2"]] = 0.05
    mlp = gpu_mlp(params, sc)
    grad = torch.empty(params.size, dtype=torch.float32, device="cuda")
    loss = sop().sop_proposal_train_step(mlp, gpu_points(sc), dev(T), grad=grad)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    lo, go, gm = oracle.mlp_loss_grad(params.astype(np.float64), sc.pos, sc.normal, sc.view,
                                      sc.rough, sc.bounds_lo, sc.bounds_hi, T,
                                      emulate_bf16=True, mass=True)
    lg = float(loss.item())
    log(f"loss gpu {lg:.7f} oracle {lo:.7f}")
    assert abs(lg - lo) <= 1e-4 * abs(lo)
    # element by element against the entry's sum of |terms|: both sides round the same
    # operands to bfloat16, so they differ by the accumulation order (~1e-7 of the mass)
    # and by the rare operand whose FP32 and FP64 values round to neighbouring bfloat16
    # numbers (a 2^-8 change of that one sample's terms)
    for name, sl in OFF.items():
        e = sum_err(g[sl], go[sl], gm[sl])
        l2 = np.linalg.norm(g[sl] - go[sl]) / np.linalg.norm(go[sl])
        log(f"grad {name}: max |d|/mass {e.max():.3e}  p99.9 {np.percentile(e, 99.9):.3e}  "
            f"(relative L2 {l2:.3e})")
        assert e.max() <= 2.0 ** -6, name
    # parameters untouched without an optimiser
    assert np.array_equal(mlp.params.cpu().numpy(), params)


def test_train_step_is_deterministic(torch_gpu):
    log("training steps repeat bit for bit (no atomics)")
    import torch
    sc, T = batch(4096, seed=3)
    params = scenes.mlp_init(seed=8)
    runs = []
    for _ in range(2):
        mlp = gpu_mlp(params, sc)
        grad = torch.empty(params.size, dtype=torch.float32, device="cuda")
        loss = sop().sop_proposal_train_step(mlp, gpu_points(sc), dev(T), grad=grad)
        g0, l0 = grad.clone(), loss.clone()
        for _ in range(3):                       # three Adam steps on the same batch
            sop().sop_proposal_train_step(mlp, gpu_points(sc), dev(T), lr=1e-3)
        torch.cuda.synchronize()
        runs.append((g0.cpu().numpy(), l0.cpu().numpy(), mlp.params.cpu().numpy()))
    for a_, b_ in zip(runs[0], runs[1]):
        assert np.array_equal(a_, b_)


def test_adam_matches_oracle(torch_gpu):
    log("Adam update")
    import torch
    rng = np.random.default_rng(9)
    n = 41344
    p = rng.standard_normal(n).astype(np.float32)
    m = (rng.standard_normal(n) * 1e-3).astype(np.float32)
    v = (rng.uniform(0, 1e-6, n)).astype(np.float32)
    g = (rng.standard_normal(n) * 1e-3).astype(np.float32)
    tp, tm, tv = dev(p), dev(m), dev(v)
    sop().sop_adam_update(tp, tm, tv, dev(g), 3e-3, 5)
    torch.cuda.synchronize()
    po, mo, vo = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    f32 = lambda x: float(np.float32(x))      # noqa: E731  (the C ABI takes float options)
    oracle.adam(po, mo, vo, g.astype(np.float64), f32(3e-3), f32(0.9), f32(0.999), f32(1e-8), 5)
    # m and v are two-term sums that can cancel: measure against the sum of |terms|
    m_mass = 0.9 * np.abs(m.astype(np.float64)) + 0.1 * np.abs(g.astype(np.float64))
    v_mass = v.astype(np.float64) + 0.001 * g.astype(np.float64) ** 2
    assert report("adam m", sum_err(tm.cpu().numpy(), mo, m_mass)) <= 1e-6
    assert report("adam v", sum_err(tv.cpu().numpy(), vo, v_mass)) <= 1e-6
    step_gpu = tp.cpu().numpy() - p
    step_orc = po - p
    assert np.max(np.abs(step_gpu - step_orc)) <= 1e-4 * 3e-3 + 1e-6


def test_train_step_moves_like_oracle(torch_gpu):
    log("one training step with Adam")
    import torch
    sc, T = batch(512, seed=5)
    params = scenes.mlp_init(seed=6)
    mlp = gpu_mlp(params, sc)
    sop().sop_proposal_train_step(mlp, gpu_points(sc), dev(T), lr=1e-3)
    torch.cuda.synchronize()
    _, go = oracle.mlp_loss_grad(params.astype(np.float64), sc.pos, sc.normal, sc.view,
                                 sc.rough, sc.bounds_lo, sc.bounds_hi, T, emulate_bf16=True)
    po = params.astype(np.float64)
    oracle.adam(po, np.zeros_like(po), np.zeros_like(po), go, 1e-3, 0.9, 0.999, 1e-8, 1)
    d_gpu = mlp.params.cpu().numpy() - params
    d_orc = po - params
    close = np.abs(d_gpu - d_orc) <= 0.05 * 1e-3
    log(f"first Adam step: {close.mean() * 100:.3f}% of parameters agree to 5% of lr")
    # step 1 of Adam is lr * g / (|g| + eps): only gradients within rounding of zero may
    # land on the other side
    assert close.mean() >= 0.995


# ------------------------------------------------------------------------------------------
# proposal-sampled shading and the training targets
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("S,eps,kind", [(32, 0.1, "dirichlet"), (100, 0.1, "dirichlet"),
                                        (64, 1.0, "dirichlet"), (16, 0.0, "onehot"),
                                        (8, 0.0, "nan")])
def test_proposal_shade_matches_oracle(torch_gpu, S, eps, kind):
    log(f"proposal shading S={S} eps={eps} probs={kind}")
    import torch
    sc = scenes.tiny_shade(n_points=509)          # not a multiple of the points per wavefront
    idx, w = oracle_knn(sc)
    if kind == "dirichlet":
        probs = scenes.bin_probs(sc.n, concentration=0.3, seed=S)
    elif kind == "onehot":
        probs = np.zeros((sc.n, 256), np.float32)
        probs[np.arange(sc.n), np.arange(sc.n) % 256] = 1.0
    else:
        probs = np.full((sc.n, 256), np.nan, np.float32)
    ref, ref_e = oracle.prop_shade(sc, idx, w, probs, eps, S, 77, irradiance=True)
    plan = gpu_plan(sc)
    rgb, irr = sop().sop_shade(plan, dev(sc.texels), dev(sc.env), gpu_points(sc), S, k=sc.k,
                               seed=77, irradiance=True, probs=dev(probs), mix_eps=eps)
    torch.cuda.synchronize()
    assert report("proposal rgb", parity_err(rgb.cpu().numpy(), ref)) <= TOL
    assert report("proposal irradiance", parity_err(irr.cpu().numpy(), ref_e)) <= TOL


def test_proposal_sampler_rejected_by_backward(torch_gpu):
    sc = scenes.tiny_shade(n_points=16)
    plan = gpu_plan(sc)
    probs = dev(scenes.bin_probs(sc.n))
    o = sop().shade_opts(16, 4, probs=probs)
    import ctypes as C
    from paper_2510_07729_amd import _lib as L
    m, e, cp = sop()._maps(dev(sc.texels)), sop()._env(dev(sc.env)), gpu_points(sc).c()
    st = plan._lib.sop_shade_backward(plan.handle, C.byref(m), C.byref(e), C.byref(cp), None,
                                      C.byref(o), 16, None, None, None, None, None, None, 0,
                                      None)
    assert st == L.SOP_ERR_UNSUPPORTED


@pytest.mark.parametrize("npb", [2, 3])
def test_dump_integrand_matches_oracle(torch_gpu, npb):
    log(f"integrand dump, {npb} draws per bin")
    import torch
    sc = scenes.tiny_shade(n_points=256)
    idx, w = oracle_knn(sc)
    ref = oracle.dump_integrand(sc, idx, w, npb, 13)
    plan = gpu_plan(sc)
    T = sop().sop_dump_integrand(plan, dev(sc.texels), dev(sc.env), gpu_points(sc), npb,
                                 k=sc.k, seed=13)
    torch.cuda.synchronize()
    assert report("bin targets", parity_err(T.cpu().numpy(), ref)) <= TOL


def test_proposal_object_scale_sampled(torch_gpu):
    """The benchmark's launch configuration: the network on 200k object points, proposal
    shading at S=32 with K=8 on all 200k; the first 1500 points (i.i.d., so a random sample
    that keeps the point indices the draws depend on) checked against the oracle, the
    network's logits on 256 of them."""
    log("proposal at object scale: 200k points, K=8, S=32; 1500 checked on the oracle")
    import torch
    sc = scenes.object_scene()
    params = scenes.mlp_init(seed=11)
    mlp = sop().Mlp(dev(params), sc.bounds_lo, sc.bounds_hi)
    pts = gpu_points(sc)
    plan = gpu_plan(sc)
    nb = sop().sop_knn(plan, pts, 8)
    _, logits = sop().sop_proposal_infer(mlp, pts, logits=True)
    probs = scenes.bin_probs(sc.n, concentration=0.3, seed=21)
    rgb = sop().sop_shade(plan, dev(sc.texels), dev(sc.env), pts, 32, nb=nb, seed=3,
                          probs=dev(probs), mix_eps=0.1)
    torch.cuda.synchronize()
    rows = np.arange(1500)
    sub = sc.subset(rows)
    idx, w = oracle_knn(sub, 8)
    ref = oracle.prop_shade(sub, idx, w, probs[rows], 0.1, 32, 3)
    assert report("object proposal rgb", parity_err(rgb.cpu().numpy()[rows], ref)) <= TOL
    r2 = rows[:256]
    lo, _ = oracle.mlp_infer(params.astype(np.float64), sc.pos[r2], sc.normal[r2],
                             sc.view[r2], sc.rough[r2], sc.bounds_lo, sc.bounds_hi)
    d = np.abs(logits.cpu().numpy()[r2] - lo)
    log(f"object logits: max |d| {d.max():.3e} (logit scale {np.abs(lo).max():.3e})")
    assert d.max() <= 2.0 ** -6 * max(1.0, np.abs(lo).max())


def test_trained_proposal_beats_fixed_directions(torch_gpu):
    """What the learned part gains: after online training on the tiny scene's geometry (the
    benchmark's recipe, about a second on the GPU), proposal sampling at 32 directions has a lower error than the paper's fixed
    Hammersley set at 32 directions and than uniform bins (the method without the network)."""
    log("proposal training gain: 3000 steps, 50k held-out points")
    import torch
    from paper_2510_07729_amd import proposal
    pool_sc = scenes.proposal_eval(262_144, seed=5)
    ev_sc = scenes.proposal_eval(50_000, seed=0)
    plan = gpu_plan(pool_sc)
    tex, env = dev(pool_sc.texels), dev(pool_sc.env)
    pool, ev = gpu_points(pool_sc), gpu_points(ev_sc)
    mlp = sop().Mlp(dev(scenes.mlp_init(seed=0)), pool_sc.bounds_lo, pool_sc.bounds_hi)
    losses = proposal.train(mlp, plan, tex, env, pool, 3000, batch=4096, lr=2e-3,
                            log_every=750)
    log(f"losses {losses}")
    assert losses[-1] < losses[0] - 0.3
    nb = sop().sop_knn(plan, ev, 4)
    ref = sop().sop_shade(plan, tex, env, ev, 4096, nb=nb, seed=123)
    mask = ev.rough >= 0.25

    def rmse(x):
        return float(torch.sqrt(torch.mean(((x - ref)[mask]) ** 2)))

    ham = rmse(sop().sop_shade(plan, tex, env, ev, 32, nb=nb, seed=7))
    probs = sop().sop_proposal_infer(mlp, ev)
    prop = rmse(sop().sop_shade(plan, tex, env, ev, 32, nb=nb, seed=7, probs=probs))
    uni = rmse(sop().sop_shade(plan, tex, env, ev, 32, nb=nb, seed=7,
                               probs=torch.full_like(probs, 1.0 / 256)))
    log(f"RMSE at 32 directions: Hammersley {ham:.4f}, uniform bins {uni:.4f}, "
        f"trained proposal {prop:.4f}")
    assert prop < 0.8 * ham and prop < 0.8 * uni


@pytest.mark.parametrize("n,k,S", [(509, 4, 32), (1000, 8, 7), (16, 4, 64), (1, 8, 3)])
def test_fused_network_sampler_matches_two_steps(torch_gpu, n, k, S):
    """The network evaluated inside the shading kernel gives the two-step result (inference,
    then shading with its probabilities) up to the order of the per-point sums."""
    log(f"fused proposal shading: N={n} K={k} S={S}")
    import torch
    sc = scenes.tiny_shade(n_points=n, seed=3)
    mlp = sop().Mlp(dev(scenes.mlp_init(seed=5)), sc.bounds_lo, sc.bounds_hi)
    pts = gpu_points(sc)
    plan = gpu_plan(sc)
    nb = sop().sop_knn(plan, pts, k)
    probs = sop().sop_proposal_infer(mlp, pts)
    tex, env = dev(sc.texels), dev(sc.env)
    two, two_e = sop().sop_shade(plan, tex, env, pts, S, nb=nb, seed=9, irradiance=True,
                                 probs=probs, mix_eps=0.1)
    one, one_e = sop().sop_shade(plan, tex, env, pts, S, nb=nb, seed=9, irradiance=True,
                                 net=mlp, mix_eps=0.1)
    torch.cuda.synchronize()
    assert report("fused vs two-step rgb", parity_err(one.cpu().numpy(), two.cpu().numpy())) <= 1e-5
    assert report("fused vs two-step irradiance",
                  parity_err(one_e.cpu().numpy(), two_e.cpu().numpy())) <= 1e-5


def exact_logit_network(n_active: int, seed: int):
    """A network whose logits both sides compute exactly: random first and second layers,
    W3 = 0 and b3 = 0 on n_active bins (a power of two) and -1000 elsewhere, so that the
    softmax is exactly 1/n_active on the active bins and 0 elsewhere in FP32 and FP64 alike
    (exp(0) = 1, exp(-1000) = 0). Every mass decision is then the same on both sides."""
    params = scenes.mlp_init(seed=seed)
    params[OFF["b1"]] = 0.1
    params[OFF["W3"]] = 0.0
    b3 = np.full(256, -1000.0, np.float32)
    b3[np.random.default_rng(seed).choice(256, n_active, replace=False)] = 0.0
    params[OFF["b3"]] = b3
    return params


@pytest.mark.parametrize("scene,n_active,S,k", [("tiny", 8, 32, 4), ("tiny", 256, 7, 4),
                                                ("tiny", 1, 16, 4), ("object", 64, 32, 8)])
def test_fused_network_sampler_matches_oracle(torch_gpu, scene, n_active, S, k):
    """The fused kernel (network on the matrix cores, softmax, masses, draws, shading in one
    launch) against the oracle's network followed by the oracle's proposal shading, element
    by element, for networks whose bin probabilities both compute exactly."""
    log(f"fused proposal shading vs oracle: {scene} scene, {n_active} active bins, S={S}, K={k}")
    import torch
    if scene == "tiny":
        sc = scenes.tiny_shade(n_points=509, seed=4)
    else:
        full = scenes.object_scene()
        sc = full.subset(np.arange(2000))
    params = exact_logit_network(n_active, seed=n_active + S)
    lo_, probs = oracle.mlp_infer(params.astype(np.float64), sc.pos, sc.normal, sc.view,
                                  sc.rough, sc.bounds_lo, sc.bounds_hi, emulate_bf16=True)
    assert np.all(np.isin(probs, (0.0, 1.0 / n_active)))
    idx, w = oracle_knn(sc, k)
    ref, ref_e = oracle.prop_shade(sc, idx, w, probs.astype(np.float32), 0.1, S, 19,
                                   irradiance=True)
    mlp = sop().Mlp(dev(params), sc.bounds_lo, sc.bounds_hi)
    plan = gpu_plan(sc)
    rgb, irr = sop().sop_shade(plan, dev(sc.texels), dev(sc.env), gpu_points(sc), S, k=k,
                               seed=19, irradiance=True, net=mlp, mix_eps=0.1)
    torch.cuda.synchronize()
    assert report("fused vs oracle rgb", parity_err(rgb.cpu().numpy(), ref)) <= TOL
    assert report("fused vs oracle irradiance", parity_err(irr.cpu().numpy(), ref_e)) <= TOL


def test_training_resumes_bit_for_bit_from_checkpoint(torch_gpu, tmp_path):
    """A training run stopped after 6 of 12 steps, saved, loaded into a fresh network and
    resumed ends with the same parameters, Adam moments and step count, bit for bit, as
    the run that was never interrupted."""
    from paper_2510_07729_amd import proposal
    sc = scenes.proposal_eval(16_384, seed=3)
    plan = gpu_plan(sc)
    tex, env, pool = dev(sc.texels), dev(sc.env), gpu_points(sc)
    init = scenes.mlp_init(seed=1)
    whole = sop().Mlp(dev(init), sc.bounds_lo, sc.bounds_hi)
    proposal.train(whole, plan, tex, env, pool, 12, batch=4096, lr=2e-3, seed=9)
    part = sop().Mlp(dev(init), sc.bounds_lo, sc.bounds_hi)
    proposal.train(part, plan, tex, env, pool, 12, batch=4096, lr=2e-3, seed=9, stop=6)
    path = str(tmp_path / "proposal.safetensors")
    part.save(path, iteration=6)
    resumed, meta = sop().Mlp.load(path, device="cuda")
    assert int(meta["iteration"]) == 6 and resumed.step == 6
    proposal.train(resumed, plan, tex, env, pool, 12, batch=4096, lr=2e-3, seed=9, start=6)
    torch_gpu.cuda.synchronize()
    assert resumed.step == whole.step == 12
    for a, b in ((resumed.params, whole.params), (resumed.m, whole.m), (resumed.v, whole.v)):
        assert torch_gpu.equal(a, b)
    assert not torch_gpu.equal(resumed.params, dev(init))
