"""Benchmark of the SOP hot path on one MI355X.

One step = one pass of the whole path over the object workload: rebuild the probe grid,
re-register the 100k Gaussians in the bake grid and bake 4096 probes at 32x32 (4.19M rays,
probes traced in the probe grid's Morton order), order the 200k shading points and find
their 8 nearest probes, shade them with 128 directions (forward) and run the adjoint
(backward) into the probe and environment gradients; then run the proposal network on the
200k points, shade them again with 32 directions drawn from its bin distributions, and take
one proposal training step (fresh bin targets for 4096 points + Adam). value = the metric's
shaded point-direction samples per second forward + backward, N*S / (t_fwd + t_bwd) with
S = 128 and the two kernels' times measured inside the step; the whole step's rate is
reported next to it. After the timed region: the G-buffer frames workload (16.6M points),
the learned proposal's speedup at matched error (as the workload states it and the online
variant), and the studies of the rows after the hot path.

Prints ONE JSON line. Per-kernel durations are measured with HIP events on the stream the
kernels run on; algorithmic flop counts per sample are documented below.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "shaded point·direction samples/s fwd+bwd; % HBM roofline; speedup at matched error"
PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector, published (packed FMA)
PEAK_HBM_GBS = 8000.0
S_PROP = 32            # proposal-sampled directions per point in the step
MIX_EPS = 0.1          # uniform-bin share of the proposal mixture
TRAIN_BATCH = 4096     # points per proposal training step


# Algorithmic FP32 operations per sample (+, -, *, / and each transcendental, sqrt, floor
# count 1; a fused multiply-add counts 2), counted from the definitions the kernels
# implement (direction, environment fetch, octahedral taps, K-probe blend, incident light,
# BRDF, accumulation). Per-point work (frame, material constants) is not counted.
def flops_fwd(K: int) -> int:
    direction, env, taps, light, brdf, acc = 24, 45, 25, 7, 69, 6
    return direction + env + taps + 36 * K + light + brdf + acc


def flops_bwd(K: int) -> int:
    recompute = flops_fwd(K) - 6
    material, texture, environment = 28 + 81, 20 * K, 12
    return recompute + material + texture + environment


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-proposal-study", action="store_true")
    ap.add_argument("--proposal-steps", type=int, default=6000)
    ap.add_argument("--no-trace-study", action="store_true")
    ap.add_argument("--no-shadow-study", action="store_true")
    ap.add_argument("--no-place-study", action="store_true")
    ap.add_argument("--no-env-study", action="store_true")
    ap.add_argument("--no-frames-study", action="store_true")
    ap.add_argument("--no-envis-study", action="store_true")
    ap.add_argument("--frames-only", action="store_true",
                    help="only the G-buffer frames forward (16.6M points, f16 maps, S=64, "
                         "K=8; 1 warm-up + 3 timed calls; for kernel traces of that path)")

    ap.add_argument("--place-only", action="store_true",
                    help="only probe placement and the losses of the object workload (for "
                         "kernel traces of that path)")
    ap.add_argument("--shadow-only", action="store_true",
                    help="only the cast-shadow ratio of the shadow workload with both samplers "
                         "(1 warm-up + 3 timed calls each; for kernel traces of that path)")
    ap.add_argument("--trace-only", action="store_true",
                    help="only traced shading of the object workload at 128 directions "
                         "(1 warm-up + 3 timed calls; for kernel traces of that path)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--peaks", action="store_true",
                    help="only the device-rate microbenchmarks (libsop_peaks.so): HBM copy, "
                         "FP32/FP64 FMA, float atomics, LDS and global gathers")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (it would "
              "shard the shading points by Morton range over replicated probes and "
              "environment, with one all-reduce of the environment and probe-texture "
              "gradients in the backward, and the bake by probe)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2510_07729_amd import _lib as L
    from paper_2510_07729_amd import proposal, scenes, sop

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.copy_calibration:
        return copy_calibration(torch, dev)
    if args.peaks:
        return peaks()
    if args.trace_only:
        return trace_only(torch, dev, sop, scenes)
    if args.shadow_only:
        return shadow_only(torch, dev, sop, scenes)
    if args.frames_only:
        print(json.dumps(frames_study(torch, dev, sop, scenes, reps=3, cpu=False)), flush=True)
        return 0

    if args.place_only:
        import numpy as np
        tex = torch.from_numpy(scenes.probe_textures(scenes.rng(scenes.CFG_OBJECT, 1, 0), 4096,
                                                     32)).to(dev)
        print(json.dumps(place_study(torch, sop, scenes, time_ms_plain, tex)), flush=True)
        return 0
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)   # noqa: E731

    # ------------------------------------------------------------------ workload (untimed)
    t0 = time.time()
    gs = scenes.object_gaussians()
    probes_np = scenes.object_probes()
    sc = scenes.object_scene()
    N, S, K, R = sc.n, sc.n_dirs, sc.k, 32
    P = probes_np.shape[0]
    G = gs.count
    grad_np = np.random.default_rng(123).standard_normal((N, 3)).astype(np.float32)
    print(f"# workload built in {time.time() - t0:.1f}s: G={G} P={P} R={R} N={N} S={S} K={K}",
          file=sys.stderr, flush=True)

    g_mean, g_scale, g_rot, g_op, g_col = (d(gs.mean), d(gs.scale), d(gs.rotation),
                                           d(gs.opacity), d(gs.color))
    probes = d(probes_np)
    env = d(sc.env)
    pts = sop.Points(d(sc.pos), d(sc.normal), d(sc.albedo), d(sc.rough), d(sc.metal),
                     view=d(sc.view))
    grad = d(grad_np)
    tex = torch.empty((P, R, R, 4), dtype=torch.float32, device=dev)
    dep = torch.empty((P, R, R), dtype=torch.float32, device=dev)
    rgb = torch.empty((N, 3), dtype=torch.float32, device=dev)
    g_env = torch.zeros(env.shape, dtype=torch.float32, device=dev)
    g_tex = torch.zeros(tex.shape, dtype=torch.float32, device=dev)

    bake_plan = sop.BakePlan(g_mean, g_scale, g_rot, g_op, g_col)
    plan = sop.Plan(probes, sc.bounds_lo, sc.bounds_hi)
    ws_f = sop.workspace(plan.workspace_size(sop.L.SOP_OP_SHADE, N, K, S, env.shape[:2], True), dev)
    ws_b = sop.workspace(plan.workspace_size(sop.L.SOP_OP_SHADE_BACKWARD, N, K, S, env.shape[:2],
                                             True), dev)

    # learned proposal on the same points: network inference, proposal-sampled shading at
    # S_PROP directions, and one training step (fresh bin targets for a batch + Adam)
    mlp_obj = proposal.default_mlp(dev, sc.bounds_lo, sc.bounds_hi, seed=0)
    probs = torch.empty((N, L.SOP_MLP_BINS), dtype=torch.float32, device=dev)
    rgb_p = torch.empty((N, 3), dtype=torch.float32, device=dev)
    ws_inf = sop.proposal_workspace(L.SOP_OP_PROPOSAL_INFER, N, dev)
    ws_pf = sop.workspace(plan.workspace_size(L.SOP_OP_SHADE, N, K, S_PROP, env.shape[:2], True),
                          dev)
    pts_tb = sop.Points(pts.pos[:TRAIN_BATCH], pts.normal[:TRAIN_BATCH], pts.albedo[:TRAIN_BATCH],
                        pts.rough[:TRAIN_BATCH], pts.metal[:TRAIN_BATCH],
                        view=pts.view[:TRAIN_BATCH])
    T_tb = torch.empty((TRAIN_BATCH, L.SOP_MLP_BINS), dtype=torch.float32, device=dev)
    loss_tb = torch.empty(1, dtype=torch.float32, device=dev)
    ws_dump = sop.workspace(plan.workspace_size(L.SOP_OP_DUMP_INTEGRAND, TRAIN_BATCH, K, 1,
                                                env.shape[:2]), dev)
    ws_tr = sop.proposal_workspace(L.SOP_OP_PROPOSAL_TRAIN, TRAIN_BATCH, dev)

    names = ["bake_grid", "bake", "probe_grid", "knn", "shade_fwd", "shade_bwd",
             "proposal_infer", "proposal_shade", "proposal_train"]
    ev = {n: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for n in names}
    acc = {n: 0.0 for n in names}

    it_count = [0]

    def step(timed: bool):
        it_count[0] += 1

        def mark(n, i):
            if timed:
                ev[n][i].record()
        mark("probe_grid", 0)
        plan.rebuild(probes)
        mark("probe_grid", 1)
        mark("bake_grid", 0)
        bake_plan.update(g_mean, g_scale, g_rot, g_op, g_col)
        mark("bake_grid", 1)
        mark("bake", 0)
        sop.sop_bake(bake_plan, probes, R, texels=tex, depth_out=dep, order_by=plan)
        mark("bake", 1)
        mark("knn", 0)
        nb = sop.sop_knn(plan, pts, K)
        mark("knn", 1)
        mark("shade_fwd", 0)
        sop.sop_shade(plan, tex, env, pts, S, nb=nb, ws=ws_f, out=rgb)
        mark("shade_fwd", 1)
        g_env.zero_()
        g_tex.zero_()
        mark("shade_bwd", 0)
        sop.sop_shade_backward(plan, tex, env, pts, grad, S, nb=nb, g_env=g_env, g_tex=g_tex,
                               ws=ws_b)
        mark("shade_bwd", 1)
        mark("proposal_infer", 0)
        sop.sop_proposal_infer(mlp_obj, pts, ws=ws_inf, out=probs)
        mark("proposal_infer", 1)
        mark("proposal_shade", 0)
        sop.sop_shade(plan, tex, env, pts, S_PROP, nb=nb, ws=ws_pf, out=rgb_p, probs=probs,
                      mix_eps=MIX_EPS)
        mark("proposal_shade", 1)
        mark("proposal_train", 0)
        sop.sop_dump_integrand(plan, tex, env, pts_tb, 1, k=K, seed=it_count[0], out=T_tb,
                               ws=ws_dump)
        sop.sop_proposal_train_step(mlp_obj, pts_tb, T_tb, lr=1e-4, loss=loss_tb, ws=ws_tr)
        mark("proposal_train", 1)
        if timed:
            torch.cuda.synchronize()
            for n in names:
                acc[n] += ev[n][0].elapsed_time(ev[n][1])

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    bake_plan.check()
    assert bool(torch.isfinite(rgb).all()), "non-finite shading output"

    # whole-step timing (no per-phase synchronisation inside)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        step(False)
    end.record()
    torch.cuda.synchronize()
    ms_per_step = start.elapsed_time(end) / args.steps

    # per-phase timing in separate passes
    for _ in range(args.steps):
        step(True)
    phase = {n: acc[n] / args.steps for n in names}
    print(f"# phases (ms): {json.dumps({k: round(v, 4) for k, v in phase.items()})}",
          file=sys.stderr, flush=True)

    samples = N * S
    # the metric: samples per second of the shading forward + backward
    value = samples / ((phase["shade_fwd"] + phase["shade_bwd"]) * 1e-3)
    step_rate = samples / (ms_per_step * 1e-3)

    # roofline of the dominant kernel (each phase is one kernel launch except bake_grid)
    dom = max(("shade_fwd", "shade_bwd", "bake"), key=lambda n: phase[n])
    if dom == "bake":
        work = bake_work()
        rays = P * R * R
        flops = rays * work["resolved_per_ray_mean"] * work["flops_per_resolved"]
        achieved = flops / (phase["bake"] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": "k_bake", "achieved": round(achieved, 5),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 6),
                "traffic": measured_traffic("k_bake"),
                "flops_per_unit": work["flops_per_resolved"],
                "units_per_launch": round(rays * work["resolved_per_ray_mean"]),
                "unit_def": "Gaussian resolved on a ray (accepted, up to the one ending it)",
                "launch_ms": round(phase["bake"], 4)}
        # how busy the vector ALUs were while doing the search (counter summary)
        issue = counter_summary("k_bake_object_valu.txt", "valu_issue_fraction")
        if issue is not None:
            roof["valu_issue_frac"] = issue
    else:
        f = flops_fwd(K) if dom == "shade_fwd" else flops_bwd(K)
        kern = "k_shade_fwd_cl" if dom == "shade_fwd" else "k_shade_bwd_batched"
        achieved = samples * f / (phase[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": kern, "achieved": round(achieved, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": measured_traffic(kern),
                "flops_per_unit": f, "units_per_launch": samples,
                "unit_def": "shaded point-direction sample", "launch_ms": round(phase[dom], 4)}
    # the shading kernels' own figures (the metric's fwd+bwd rate)
    shade_roof = {}
    for n, f, kern in (("shade_fwd", flops_fwd(K), "k_shade_fwd_cl"),
                       ("shade_bwd", flops_bwd(K), "k_shade_bwd_batched")):
        a = samples * f / (phase[n] * 1e-3) / 1e12
        shade_roof[n] = {"achieved_tflops": round(a, 3), "frac": round(a / PEAK_FP32_TFLOPS, 4),
                         "flops_per_sample": f, "launch_ms": round(phase[n], 4)}
        # HBM side: counter-measured bytes of the same kernel over its measured time
        hb = measured_traffic(kern)
        if hb is not None:
            bw = hb / (phase[n] * 1e-3) / 1e9
            shade_roof[n].update({"hbm_bytes": round(hb), "hbm_GBps": round(bw, 1),
                                  "hbm_frac": round(bw / PEAK_HBM_GBS, 4)})

    # the two ways to shade with the proposal on this workload, timed outside the step:
    # network to memory then sampling (two calls), or the network inside the shading kernel
    def time_ms(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record()
        for _ in range(reps):
            fn()
        a1.record()
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) / reps
    nb_p = sop.sop_knn(plan, pts, K)
    t_two = time_ms(lambda: (sop.sop_proposal_infer(mlp_obj, pts, ws=ws_inf, out=probs),
                             sop.sop_shade(plan, tex, env, pts, S_PROP, nb=nb_p, ws=ws_pf,
                                           out=rgb_p, probs=probs, mix_eps=MIX_EPS)))
    t_fused = time_ms(lambda: sop.sop_shade(plan, tex, env, pts, S_PROP, nb=nb_p, ws=ws_pf,
                                            out=rgb_p, net=mlp_obj, mix_eps=MIX_EPS))
    proposal_paths = {"two_call_ms": round(t_two, 4), "fused_ms": round(t_fused, 4)}

    # the deterministic adjoint (exact accumulation of g_env and g_tex), outside the step:
    # its time next to the step's adjoint, and that two runs give the same bits
    acc = sop.workspace(L.load().sop_shade_backward_acc_size(P, R, int(env.shape[0]),
                                                             int(env.shape[1])), dev)
    ge_d, gt_d = torch.zeros_like(g_env), torch.zeros_like(g_tex)

    def det_bwd():
        ge_d.zero_()
        gt_d.zero_()
        return sop.sop_shade_backward(plan, tex, env, pts, grad, S, nb=nb_p, g_env=ge_d,
                                      g_tex=gt_d, ws=ws_b, deterministic=True, acc=acc)
    t_det = time_ms(det_bwd, reps=5)
    first = (ge_d.clone(), gt_d.clone())
    det_bwd()
    torch.cuda.synchronize()
    deterministic_bwd = {"ms": round(t_det, 4), "atomic_ms": round(phase["shade_bwd"], 4),
                         "same_bits_twice": bool(torch.equal(first[0], ge_d)
                                                 and torch.equal(first[1], gt_d))}
    del first, ge_d, gt_d, acc

    trace = None
    if not args.no_trace_study:
        trace = trace_study(torch, sop, scenes, time_ms, bake_plan, plan, env, pts, tex, nb_p,
                            S, phase, (sc.bounds_lo, sc.bounds_hi))
        print(f"# trace study: {json.dumps(trace)}", file=sys.stderr, flush=True)

    shadow = None
    if not args.no_shadow_study:
        shadow = shadow_study(torch, sop, scenes, time_ms, bake_plan, R)
        print(f"# shadow study: {json.dumps(shadow)}", file=sys.stderr, flush=True)

    envs = None
    if not args.no_env_study:
        import numpy as np
        sky = torch.from_numpy(np.random.default_rng(5).lognormal(0.0, 1.5, (256, 256, 3))
                               .astype(np.float32)).to(dev)
        oct_env = sop.OctEnv(sky)
        g_sky = torch.zeros_like(sky)
        ws_fo = sop.workspace(plan.workspace_size(L.SOP_OP_SHADE, N, K, S, (256, 256), True), dev)
        ws_bo = sop.workspace(plan.workspace_size(L.SOP_OP_SHADE_BACKWARD, N, K, S, (256, 256),
                                                  True), dev)
        t_fo = time_ms(lambda: sop.sop_shade(plan, tex, oct_env, pts, S, nb=nb_p, ws=ws_fo,
                                             out=rgb))
        t_bo = time_ms(lambda: sop.sop_shade_backward(plan, tex, oct_env, pts, grad, S, nb=nb_p,
                                                      g_env=g_sky, g_tex=g_tex, ws=ws_bo))
        envs = {"workload": "object: 200k points, S=128, K=8; the step's 256x512 "
                            "equirectangular sky against a 256x256 octahedral one",
                "equirect_fwd_ms": round(phase["shade_fwd"], 4),
                "equirect_bwd_ms": round(phase["shade_bwd"], 4),
                "octahedral_fwd_ms": round(t_fo, 4), "octahedral_bwd_ms": round(t_bo, 4)}
        print(f"# env study: {json.dumps(envs)}", file=sys.stderr, flush=True)

    place = None
    if not args.no_place_study:
        place = place_study(torch, sop, scenes, time_ms, tex)
        print(f"# place study: {json.dumps(place)}", file=sys.stderr, flush=True)

    frames = None
    if not args.no_frames_study:
        frames = frames_study(torch, dev, sop, scenes, cpu=not args.no_cpu_baseline)
        print(f"# frames study: {json.dumps(frames)}", file=sys.stderr, flush=True)

    envis = None
    if not args.no_envis_study:
        envis = envis_study(torch, sop, scenes, time_ms, plan, tex, pts, nb_p, S, K,
                            phase["shade_fwd"])
        print(f"# envis study: {json.dumps(envis)}", file=sys.stderr, flush=True)

    study = study_written = None
    if not args.no_proposal_study:
        study_written = proposal_study_written(torch, dev)
        print(f"# proposal study (as the workload states it): {json.dumps(study_written)}",
              file=sys.stderr, flush=True)
        study = proposal_study(torch, dev, args.proposal_steps)
        print(f"# proposal study (online): {json.dumps(study)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sc, gs, probes_np, R, args.cpu_seconds, samples)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "object_scene: bake 100k Gaussians into 4096 probes x 32x32 "
                               "texels, probe grid, kNN (K=8), shade fwd+bwd of 200k points "
                               "x 128 directions, env 256x512; proposal network on 200k "
                               "points, proposal shade x 32 directions, one proposal "
                               "training step (4096 points)",
                   "points": N, "dirs": S, "k": K, "probes": P, "res": R, "gaussians": G},
        "value_def": "N*S / (t_shade_fwd + t_shade_bwd), both kernels timed inside the step",
        "step_samples_per_s": round(step_rate, 1),
        "phase_ms": {k: round(v, 4) for k, v in phase.items()},
        "roofline": roof,
        "shade_roofline": shade_roof,
        "proposal_paths": proposal_paths,
        "deterministic_bwd": deterministic_bwd,
        "frames_study": frames,
        "proposal_study_as_written": study_written,
        "proposal_study": study,
        "envis_study": envis,
        "trace_study": trace,
        "shadow_study": shadow,
        "place_study": place,
        "env_study": envs,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


def _proposal_eval(torch, sop, plan, tex, env, ev, nb, mlp, ref, mask) -> dict:
    """Hammersley and proposal estimates of the points `ev` against the reference `ref`:
    RMSE (over `mask`, or all points when None) and time per call at each direction count,
    S* = the fewest proposal directions whose RMSE reaches the Hammersley RMSE at 128, and
    the speedup t(Hammersley 128) / min(t(network) + t(proposal S*), t(fused S*))."""
    def rmse(x):
        d = (x - ref) if mask is None else (x - ref)[mask]
        return float(torch.sqrt(torch.mean(d ** 2)))

    def timed(fn, reps=10):
        out = fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            out = fn()
        b.record()
        torch.cuda.synchronize()
        return out, a.elapsed_time(b) / reps

    ham = {}
    for S in (16, 32, 64, 128, 256):
        out, ms = timed(lambda: sop.sop_shade(plan, tex, env, ev, S, nb=nb, seed=7))
        ham[S] = {"rmse": round(rmse(out), 5), "ms": round(ms, 4)}
    # the cosine-weighted set of the same counts (no adjoint, forward only)
    cos = {}
    for S in (16, 32, 64, 128, 256):
        out, ms = timed(lambda: sop.sop_shade(plan, tex, env, ev, S, nb=nb, seed=7,
                                              cosine=True))
        cos[S] = {"rmse": round(rmse(out), 5), "ms": round(ms, 4)}
    probs, t_mlp = timed(lambda: sop.sop_proposal_infer(mlp, ev))
    prop = {}
    for S in (4, 8, 16, 24, 32, 64):
        out, ms = timed(lambda: sop.sop_shade(plan, tex, env, ev, S, nb=nb, seed=7, probs=probs,
                                              mix_eps=MIX_EPS))
        prop[S] = {"rmse": round(rmse(out), 5), "ms": round(ms, 4)}
    target = ham[128]["rmse"]
    s_star = next((S for S in sorted(prop) if prop[S]["rmse"] <= target), None)
    # the same draws with the network evaluated inside the shading kernel (no probability
    # array in memory); the speedup is taken with the faster of the two paths
    _, t_fused = timed(lambda: sop.sop_shade(plan, tex, env, ev, s_star or 32, nb=nb, seed=7,
                                             net=mlp, mix_eps=MIX_EPS))
    t_two = (t_mlp + prop[s_star]["ms"]) if s_star else None
    best = min(t_two, t_fused) if s_star else None
    speedup = (ham[128]["ms"] / best) if s_star else None
    return {"hammersley": ham, "cosine": cos, "proposal": prop,
            "network_ms": round(t_mlp, 4),
            "S_star": s_star,
            "speedup_vs_hammersley_128": round(speedup, 3) if speedup else None,
            "speedup_path": ("fused" if t_fused < t_two else "two_call") if s_star else None,
            "two_call_ms_at_S_star": round(t_two, 4) if s_star else None,
            "fused_ms_at_S_star": round(t_fused, 4)}


def _reference_spot_check(torch, ev_sc, ref, n_dirs=4096, n_check=1000, seed=123) -> dict:
    """The GPU reference estimate (Hammersley, n_dirs directions) against the oracle on
    n_check sampled points: max and 99.9th percentile of the relative error (floored at
    1e-3 of the mean, as the parity tests measure)."""
    import numpy as np

    import oracle
    rows = np.sort(np.random.default_rng(41).choice(ev_sc.n, n_check, replace=False))
    sub = ev_sc.subset(rows)
    idx, w = oracle.knn(sub.probe_pos, sub.bounds_lo, sub.bounds_hi, sub.pos, sub.normal,
                        sub.k)
    ro = oracle.shade(sub, idx, w, n_dirs=n_dirs, seed=seed)
    g = ref.cpu().numpy()[rows].astype(np.float64)
    tau = 1e-3 * float(np.mean(np.abs(ro)))
    err = np.abs(g - ro) / np.maximum(np.abs(ro), tau)
    return {"points": n_check, "dirs": n_dirs, "max_rel_err": float(f"{err.max():.3e}"),
            "p99_9_rel_err": float(f"{np.percentile(err, 99.9):.3e}")}


def proposal_study_written(torch, dev, train_steps: int = 3000, eval_every: int = 100) -> dict:
    """The learned-proposal workload as stated: the network is trained on 2,097,152
    integrand samples of the tiny scene (4096 points x 512 directions, two per bin, dumped
    once), then 200k held-out points are shaded with the Hammersley set and with proposal
    samples; RMSE over all points and RGB against the 4096-direction Hammersley estimate,
    which is itself spot-checked against the oracle on 1000 points. With one fixed batch the
    network overfits it as the steps go on, so training stops early: every `eval_every`
    steps the proposal RMSE at 32 directions is measured on 4096 validation points (their
    own stream, not the evaluation set) and the parameters with the lowest one are kept."""
    import numpy as np

    from paper_2510_07729_amd import _lib as L
    from paper_2510_07729_amd import proposal, scenes, sop
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)   # noqa: E731

    def pts_of(sc):
        return sop.Points(d(sc.pos), d(sc.normal), d(sc.albedo), d(sc.rough), d(sc.metal),
                          view=d(sc.view))

    train_sc = scenes.proposal_eval(TRAIN_BATCH, seed=5)
    ev_sc = scenes.proposal_eval(200_000, seed=0)
    plan = sop.Plan(d(train_sc.probe_pos), train_sc.bounds_lo, train_sc.bounds_hi)
    tex, env = d(train_sc.texels), d(train_sc.env)
    tr, ev = pts_of(train_sc), pts_of(ev_sc)
    mlp = proposal.default_mlp(dev, train_sc.bounds_lo, train_sc.bounds_hi, seed=0)
    val = pts_of(scenes.proposal_eval(4096, seed=17))
    nb_val = sop.sop_knn(plan, val, 4)
    ref_val = sop.sop_shade(plan, tex, env, val, 4096, nb=nb_val, seed=123)
    mask_val = val.rough >= 0.25

    def val_rmse():
        probs = sop.sop_proposal_infer(mlp, val)
        x = sop.sop_shade(plan, tex, env, val, 32, nb=nb_val, seed=7, probs=probs,
                          mix_eps=MIX_EPS)
        return float(torch.sqrt(torch.mean(((x - ref_val)[mask_val]) ** 2)))

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    T = sop.sop_dump_integrand(plan, tex, env, tr, 2, k=4, seed=0)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ws_t = sop.proposal_workspace(L.SOP_OP_PROPOSAL_TRAIN, tr.n, dev)
    best = (val_rmse(), 0, mlp.params.clone())
    trace = []
    for it in range(train_steps):
        lr = 2e-3 * 0.5 * (1.0 + math.cos(math.pi * it / train_steps))
        sop.sop_proposal_train_step(mlp, tr, T, lr=lr, loss=loss, ws=ws_t)
        if (it + 1) % eval_every == 0:
            r = val_rmse()
            trace.append((it + 1, round(float(loss.item()), 4), round(r, 5)))
            if r < best[0]:
                best = (r, it + 1, mlp.params.clone())
    mlp.params.copy_(best[2])
    e1.record()
    torch.cuda.synchronize()
    losses = [t[1] for t in trace[:: max(1, len(trace) // 5)]]
    nb = sop.sop_knn(plan, ev, 4)
    ref = sop.sop_shade(plan, tex, env, ev, 4096, nb=nb, seed=123)
    masked = _proposal_eval(torch, sop, plan, tex, env, ev, nb, mlp, ref, ev.rough >= 0.25)
    out = {"workload": "tiny scene geometry; trained on 4096 points x 512 directions "
                       "(2,097,152 integrand samples, dumped once); 200k held-out points, "
                       "K=4, RMSE over all points and RGB against 4096 Hammersley directions",
           "train_integrand_samples": TRAIN_BATCH * 512, "train_steps": train_steps,
           "kept_step": best[1], "validation_rmse_at_kept": round(best[0], 5),
           "validation_trace": trace[:: max(1, len(trace) // 8)],
           "train_ms": round(e0.elapsed_time(e1), 1),
           "loss_trace": [round(x, 4) for x in losses], "mix_eps": MIX_EPS}
    out.update(_proposal_eval(torch, sop, plan, tex, env, ev, nb, mlp, ref, None))
    # the same network judged over the points whose lobes the reference resolves
    out["roughness_ge_0.25"] = {k: masked[k] for k in ("hammersley", "proposal", "S_star",
                                                        "speedup_vs_hammersley_128")}
    out["reference_vs_oracle"] = _reference_spot_check(torch, ev_sc, ref)
    return out


def proposal_study(torch, dev, steps: int) -> dict:
    """Speedup at matched error of the learned proposal on the tiny scene's geometry (64
    probes with 16x16 maps, 32x64 environment, K=4), online variant: training on a pool of
    262,144 points with fresh targets every step, then 200k held-out points shaded with the
    fixed Hammersley set and with proposal samples, each against a 4096-direction Hammersley
    reference. RMSE is taken over the points with roughness >= 0.25, whose lobes the
    reference itself resolves (narrower lobes are not converged by 4096 uniform directions
    either)."""
    import numpy as np

    from paper_2510_07729_amd import proposal, scenes, sop
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)   # noqa: E731

    def pts_of(sc):
        return sop.Points(d(sc.pos), d(sc.normal), d(sc.albedo), d(sc.rough), d(sc.metal),
                          view=d(sc.view))

    pool_sc = scenes.proposal_eval(262_144, seed=5)
    ev_sc = scenes.proposal_eval(200_000, seed=0)
    plan = sop.Plan(d(pool_sc.probe_pos), pool_sc.bounds_lo, pool_sc.bounds_hi)
    tex, env = d(pool_sc.texels), d(pool_sc.env)
    pool, ev = pts_of(pool_sc), pts_of(ev_sc)
    mlp = proposal.default_mlp(dev, pool_sc.bounds_lo, pool_sc.bounds_hi, seed=0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    losses = proposal.train(mlp, plan, tex, env, pool, steps, batch=TRAIN_BATCH, lr=2e-3,
                            log_every=max(1, steps // 4))
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)

    nb = sop.sop_knn(plan, ev, 4)
    ref = sop.sop_shade(plan, tex, env, ev, 4096, nb=nb, seed=123)
    out = {"workload": "tiny scene geometry, 200k held-out points, K=4, RMSE over "
                       "roughness >= 0.25 against 4096 Hammersley directions",
           "train_steps": steps, "train_batch": TRAIN_BATCH,
           "train_integrand_samples": proposal.integrand_samples(steps, TRAIN_BATCH),
           "train_ms": round(train_ms, 1), "loss_trace": [round(x, 4) for x in losses],
           "mix_eps": MIX_EPS}
    out.update(_proposal_eval(torch, sop, plan, tex, env, ev, nb, mlp, ref, ev.rough >= 0.25))
    return out


def frames_oracle(sc, stride=64) -> dict:
    """The oracle's forward on every stride-th pixel of the frames workload (its neighbour
    lists found and its maps widened to FP64 beforehand, after one untimed warm-up call),
    with all host threads, extrapolated to the whole workload and labelled as such."""
    import dataclasses

    import numpy as np

    import oracle
    # every stride-th pixel of every frame, frame-major, so each point keeps its camera
    ppf = sc.points_per_frame
    per = np.arange(0, ppf, stride)
    rows = np.concatenate([f * ppf + per for f in range(sc.cam_pos.shape[0])])
    sub = dataclasses.replace(sc, pos=sc.pos[rows], normal=sc.normal[rows],
                              albedo=sc.albedo[rows], rough=sc.rough[rows],
                              metal=sc.metal[rows], points_per_frame=len(per),
                              texels=sc.texels.astype(np.float64))
    idx, w = oracle.knn(sub.probe_pos, sub.bounds_lo, sub.bounds_hi, sub.pos, sub.normal,
                        sub.k)
    warm = dataclasses.replace(sub, pos=sub.pos[:64], normal=sub.normal[:64],
                               albedo=sub.albedo[:64], rough=sub.rough[:64],
                               metal=sub.metal[:64], points_per_frame=64)
    oracle.shade(warm, idx[:64], w[:64])
    t = time.time()
    oracle.shade(sub, idx, w)
    dt = time.time() - t
    samples = len(rows) * sc.n_dirs
    return {"kind": "oracle", "samples_per_s": round(samples / dt, 1),
            "cores": oracle.max_threads(),
            "sample": f"shade forward on every {stride}th pixel of each frame ({len(rows)} of "
                      f"{sc.n} points, "
                      f"{dt:.1f}s), neighbour lists found beforehand; "
                      f"extrapolated to all points: {sc.n * sc.n_dirs / (samples / dt):.1f}s"}


def frames_study(torch, dev, sop, scenes, reps=10, cpu=True) -> dict:
    """The G-buffer frames workload: 8 frames of 1920x1080 (16,588,800 points, views from
    the frames' cameras), 16,384 probes with 32x32 f16 maps, S = 64, K = 8, 256x512
    environment: one forward call over all frames with the neighbour lists given, timed with
    events, its samples per second and its share of the FP32 roof."""
    import numpy as np
    from paper_2510_07729_amd import _lib as L
    t0 = time.time()
    sc = scenes.gbuffer_frames()
    build_s = time.time() - t0
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)   # noqa: E731
    N, S, K = sc.n, sc.n_dirs, sc.k
    pts = sop.Points(d(sc.pos), d(sc.normal), d(sc.albedo), d(sc.rough), d(sc.metal),
                     cam_pos=d(sc.cam_pos), points_per_frame=sc.points_per_frame)
    plan = sop.Plan(d(sc.probe_pos), sc.bounds_lo, sc.bounds_hi)
    tex, env = d(sc.texels), d(sc.env)
    cpu_ref = frames_oracle(sc) if cpu else None
    del sc
    t_knn = time_ms_plain(lambda: sop.sop_knn(plan, pts, K), reps=3)
    nb = sop.sop_knn(plan, pts, K)
    out = torch.empty((N, 3), dtype=torch.float32, device=dev)
    ws = sop.workspace(plan.workspace_size(L.SOP_OP_SHADE, N, K, S, env.shape[:2], True), dev)
    t = time_ms_plain(lambda: sop.sop_shade(plan, tex, env, pts, S, nb=nb, ws=ws, out=out),
                      reps=reps)
    assert bool(torch.isfinite(out).all()), "non-finite frames output"
    samples = N * S
    ach = samples * flops_fwd(K) / (t * 1e-3) / 1e12
    res = {"workload": "8 frames x 1920x1080 G-buffers (16,588,800 points, camera views), "
                       "16,384 probes with 32x32 f16 maps, S=64, K=8, env 256x512",
           "points": N, "dirs": S, "k": K, "build_s": round(build_s, 1),
           "knn_ms": round(t_knn, 3), "shade_fwd_ms": round(t, 3),
           "samples_per_s": round(samples / (t * 1e-3), 1),
           "frames_per_s": round(8 / (t * 1e-3), 2),
           "cpu_oracle": cpu_ref,
           "roofline": {"bound": "alu", "kernel": "k_shade_fwd_cl", "achieved": round(ach, 3),
                        "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(ach / PEAK_FP32_TFLOPS, 4),
                        "flops_per_unit": flops_fwd(K), "units_per_launch": samples}}
    hb = measured_traffic("k_shade_fwd_cl", "frames")
    if hb is not None:
        bw = hb / (t * 1e-3) / 1e9
        res["roofline"]["traffic"] = round(hb)
        res["hbm_GBps"] = round(bw, 1)
        res["hbm_frac"] = round(bw / PEAK_HBM_GBS, 4)
    return res


def envis_study(torch, sop, scenes, time_ms, plan, tex, pts, nb, S, K, t_fwd_equirect,
                subset=4096, S_ref=4096) -> dict:
    """Object relighting with environment importance sampling (Eq. 18) against the
    Hammersley set on the object workload, under a 256x256 octahedral outdoor sky whose sun
    holds ~70% of the energy: the time of each at the step's S on all points, and their
    relative RMSE of the irradiance output (the cosine-weighted incident light; rgb errors
    of uniform sampling are dominated by rare hits of narrow GGX lobes on the sun) against a
    Hammersley estimate at S_ref directions on `subset` points; S* = the fewest importance
    samples whose error is at most the Hammersley error at S. Two weightings of the same
    draws: "env" with the paper's mean-solid-angle density, which converges to 4 pi times
    the mean of the integrand over the octahedral square, not to the integral, so its error
    levels off at that bias; "env_exact" with the draws' exact density (unbiased)."""
    import numpy as np
    dev = pts.pos.device
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)   # noqa: E731
    sky = sop.OctEnv(d(scenes.octahedral_sky(np.random.default_rng(9), 256)))
    sub = sop.Points(pts.pos[:subset], pts.normal[:subset], pts.albedo[:subset],
                     pts.rough[:subset], pts.metal[:subset], view=pts.view[:subset])
    nbs = sop.sop_knn(plan, sub, K)
    _, ref = sop.sop_shade(plan, tex, sky, sub, S_ref, nb=nbs, seed=77, irradiance=True)
    norm = float(torch.sqrt(torch.mean(ref ** 2)))

    def err(out):
        x = out[1]
        return round(float(torch.sqrt(torch.mean((x - ref) ** 2))) / norm, 5)

    counts = (4, 8, 16, 32, 64, 128, 256)
    modes = {"env": True, "env_exact": "exact"}
    e_ham = {n: err(sop.sop_shade(plan, tex, sky, sub, n, nb=nbs, seed=5, irradiance=True))
             for n in counts}
    e_cos = {n: err(sop.sop_shade(plan, tex, sky, sub, n, nb=nbs, seed=5, irradiance=True,
                                  cosine=True)) for n in counts}
    t_ham = time_ms(lambda: sop.sop_shade(plan, tex, sky, pts, S, nb=nb, seed=5))
    out = {"workload": "object: 200k points, K=8, 256x256 octahedral sky with a sun "
                       "(~70% of the energy); errors on 4096 points against 4096 "
                       "Hammersley directions",
           "error_on": "irradiance", "dirs": S, "hammersley_ms": round(t_ham, 4),
           "rel_rmse": {"hammersley": e_ham, "cosine": e_cos}}
    for name, mode in modes.items():
        e = {n: err(sop.sop_shade(plan, tex, sky, sub, n, nb=nbs, seed=5, irradiance=True,
                                  env_sampling=mode)) for n in counts}
        t_env = time_ms(lambda: sop.sop_shade(plan, tex, sky, pts, S, nb=nb, seed=5,
                                              env_sampling=mode))
        s_star = next((n for n in counts if e[n] <= e_ham[S]), None)
        t_star = (time_ms(lambda: sop.sop_shade(plan, tex, sky, pts, s_star, nb=nb, seed=5,
                                                env_sampling=mode)) if s_star else None)
        # the matched count and speedup for smaller Hammersley budgets too
        matched = {}
        for nh in (16, 32, 64):
            ne = next((n for n in counts if e[n] <= e_ham[nh]), None)
            if ne is None:
                matched[nh] = None
                continue
            th = time_ms(lambda: sop.sop_shade(plan, tex, sky, pts, nh, nb=nb, seed=5))
            te = time_ms(lambda: sop.sop_shade(plan, tex, sky, pts, ne, nb=nb, seed=5,
                                               env_sampling=mode))
            matched[nh] = {"env_dirs": ne, "hammersley_ms": round(th, 4),
                           "env_ms": round(te, 4), "speedup": round(th / te, 3)}
        out["rel_rmse"][name] = e
        out[name] = {"ms": round(t_env, 4), "S_star": s_star,
                     "ms_at_S_star": round(t_star, 4) if t_star else None,
                     "speedup_matched": round(t_ham / t_star, 3) if t_star else None,
                     "matched_at_smaller_budgets": matched}
    return out


def trace_study(torch, sop, scenes, time_ms, bake_plan, plan, env, pts, tex, nb, S, phase,
                bounds, subset=4096, S_ref=4096, seed_ref=77) -> dict:
    """Traced shading (every sample's O and L_in from its own ray through the Gaussians)
    against probe shading on the object workload: the time of each at the step's S, and
    their errors against a traced reference at S_ref directions on a point subset. The
    errors are taken on the irradiance output (the cosine-weighted incident light, which
    holds exactly what the probes approximate, O and L_in, without the noise of sampling
    narrow specular lobes uniformly); S* is the fewest traced directions whose error is at
    most the probes' error at S."""
    import numpy as np
    dev = pts.pos.device
    N = pts.n
    offset = 0.01 * scenes.OBJECT_DIAGONAL
    H, W = int(env.shape[0]), int(env.shape[1])
    lib = bake_plan._lib
    rgb_t = torch.empty((N, 3), dtype=torch.float32, device=dev)
    # rays of nearby points are traced together: a plan over the shading points orders them
    torch.cuda.synchronize()
    t0 = time.time()
    order = sop.Plan(pts.pos, bounds[0], bounds[1])
    torch.cuda.synchronize()
    t_order = (time.time() - t0) * 1e3

    def ws_for(n, s):
        return sop.workspace(lib.sop_shade_traced_workspace_size(order.handle, n, s, H, W, 0),
                             dev)

    ws_t = ws_for(N, S)
    t_trace = time_ms(lambda: sop.sop_shade_traced(bake_plan, env, pts, S, offset,
                                                   order_by=order, ws=ws_t, out=rgb_t), reps=3)
    del ws_t
    rgb_sop, irr_sop = sop.sop_shade(plan, tex, env, pts, S, nb=nb, irradiance=True)
    rows = torch.from_numpy(np.sort(np.random.default_rng(11).choice(N, subset, replace=False)))
    rows = rows.to(dev)
    sub = sop.Points(pts.pos[rows], pts.normal[rows], pts.albedo[rows], pts.rough[rows],
                     pts.metal[rows], view=pts.view[rows])
    _, ref = sop.sop_shade_traced(bake_plan, env, sub, S_ref, offset, seed=seed_ref,
                                  irradiance=True, order_by=order)
    den = float((ref.double() ** 2).mean())

    def rel_rmse(x):
        return float(((x.double() - ref.double()) ** 2).mean() / den) ** 0.5

    err_sop = rel_rmse(irr_sop[rows])
    err_trace = {}
    for s in (4, 8, 16, 32, 64, 128, 256, 512, 1024):
        _, irr = sop.sop_shade_traced(bake_plan, env, sub, s, offset, irradiance=True,
                                      order_by=order)
        err_trace[s] = rel_rmse(irr)
    # the probes' own bias: probe shading against traced shading with the same directions
    rgb_tr_S, irr_tr_S = sop.sop_shade_traced(bake_plan, env, sub, S, offset, irradiance=True,
                                              order_by=order)
    bias = float(((irr_sop[rows].double() - irr_tr_S.double()) ** 2).mean() / den) ** 0.5
    s_star = min((s for s, e in err_trace.items() if e <= err_sop), default=None)
    t_star = None
    if s_star is not None:
        ws_s = ws_for(N, s_star)
        t_star = time_ms(lambda: sop.sop_shade_traced(bake_plan, env, pts, s_star, offset,
                                                      order_by=order, ws=ws_s, out=rgb_t),
                         reps=3)
        del ws_s
    t_sop = phase["shade_fwd"]
    t_bake = phase["bake"] + phase["bake_grid"]
    return {
        "workload": "object_scene: 100k Gaussians, 200k points, rays from x + 1% of the "
                    "diagonal along n, env 256x512",
        "dirs": S, "trace_ms": round(t_trace, 3), "rays_per_s": round(N * S / (t_trace * 1e-3)),
        "point_order_ms": round(t_order, 3),
        "sop_shade_ms": round(t_sop, 4), "sop_bake_ms": round(t_bake, 3),
        "speedup_same_dirs": round(t_trace / t_sop, 2),
        "speedup_same_dirs_with_bake": round(t_trace / (t_sop + t_bake), 3),
        "error_on": "irradiance", "ref_dirs": S_ref, "ref_points": subset,
        "rel_rmse_sop": round(err_sop, 5),
        "rel_rmse_sop_vs_trace_same_dirs": round(bias, 5),
        "rel_rmse_trace": {str(k): round(v, 5) for k, v in err_trace.items()},
        "S_star": s_star, "trace_ms_at_S_star": None if t_star is None else round(t_star, 3),
        "speedup_matched": None if t_star is None else round(t_star / t_sop, 2),
        "speedup_matched_with_bake": None if t_star is None else round(t_star / (t_sop + t_bake),
                                                                       3),
    }


def time_ms_plain(fn, reps=10):
    """Average milliseconds of fn() on the current stream (one untimed call first)."""
    import torch
    fn()
    torch.cuda.synchronize()
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a0.record()
    for _ in range(reps):
        fn()
    a1.record()
    torch.cuda.synchronize()
    return a0.elapsed_time(a1) / reps


def place_study(torch, sop, scenes, time_ms, tex) -> dict:
    """Probe placement of the object workload on the GPU (4096 probes by farthest point
    sampling over 65,536 surface samples, raised by 1% of the diagonal) and the losses of
    the reconstruction step: L_sops of the step's baked maps against a perturbed copy (the
    traced targets) with its gradient, L_lam of 200k points; their HBM rates against the
    8 TB/s peak (bytes: both maps read and the gradient written; roughness and metallic read,
    their gradients written)."""
    import numpy as np
    dev = tex.device
    pts, nrm = scenes.object_surface(scenes.rng(scenes.CFG_OBJECT, 10, 0), 65536)
    pts_t = torch.from_numpy(pts.astype(np.float32)).to(dev)
    nrm_t = torch.from_numpy(nrm.astype(np.float32)).to(dev)
    off = 0.01 * scenes.OBJECT_DIAGONAL
    t_fps = time_ms(lambda: sop.sop_place_probes(pts_t, nrm_t, 4096, 0, off), reps=3)
    target = tex * 0.97 + 0.01
    T = tex.numel() // 4
    ws = sop.workspace(sop.L.load().sop_loss_workspace_size(T), dev)
    loss_o = torch.empty(2, dtype=torch.float32, device=dev)
    grad_o = torch.empty_like(tex)
    # the C entry point with its arguments built once: the call costs a few microseconds of
    # host time, not the tens a wrapper that allocates its outputs would add to a ~35 us kernel
    lib = sop.L.load()
    args = (tex.data_ptr(), target.data_ptr(), T, loss_o.data_ptr(), grad_o.data_ptr(),
            ws.data_ptr(), ws.numel(), sop._stream())
    sop.L.check(lib.sop_sops_loss(*args), "sop_sops_loss")
    t_sops = time_ms(lambda: lib.sop_sops_loss(*args), reps=50)
    g = np.random.default_rng(3)
    r = torch.from_numpy(g.uniform(0.05, 1, 200_000).astype(np.float32)).to(dev)
    m = torch.from_numpy(g.uniform(0, 1, 200_000).astype(np.float32)).to(dev)
    t_lam = time_ms(lambda: sop.sop_lam_loss(r, m), reps=20)
    b_sops = 3 * 16 * T
    b_lam = 4 * 4 * 200_000
    return {
        "workload": "object: 4096 probes from 65,536 surface samples; L_sops on the 4096 "
                    "baked 32x32 maps; L_lam on 200k points",
        "fps_ms": round(t_fps, 3), "fps_picks": 4096, "fps_points": 65536,
        "fps_hbm_bytes": measured_traffic("k_fps"),
        "sops_loss_ms": round(t_sops, 4), "sops_bytes": b_sops,
        "sops_GBps": round(b_sops / (t_sops * 1e-3) / 1e9, 1),
        "sops_hbm_frac": round(b_sops / (t_sops * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "sops_hbm_bytes": measured_traffic("k_sops_loss"),
        "lam_hbm_bytes": measured_traffic("k_lam_loss"),
        "lam_loss_ms": round(t_lam, 4), "lam_bytes": b_lam,
        "lam_GBps": round(b_lam / (t_lam * 1e-3) / 1e9, 1),
    }


def shadow_setup(torch, sop, scenes, bake_plan, R, dev):
    """The shadow workload on the GPU: 2048 ground probes baked from the object's Gaussians
    (channel 3 = the object's occlusion O'), their plan and the ground points' neighbours."""
    import numpy as np
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)   # noqa: E731
    sc = scenes.shadow_scene(textures=np.zeros((1, 2, 2, 4), np.float32))
    probes = d(sc.probe_pos)
    plan = sop.Plan(probes, sc.bounds_lo, sc.bounds_hi)
    tex, _ = sop.sop_bake(bake_plan, probes, R, depth=False, order_by=plan)
    pts = sop.Points(d(sc.pos), d(sc.normal), None, None, None)
    nb = sop.sop_knn(plan, pts, sc.k)
    return sc, plan, tex, d(sc.env), pts, nb


def shadow_study(torch, sop, scenes, time_ms, bake_plan, R, subset=4096, S_ref=4096) -> dict:
    """Cast-shadow ratio of the ground under the object with the Hammersley set and with
    environment importance sampling (Eq. 18) at S = 64: time of each, and their errors
    against a Hammersley reference at S_ref on a point subset, over the points the object
    shadows (reference ratio below 0.98 in some channel); S* is the fewest importance
    samples whose error is at most the Hammersley error at 64, for the draws weighted with
    Eq. 18's density and with their exact density."""
    import numpy as np
    from paper_2510_07729_amd import _lib as L
    dev = torch.device("cuda", 0)
    sc, plan, tex, env, pts, nb = shadow_setup(torch, sop, scenes, bake_plan, R, dev)
    N, S = sc.n, sc.n_dirs
    out = torch.empty((N, 3), dtype=torch.float32, device=dev)

    def run(n_dirs, sampler, p=pts, nbl=nb, o=out):
        return sop.sop_shadow_ratio(plan, tex, env, p, n_dirs, nb=nbl, sampler=sampler, out=o)

    t_ham = time_ms(lambda: run(S, L.SOP_SHADOW_HAMMERSLEY))
    t_env = time_ms(lambda: run(S, L.SOP_SHADOW_ENV))
    t_env_x = time_ms(lambda: run(S, L.SOP_SHADOW_ENV_EXACT))
    rows = torch.from_numpy(np.sort(np.random.default_rng(13).choice(N, subset, replace=False)))
    rows = rows.to(dev)
    sub = sop.Points(pts.pos[rows], pts.normal[rows], None, None, None)
    nb_s = sop.sop_knn(plan, sub, sc.k)
    ref = sop.sop_shadow_ratio(plan, tex, env, sub, S_ref, nb=nb_s,
                               sampler=L.SOP_SHADOW_HAMMERSLEY, seed=101).double()
    shadowed = (ref < 0.98).any(dim=1)
    n_sh = int(shadowed.sum())

    def err(x):
        x = x.double()
        return float(((x[shadowed] - ref[shadowed]) ** 2).mean().sqrt()) if n_sh else 0.0

    samplers = (("hammersley", L.SOP_SHADOW_HAMMERSLEY), ("env", L.SOP_SHADOW_ENV),
                ("env_exact", L.SOP_SHADOW_ENV_EXACT))
    e = {name: {} for name, _ in samplers}
    for s_ in (4, 8, 16, 32, 64, 128, 256):
        for name, smp in samplers:
            e[name][str(s_)] = round(err(sop.sop_shadow_ratio(plan, tex, env, sub, s_, nb=nb_s,
                                                              sampler=smp)), 5)
    target = e["hammersley"][str(S)]
    s_star = min((int(k) for k, v in e["env"].items() if v <= target), default=None)
    t_star = None if s_star is None else time_ms(lambda: run(s_star, L.SOP_SHADOW_ENV))
    s_star_x = min((int(k) for k, v in e["env_exact"].items() if v <= target), default=None)
    t_star_x = (None if s_star_x is None
                else time_ms(lambda: run(s_star_x, L.SOP_SHADOW_ENV_EXACT)))
    mean_ratio = float(run(S, L.SOP_SHADOW_HAMMERSLEY).mean())
    return {
        "workload": "shadow_scene: object over a ground plane, 2048 ground probes (32x32) "
                    "baked from the object's 100k Gaussians, 500k ground points, 256x256 "
                    "octahedral sky with a sun, K=8",
        "dirs": S, "points": N, "hammersley_ms": round(t_ham, 4), "env_ms": round(t_env, 4),
        "env_exact_ms": round(t_env_x, 4),
        "samples_per_s_hammersley": round(N * S / (t_ham * 1e-3)),
        "samples_per_s_env": round(N * S / (t_env * 1e-3)),
        "mean_ratio": round(mean_ratio, 4),
        "ref_dirs": S_ref, "ref_points": subset, "shadowed_points": n_sh,
        "rmse_ratio": e, "S_star_env": s_star,
        "env_ms_at_S_star": None if t_star is None else round(t_star, 4),
        "speedup_matched": None if t_star is None else round(t_ham / t_star, 3),
        "S_star_env_exact": s_star_x,
        "env_exact_ms_at_S_star": None if t_star_x is None else round(t_star_x, 4),
        "speedup_matched_exact": None if t_star_x is None else round(t_ham / t_star_x, 3),
    }


def shadow_only(torch, dev, sop, scenes) -> int:
    """The shadow ratio of the shadow workload with both samplers at S = 64: one warm-up and
    three timed calls each (the probes baked from the object's Gaussians once)."""
    import numpy as np
    from paper_2510_07729_amd import _lib as L
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)   # noqa: E731
    gs = scenes.object_gaussians()
    bplan = sop.BakePlan(d(gs.mean), d(gs.scale), d(gs.rotation), d(gs.opacity), d(gs.color))
    sc, plan, tex, env, pts, nb = shadow_setup(torch, sop, scenes, bplan, 32, dev)
    res = {}
    for name, smp in (("hammersley", L.SOP_SHADOW_HAMMERSLEY), ("env", L.SOP_SHADOW_ENV)):
        out = sop.sop_shadow_ratio(plan, tex, env, pts, sc.n_dirs, nb=nb, sampler=smp)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            sop.sop_shadow_ratio(plan, tex, env, pts, sc.n_dirs, nb=nb, sampler=smp, out=out)
        e1.record()
        torch.cuda.synchronize()
        res[name + "_ms"] = round(e0.elapsed_time(e1) / 3, 4)
    print(json.dumps(res), flush=True)
    return 0


def trace_only(torch, dev, sop, scenes) -> int:
    """Traced shading of the object workload (200k points, 128 directions, 100k Gaussians):
    one warm-up and three timed calls, points ordered by a plan over themselves."""
    import numpy as np
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)   # noqa: E731
    gs = scenes.object_gaussians()
    sc = scenes.object_scene(textures=np.zeros((1, 2, 2, 4), np.float32))
    bplan = sop.BakePlan(d(gs.mean), d(gs.scale), d(gs.rotation), d(gs.opacity), d(gs.color))
    pts = sop.Points(d(sc.pos), d(sc.normal), d(sc.albedo), d(sc.rough), d(sc.metal),
                     view=d(sc.view))
    env = d(sc.env)
    order = sop.Plan(pts.pos, sc.bounds_lo, sc.bounds_hi)
    off = 0.01 * scenes.OBJECT_DIAGONAL
    rgb = sop.sop_shade_traced(bplan, env, pts, sc.n_dirs, off, order_by=order)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        sop.sop_shade_traced(bplan, env, pts, sc.n_dirs, off, order_by=order, out=rgb)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    print(json.dumps({"traced_shade_ms": round(ms, 3), "points": sc.n, "dirs": sc.n_dirs,
                      "gaussians": gs.count,
                      "rays_per_s": round(sc.n * sc.n_dirs / (ms * 1e-3))}), flush=True)
    return 0


def peaks() -> int:
    """Device-rate microbenchmarks (paper_2510_07729_amd/csrc/peaks.hip), each the mean of
    20 launches after one warm-up; prints one JSON line per benchmark."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2510_07729_amd", "libsop_peaks.so"))
    lib.sop_peak_name.restype = C.c_char_p
    lib.sop_peak_unit.restype = C.c_char_p
    lib.sop_peak_run.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double)]
    for w in range(lib.sop_peak_count()):
        rate, ms = C.c_double(), C.c_double()
        rc = lib.sop_peak_run(w, 20, C.byref(rate), C.byref(ms))
        if rc != 0:
            print(json.dumps({"peak": lib.sop_peak_name(w).decode(), "error": rc}), flush=True)
            return 1
        print(json.dumps({"peak": lib.sop_peak_name(w).decode(), "rate": round(rate.value, 2),
                          "unit": lib.sop_peak_unit(w).decode(),
                          "ms_per_launch": round(ms.value, 4)}), flush=True)
    return 0


def copy_calibration(torch, dev) -> int:
    """A plain device-to-device copy of 1 GiB, three times: its FETCH_SIZE / WRITE_SIZE
    counters per dispatch give the scale between those counters and HBM bytes."""
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "repeats": 3}))
    return 0


def bake_work() -> dict:
    """Resolved Gaussians per ray on this workload, measured once with the brute-force
    reference trace (tests/golden/make_bake_work.py) and stored as data."""
    with open(os.path.join(ROOT, "tests", "golden", "bake_work_object.json")) as f:
        return json.load(f)


def counter_summary(fname: str, key: str):
    """A figure from a committed rocprofv3 counter summary under profiles/, or None when the
    summary is missing or was taken on a different source of the kernel."""
    import hashlib
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = vals.get("source")
    if not src or key not in vals:
        return None
    fn, digest = src.split("@")
    h = hashlib.sha256(open(os.path.join(ROOT, fn), "rb").read()).hexdigest()[:16]
    return float(vals[key]) if h == digest else None


def measured_traffic(kernel: str, workload: str = "object"):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this kernel
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None when the
    summary is missing or was taken on a different source of the kernel."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = vals.get("source")
    if not src or "bytes_per_launch" not in vals:
        return None
    fname, digest = src.split("@")
    h = hashlib.sha256(open(os.path.join(ROOT, fname), "rb").read()).hexdigest()[:16]
    return float(vals["bytes_per_launch"]) if h == digest else None


def cpu_baseline(sc, gs, probes_np, R, seconds, samples_gpu_step):
    """The oracle on a bounded sample of the same workload. value: shading forward +
    backward samples per second (the metric; the neighbour lists are found beforehand and
    not timed, as on the GPU, where the search is its own phase) with all host threads, on
    a subset of points sized to about a third of the budget; the same at one thread; and the
    whole step's rate with the brute-force bake of a subset of rays added, extrapolated to
    200k points and 4.19M rays."""
    import numpy as np

    import oracle
    threads = oracle.max_threads()
    rng = np.random.default_rng(7)

    def shade_time(m):
        rows = rng.choice(sc.n, m, replace=False)
        sub = sc.subset(rows)
        grad = rng.standard_normal((m, 3))
        idx, w = oracle.knn(sub.probe_pos, sub.bounds_lo, sub.bounds_hi, sub.pos, sub.normal,
                            sub.k)
        t = time.time()
        oracle.shade(sub, idx, w)
        oracle.shade_backward(sub, idx, w, grad)
        return time.time() - t

    def grow(fn, start, limit, budget):
        """run fn on growing sample sizes until one takes about `budget` seconds"""
        m = start
        t = fn(m)
        while t < 0.7 * budget and m < limit:
            m = int(min(limit, m * min(8.0, max(1.5, budget / max(t, 1e-3)))))
            t = fn(m)
        return m, t

    m, t_shade = grow(shade_time, 256, sc.n, seconds / 3.0)
    per_point = t_shade / m
    oracle.set_threads(1)
    try:
        m1, t_shade1 = grow(shade_time, 16, sc.n, seconds / 3.0)
    finally:
        oracle.set_threads(threads)
    per_point1 = t_shade1 / m1

    P = probes_np.shape[0]
    def bake_time(n):
        rp = rng.integers(0, P, n).astype(np.int32)
        rt = rng.integers(0, R * R, n).astype(np.int32)
        t = time.time()
        oracle.bake_rays(gs, probes_np.astype(np.float64), R, rp, rt)
        return time.time() - t

    nr, t_bake = grow(bake_time, 64, P * R * R, seconds / 3.0)
    per_ray = t_bake / nr

    t_step = per_point * sc.n + per_ray * P * R * R
    return {"value": round(sc.n_dirs / per_point, 1), "unit": "samples/s",
            "cores": threads, "kind": "oracle",
            "sample": f"shade fwd+bwd on {m} of {sc.n} points with {threads} threads "
                      f"({t_shade:.1f}s) and on {m1} points with 1 thread ({t_shade1:.1f}s), "
                      f"neighbour lists found beforehand; brute-force bake of {nr} of "
                      f"{P * R * R} rays ({t_bake:.1f}s) for the whole step; host CPU: "
                      f"{cpu_model()}",
            "value_1_thread": round(sc.n_dirs / per_point1, 1),
            "step_samples_per_s": round(sc.n * sc.n_dirs / t_step, 3)}


def _report_children() -> None:
    """Names any child process still alive at exit on stderr (the benchmark starts none; the
    oracle's gcc build, when its library is stale, is waited for)."""
    try:
        import psutil
        kids = psutil.Process().children(recursive=True)
    except Exception:
        return
    if kids:
        names = [f"{k.pid}:{k.name()}" for k in kids]
        print(f"# child processes at exit: {names}", file=sys.stderr, flush=True)


if __name__ == "__main__":
    rc = main()
    _report_children()
    sys.exit(rc)
