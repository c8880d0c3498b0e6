"""Helpers for the GPU parity tests: move a seeded scene to the GPU, call the library
through its C ABI, and compare with the CPU oracle by the parity metric

    err = |gpu - oracle| / max(|oracle|, tau),  tau = 1e-3 * mean(|oracle|) over the array.
"""
from __future__ import annotations

import dataclasses
import sys

import numpy as np

import oracle
from paper_2510_07729_amd import scenes

TOL = 1e-4


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_points(sc: scenes.ShadeScene, albedo=None, rough=None, metal=None):
    from paper_2510_07729_amd.sop import Points
    return Points(
        pos=dev(sc.pos), normal=dev(sc.normal),
        albedo=dev(sc.albedo if albedo is None else albedo),
        rough=dev(sc.rough if rough is None else rough),
        metal=dev(sc.metal if metal is None else metal),
        view=dev(sc.view) if sc.view is not None else None,
        cam_pos=dev(sc.cam_pos) if sc.cam_pos is not None else None,
        points_per_frame=sc.points_per_frame)


def gpu_plan(sc: scenes.ShadeScene):
    from paper_2510_07729_amd.sop import Plan
    return Plan(dev(sc.probe_pos), sc.bounds_lo, sc.bounds_hi)


def parity_err(gpu: np.ndarray, ref: np.ndarray) -> np.ndarray:
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    tau = 1e-3 * float(np.mean(np.abs(ref))) if ref.size else 0.0
    tau = max(tau, 1e-30)
    return np.abs(gpu - ref) / np.maximum(np.abs(ref), tau)


def sum_err(gpu: np.ndarray, ref: np.ndarray, mass: np.ndarray) -> np.ndarray:
    """Error of a gradient that is a sum of signed terms, relative to its natural scale
    max(|sum|, sum of |terms|): float rounding of a sum is bounded by a multiple of the
    sum of |terms|, which is the sum itself when nothing cancels."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), np.asarray(mass, np.float64))
    diff = np.abs(gpu - ref)
    out = np.zeros_like(diff)
    nz = scale > 0
    out[nz] = diff[nz] / scale[nz]
    out[~nz] = np.where(diff[~nz] > 0, np.inf, 0.0)
    return out


def report(name: str, err: np.ndarray) -> float:
    if err.size == 0:
        log(f"{name}: empty")
        return 0.0
    mx = float(np.max(err))
    p = float(np.percentile(err, 99.99))
    log(f"{name}: max err {mx:.3e}  p99.99 {p:.3e}  n={err.size}")
    return mx


def subset_frames(sc: scenes.ShadeScene, per_frame: int, seed: int = 0) -> scenes.ShadeScene:
    """Camera-mode scene restricted to `per_frame` sampled pixels of every frame (keeps the
    frame-major layout so that each point still sees its own camera)."""
    rng = np.random.default_rng(seed)
    F = sc.cam_pos.shape[0]
    ppf = sc.points_per_frame
    rows = np.concatenate([f * ppf + np.sort(rng.choice(ppf, per_frame, replace=False))
                           for f in range(F)])
    return dataclasses.replace(
        sc, pos=sc.pos[rows].copy(), normal=sc.normal[rows].copy(), view=None,
        albedo=sc.albedo[rows].copy(), rough=sc.rough[rows].copy(),
        metal=sc.metal[rows].copy(), points_per_frame=per_frame), rows


def oracle_knn(sc: scenes.ShadeScene, k=None, radius=float("inf")):
    return oracle.knn(sc.probe_pos, sc.bounds_lo, sc.bounds_hi, sc.pos, sc.normal,
                      sc.k if k is None else k, radius)
