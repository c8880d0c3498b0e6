"""Training loop of the learned direction proposal (host orchestration only).

Every step is two library calls on the GPU: sop_dump_integrand writes fresh bin targets for
a batch of shading points (the shading step's own integrand, drawn with a new seed each step)
and sop_proposal_train_step runs the network's forward, cross-entropy backward and Adam on
them. The batch is a contiguous slice of a pool of points in random order (drawn i.i.d.), so
no gather runs outside the library.
"""
from __future__ import annotations

import math
from typing import List, Optional

import torch

from . import _lib as L
from . import sop


def _slice(p: sop.Points, a: int, b: int) -> sop.Points:
    return sop.Points(pos=p.pos[a:b], normal=p.normal[a:b], albedo=p.albedo[a:b],
                      rough=p.rough[a:b], metal=p.metal[a:b],
                      view=p.view[a:b] if p.view is not None else None)


def train(mlp: sop.Mlp, plan: sop.Plan, texels: torch.Tensor, env: torch.Tensor,
          pool: sop.Points, steps: int, batch: int = 4096, lr: float = 2e-3,
          samples_per_bin: int = 1, k: int = 4, seed: int = 0,
          log_every: int = 0, start: int = 0, stop: Optional[int] = None) -> List[float]:
    """Online training on `pool` (view-mode points in random order). Learning rate follows a
    cosine decay from lr to 0 over `steps`. Iterations start .. min(stop, steps) - 1 run: a
    run stopped after iteration i and saved (Mlp.save) resumes with start = i + 1 and
    continues bit for bit, since a step's batch, seed and learning rate depend only on its
    iteration number.
    Returns the losses read back every `log_every` steps."""
    if pool.view is None:
        raise ValueError("the training pool needs per-point view directions")
    n = pool.n
    batch = min(batch, n)
    per_epoch = n // batch
    dev = pool.pos.device
    T = torch.empty((batch, L.SOP_MLP_BINS), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ws_d = sop.workspace(plan.workspace_size(L.SOP_OP_DUMP_INTEGRAND, batch, k, 1, env.shape[:2]),
                         dev)
    ws_t = sop.proposal_workspace(L.SOP_OP_PROPOSAL_TRAIN, batch, dev)
    out: List[float] = []
    for it in range(start, steps if stop is None else min(stop, steps)):
        a = (it % per_epoch) * batch
        sub = _slice(pool, a, a + batch)
        sop.sop_dump_integrand(plan, texels, env, sub, samples_per_bin, k=k,
                               seed=(seed * 1_000_003 + it) & 0xFFFFFFFF, out=T, ws=ws_d)
        cur = lr * 0.5 * (1.0 + math.cos(math.pi * it / steps))
        sop.sop_proposal_train_step(mlp, sub, T, lr=cur, loss=loss, ws=ws_t)
        if log_every and (it % log_every == 0 or it == steps - 1):
            out.append(float(loss.item()))
    return out


def train_fixed(mlp: sop.Mlp, plan: sop.Plan, texels: torch.Tensor, env: torch.Tensor,
                pts: sop.Points, steps: int, samples_per_bin: int = 2, lr: float = 2e-3,
                k: int = 4, seed: int = 0, log_every: int = 0) -> List[float]:
    """Training on one fixed set of integrand samples: the bin targets of `pts` are dumped
    once (pts.n * 256 * samples_per_bin evaluations of the integrand), then `steps` Adam
    steps are taken on that batch with a cosine decay of the learning rate from lr to 0.
    Returns the losses read back every `log_every` steps."""
    if pts.view is None:
        raise ValueError("the training points need per-point view directions")
    dev = pts.pos.device
    T = sop.sop_dump_integrand(plan, texels, env, pts, samples_per_bin, k=k,
                               seed=seed & 0xFFFFFFFF)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ws_t = sop.proposal_workspace(L.SOP_OP_PROPOSAL_TRAIN, pts.n, dev)
    out: List[float] = []
    for it in range(steps):
        cur = lr * 0.5 * (1.0 + math.cos(math.pi * it / steps))
        sop.sop_proposal_train_step(mlp, pts, T, lr=cur, loss=loss, ws=ws_t)
        if log_every and (it % log_every == 0 or it == steps - 1):
            out.append(float(loss.item()))
    return out


def integrand_samples(steps: int, batch: int, samples_per_bin: int = 1) -> int:
    """Number of integrand evaluations a training run of `steps` steps consumes."""
    return steps * batch * L.SOP_MLP_BINS * samples_per_bin


def default_mlp(device, bounds_lo, bounds_hi, seed: int = 0,
                params: Optional[torch.Tensor] = None) -> sop.Mlp:
    from . import scenes
    p = params if params is not None else torch.from_numpy(scenes.mlp_init(seed=seed)).to(device)
    return sop.Mlp(p, bounds_lo, bounds_hi)
