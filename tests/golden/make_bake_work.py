"""Writes bake_work_object.json: how many Gaussians the bake definition (Sec. 3.1.2, SOP
textures initialised by ray tracing; compositing of Eq. 1) has to resolve per ray on the
object workload (100k Gaussians, 4096 probes at 32x32), measured with the oracle's
brute-force trace on a seeded sample of rays. A resolved Gaussian is an accepted one
(t* > t_min, alpha >= alpha_min) up to and including the one that ends the ray.

This is the algorithmic work unit of the bake's roofline; only the oracle is called.
Usage: python tests/golden/make_bake_work.py [n_rays]
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle                                   # noqa: E402
from paper_2510_07729_amd import scenes        # noqa: E402

# FP32 operations of one resolved Gaussian, counted from the definition (FMA = 2):
# Sigma^-1 d (15), t* from two dot products and a divide (11), mu - o (3),
# x = o + t* d - mu (9), Sigma^-1 x (15), m^2 (5), exp(-m^2/2) (2), alpha clamp (2),
# compositing of colour, depth, weight and transmittance (11).
FLOPS_PER_RESOLVED = 73


def main(n_rays: int = 4096) -> None:
    gs = scenes.object_gaussians()
    probes = scenes.object_probes()
    R = 32
    rng = np.random.default_rng(20251007)
    rp = rng.integers(0, probes.shape[0], n_rays).astype(np.int32)
    rt = rng.integers(0, R * R, n_rays).astype(np.int32)
    _, _, used = oracle.bake_rays(gs, probes.astype(np.float64), R, rp, rt, used=True)
    mean = float(used.mean())
    out = {"workload": "object scene: 100k Gaussians, 4096 probes, 32x32 texels",
           "rays_sampled": n_rays, "seed": 20251007,
           "resolved_per_ray_mean": mean,
           "resolved_per_ray_stderr": float(used.std(ddof=1) / np.sqrt(n_rays)),
           "resolved_per_ray_max": int(used.max()),
           "flops_per_resolved": FLOPS_PER_RESOLVED}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bake_work_object.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 4096)
