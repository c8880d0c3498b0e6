"""sop_shade_noalloc (shading with the library's fixed device scratch, for callers that
cannot allocate) against sop_shade with a caller workspace, through the C ABI: two calls
in a row, the second with fewer points, each identical to sop_shade; a call whose workspace
would exceed the fixed array is refused before any device work."""
import numpy as np
import pytest

from paper_2510_07729_amd import scenes
from tests.gpu_util import dev, gpu_plan, gpu_points, log

pytestmark = pytest.mark.gpu


def test_noalloc_matches_workspace_call_twice():
    import torch
    from paper_2510_07729_amd import _lib as L
    from paper_2510_07729_amd import sop
    assert torch.cuda.is_available()
    sc = scenes.object_scene()
    plan = gpu_plan(sc)
    tex, env = dev(sc.texels), dev(sc.env)
    # first call: the whole object workload with the neighbour search inside the call
    # (the largest scratch use); second: fewer points with given neighbour lists, so stale
    # contents of the first call sit in the array
    for n, with_nb, seed in ((sc.n, False, 5), (777, True, 6)):
        log(f"no-alloc shading: N={n}, neighbour lists given: {with_nb}")
        sub = sc.subset(np.arange(n))
        pts = gpu_points(sub)
        nb = sop.sop_knn(plan, pts, sc.k) if with_nb else None
        ref, ref_e = sop.sop_shade(plan, tex, env, pts, sc.n_dirs, k=sc.k, nb=nb, seed=seed,
                                   irradiance=True)
        out = torch.full((n, 3), float("nan"), device="cuda")
        irr = torch.full((n, 3), float("nan"), device="cuda")
        sop.sop_shade_noalloc(plan, tex, env, pts, sc.n_dirs, out, k=sc.k, nb=nb, seed=seed,
                              irradiance=irr)
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and torch.equal(irr, ref_e)
    # a workspace beyond the array: the neighbour lists of 600k points at K = 8 (43 MB)
    big = scenes.tiny_shade(n_points=600_000, seed=2)
    plan_b = gpu_plan(big)
    out = torch.zeros((big.n, 3), device="cuda")
    with pytest.raises(L.SopError) as e:
        sop.sop_shade_noalloc(plan_b, dev(big.texels), dev(big.env), gpu_points(big), 64, out,
                              k=8)
    assert e.value.status == L.SOP_ERR_WORKSPACE_TOO_SMALL
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 0).all())
