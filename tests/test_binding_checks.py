"""The Python binding checks every tensor's shape (and the dtype of accumulated gradients)
before a pointer reaches the C ABI, which receives bare pointers and cannot check sizes:
a wrong size would otherwise turn into an out-of-bounds device access. These checks run
before any device work, so CPU tensors reach them."""
import types

import pytest
import torch

from paper_2510_07729_amd import sop

N, P, R = 10, 6, 8


def pts(n=N, **over):
    f = dict(pos=torch.zeros(n, 3), normal=torch.zeros(n, 3), albedo=torch.zeros(n, 3),
             rough=torch.zeros(n), metal=torch.zeros(n), view=torch.zeros(n, 3))
    f.update(over)
    return sop.Points(**f)


def plan(p=P):
    return types.SimpleNamespace(n_probes=p)


def tex(p=P, dtype=torch.float32):
    return torch.zeros(p, R, R, 4, dtype=dtype)


ENV = torch.zeros(4, 8, 3)


@pytest.mark.parametrize("field,bad", [("pos", torch.zeros(N, 2)), ("normal", torch.zeros(N - 1, 3)),
                                       ("albedo", torch.zeros(N, 4)), ("rough", torch.zeros(N + 1)),
                                       ("metal", torch.zeros(N, 1)), ("view", torch.zeros(3, N))])
def test_points_rows(field, bad):
    with pytest.raises(ValueError, match=field):
        pts(**{field: bad}).check()


def test_camera_mode_frame_count():
    p = pts(view=None, cam_pos=torch.zeros(3, 3), points_per_frame=4)
    with pytest.raises(ValueError, match="points_per_frame"):
        p.check()
    pts(view=None, cam_pos=torch.zeros(2, 3), points_per_frame=5).check()


def test_texture_count_must_match_plan():
    with pytest.raises(ValueError, match="plan"):
        sop.sop_shade(plan(P + 1), tex(), ENV, pts(), 16)
    with pytest.raises(ValueError, match="plan"):
        sop.sop_shade_backward(plan(P - 1), tex(), ENV, pts(), torch.zeros(N, 3), 16)


def test_shade_output_and_probability_shapes():
    with pytest.raises(ValueError, match="out"):
        sop.sop_shade(plan(), tex(), ENV, pts(), 16, out=torch.zeros(N, 4))
    with pytest.raises(ValueError, match="probs"):
        sop.sop_shade(plan(), tex(), ENV, pts(), 16, probs=torch.zeros(N, 255))


def test_backward_gradient_buffers():
    g = torch.zeros(N, 3)
    with pytest.raises(ValueError, match="grad_rgb"):
        sop.sop_shade_backward(plan(), tex(), ENV, pts(), torch.zeros(N - 1, 3), 16)
    # an f16 gradient over f16 texels would take f32 atomics over twice its bytes
    with pytest.raises(ValueError, match="g_tex"):
        sop.sop_shade_backward(plan(), tex(dtype=torch.float16), ENV, pts(), g, 16,
                               g_tex=torch.zeros(P, R, R, 4, dtype=torch.float16))
    with pytest.raises(ValueError, match="g_tex"):
        sop.sop_shade_backward(plan(), tex(), ENV, pts(), g, 16, g_tex=torch.zeros(P, R, R, 3))
    with pytest.raises(ValueError, match="g_env"):
        sop.sop_shade_backward(plan(), tex(), ENV, pts(), g, 16, g_env=torch.zeros(4, 9, 3))
    with pytest.raises(ValueError, match="g_env"):
        sop.sop_shade_backward(plan(), tex(), ENV, pts(), g, 16,
                               g_env=torch.zeros(4, 8, 3, dtype=torch.float64))


def test_neighbor_lists_rows():
    nb = sop.Neighbors(torch.zeros(N, dtype=torch.int32), torch.zeros(N - 2, 4, dtype=torch.int32),
                       torch.zeros(N - 2, 4))
    with pytest.raises(ValueError, match="nb.idx"):
        sop.sop_shade(plan(), tex(), ENV, pts(), 16, nb=nb)
    nb = sop.Neighbors(torch.zeros(N, dtype=torch.int32), torch.zeros(N, 4, dtype=torch.int32),
                       torch.zeros(N, 3))
    with pytest.raises(ValueError, match="nb.w"):
        sop.sop_shade(plan(), tex(), ENV, pts(), 16, nb=nb)


def test_plan_rebuild_probe_count():
    p = sop.Plan.__new__(sop.Plan)
    p.n_probes = P
    with pytest.raises(ValueError, match="probe_pos"):
        p.rebuild(torch.zeros(P + 1, 3))


def test_other_entry_points():
    with pytest.raises(ValueError, match="dirs"):
        sop.sop_query(plan(), tex(), pts(), torch.zeros(N + 1, 5, 3))
    with pytest.raises(ValueError, match="out"):
        sop.sop_dump_integrand(plan(), tex(), ENV, pts(), 1, out=torch.zeros(N, 128))
    with pytest.raises(ValueError, match="texels"):
        sop.sop_bake(None, torch.zeros(P, 3), R, texels=torch.zeros(P, R, R + 1, 4))
    with pytest.raises(ValueError, match="samples_out"):
        sop.sop_shade_traced(None, ENV, pts(), 8, 0.01, samples_out=torch.zeros(N, 7, 4))
    with pytest.raises(ValueError, match="normals"):
        sop.sop_place_probes(torch.zeros(20, 3), torch.zeros(19, 3), 4)
    with pytest.raises(ValueError, match="target"):
        sop.sop_sops_loss(torch.zeros(5, 4), torch.zeros(6, 4))
    with pytest.raises(ValueError, match="metal"):
        sop.sop_lam_loss(torch.zeros(5), torch.zeros(6))
    with pytest.raises(ValueError, match="out"):
        sop.sop_shadow_ratio(plan(), tex(), torch.zeros(8, 8, 3), pts(), 16,
                             out=torch.zeros(N + 1, 3))


def test_env_sampling_modes():
    assert sop.shade_opts(16, 4, env_sampling="exact").sampler == sop.L.SOP_SAMPLER_ENV_EXACT
    assert sop.shade_opts(16, 4, env_sampling=True).sampler == sop.L.SOP_SAMPLER_ENV
    with pytest.raises(ValueError, match="env_sampling"):
        sop.shade_opts(16, 4, env_sampling="eq18")
