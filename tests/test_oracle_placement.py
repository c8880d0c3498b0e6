"""Pins of the oracle's probe placement (farthest point sampling + normal offset, Sec. 3.1.2)
and of the L_lam / L_sops losses: hand-derived picks on a line, the defining argmax checked
by brute force on small clouds, the non-increasing pick distances every FPS run has, losses
and gradients in closed form, and the gradients against central differences."""
import numpy as np
import pytest

import oracle

F32 = np.float32


def test_fps_on_a_line_by_hand():
    # from 0 the far end 9, then the middle (4 and 5 tie at 16: lowest index), then 2, 6
    x = np.zeros((10, 3), F32)
    x[:, 0] = np.arange(10)
    c = oracle.fps(x, 10)
    assert c[:5].tolist() == [0, 9, 4, 2, 6]
    assert sorted(c.tolist()) == list(range(10))


@pytest.mark.parametrize("M,P,start", [(200, 40, 0), (257, 64, 17), (64, 64, 63)])
def test_fps_picks_the_farthest_point_every_time(M, P, start):
    """Brute force of the definition in single precision: pick k is the point with the
    largest squared distance to its nearest earlier pick (ties: lowest index)."""
    x = np.random.default_rng(M).uniform(-1, 1, (M, 3)).astype(F32)
    c = oracle.fps(x, P, start)
    assert c[0] == start
    for k in range(1, P):
        d = x[:, None, :] - x[c[:k]][None, :, :]
        s = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        m = s.min(axis=1)
        assert c[k] == int(np.flatnonzero(m == m.max())[0])


def test_fps_pick_distances_never_increase():
    x = np.random.default_rng(3).standard_normal((500, 3)).astype(F32)
    c = oracle.fps(x, 100)
    xd = x.astype(np.float64)
    pick = [np.min(np.sum((xd[c[:k]] - xd[c[k]]) ** 2, axis=1)) for k in range(1, 100)]
    assert np.all(np.diff(pick) <= 1e-6 * np.array(pick[:-1]))


def test_place_offsets_along_the_normal():
    x = np.array([[1, 2, 3], [0.5, -1, 0.25]], F32)
    n = np.array([[0, 0, 1], [0, -1, 0]], F32)
    out = oracle.place(x, n, np.array([1, 0], np.int32), 0.5)
    assert out.tolist() == [[0.5, -1.5, 0.25], [1.0, 2.0, 3.5]]


def test_sops_loss_closed_form():
    tex = np.array([[1, 2, 3, 0.5], [0, 0, 0, 0]], F32)
    tgt = np.array([[0, 2, 5, 1], [1, 1, 1, 0]], F32)
    loss, g = oracle.sops_loss(tex, tgt)
    assert loss.tolist() == [(1 + 0 + 2 + 1 + 1 + 1) / 6, (0.5 + 0) / 2]
    assert g.tolist() == [[1 / 6, 0, -1 / 6, -1 / 2], [-1 / 6, -1 / 6, -1 / 6, 0]]


def test_lam_loss_closed_form():
    loss, gr, gm = oracle.lam_loss(np.array([1, 0.5, 0.25], F32), np.array([0, 0.5, 0.25], F32))
    assert loss.tolist() == [(0 + 0.5 + 0.75) / 3, (0 + 0.5 + 0.25) / 3]
    assert gr.tolist() == [0, -1 / 3, -1 / 3] and gm.tolist() == [0, 1 / 3, 1 / 3]


def test_loss_gradients_match_central_differences():
    g = np.random.default_rng(5)
    tex = g.uniform(0, 1, (3, 4, 4, 4)).astype(F32)
    tgt = g.uniform(0, 1, tex.shape).astype(F32)
    loss, grad = oracle.sops_loss(tex, tgt)
    h = 1e-3
    for idx in [(0, 0, 0, 0), (1, 2, 3, 3), (2, 1, 0, 2), (0, 3, 3, 3)]:
        tp, tm = tex.copy(), tex.copy()
        tp[idx] += h
        tm[idx] -= h
        fd = (oracle.sops_loss(tp, tgt)[0].sum() - oracle.sops_loss(tm, tgt)[0].sum()) / (
            float(tp[idx]) - float(tm[idx]))
        assert fd == pytest.approx(grad[idx], rel=1e-3)
    r = g.uniform(0, 1, 50).astype(F32)
    m = g.uniform(0, 1, 50).astype(F32)
    _, gr, gm = oracle.lam_loss(r, m)
    for i in (0, 17, 49):
        rp, rm = r.copy(), r.copy()
        rp[i] += h
        rm[i] -= h
        fd = (oracle.lam_loss(rp, m)[0].sum() - oracle.lam_loss(rm, m)[0].sum()) / (
            float(rp[i]) - float(rm[i]))
        assert fd == pytest.approx(gr[i], rel=1e-3)
