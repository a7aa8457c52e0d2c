"""Pins of the oracle's particle image (Appendix A "Render Technique": a 2D
or perspective 3D projection onto chosen axes, colour fixed or varying
linearly with position; Appendix A.1: model-view and view-projection
transforms, a circular sprite whose intensity falls off from its centre,
additive blending)."""
import numpy as np
import pytest


def perspective(fovy_deg, aspect, near, far):
    """Textbook OpenGL perspective matrix (camera at the origin looking down -z)."""
    f = 1.0 / np.tan(np.radians(fovy_deg) / 2)
    return np.array([[f / aspect, 0, 0, 0],
                     [0, f, 0, 0],
                     [0, 0, (far + near) / (near - far), 2 * far * near / (near - far)],
                     [0, 0, -1, 0]])


def test_white_points_orthographic_equal_histogram(ora):
    # radius 0, white, identity transform: 256 x the 2D histogram of (x, -y)
    rng = np.random.default_rng(0)
    st = rng.uniform(-0.999, 0.999, size=(3, 50000))
    spec = ora.render_spec([0, 1, 2], np.eye(4), 64, 32)
    img, culled = ora.render(st, spec)
    assert culled == 0
    h, _ = ora.histogram(np.stack([st[0], -st[1]]), 0, 1, (-1.0, 1.0), (-1.0, 1.0), 64, 32)
    for k in range(3):
        assert np.array_equal(img[..., k], 256 * h)


def test_perspective_ray_invariance_and_culling(ora):
    # points along one ray from the camera project to the same pixel; points
    # behind the camera or beyond the far plane are culled
    M = perspective(60.0, 1.5, 0.5, 100.0)
    d = np.array([0.3, -0.2, -1.0])
    ts = np.array([1.0, 2.5, 7.0, 40.0])
    st = (d[:, None] * ts[None, :])
    spec = ora.render_spec([0, 1, 2], M, 300, 200)
    img, culled = ora.render(st, spec)
    assert culled == 0
    ys, xs = np.nonzero(img[..., 0])
    assert len(xs) == 1 and img[ys[0], xs[0], 0] == 256 * 4
    behind = np.array([[0.0, 0.1], [0.0, 0.1], [1.0, 200.0]])  # z > 0 is behind, z = -200 beyond far
    behind[2, 1] = -200.0
    _, culled = ora.render(behind, spec)
    assert culled == 2


def test_colour_is_linear_in_position_and_clamped(ora):
    spec = ora.render_spec([0, 1, 2], np.eye(4), 16, 16, base=(0.25, 0.5, 1.5),
                           grad=[[0.25, 0, 0], [0, -0.25, 0], [0, 0, 0]], origin=(0.0, 0.0, 0.0))
    st = np.array([[0.5], [0.5], [0.0]])
    img, _ = ora.render(st, spec)
    px = img[np.nonzero(img.sum(axis=2))][0]
    assert list(px) == [round(256 * (0.25 + 0.125)), round(256 * (0.5 - 0.125)), 256]  # blue clamped at 1


def test_additive_blending_and_accumulate(ora):
    spec = ora.render_spec([0, 1, 2], np.eye(4), 8, 8, radius=2, weight=0.7)
    st = np.array([[0.1, 0.1, -0.4], [0.2, 0.2, 0.3], [0.0, 0.0, 0.0]])
    img, _ = ora.render(st, spec)
    one, _ = ora.render(st[:, :1], spec)
    two, _ = ora.render(st[:, 2:], spec)
    assert np.array_equal(img, 2 * one + two)
    acc, _ = ora.render(st[:, 2:], spec, img=2 * one, n_culled=0)
    assert np.array_equal(acc, img)


@pytest.mark.parametrize("radius", [1, 2, 4])
def test_sprite_symmetry_and_weights(ora, radius):
    # a particle at a pixel centre gives a sprite symmetric under the 8
    # symmetries of the square, peaking at weight (1 - (1/sqrt(2))... ) and
    # with the centre pixel at full weight
    W = 2 * radius + 9
    px = (W // 2 + 0.5)
    a = px / W * 2 - 1
    st = np.array([[a], [-a], [0.0]])
    spec = ora.render_spec([0, 1, 2], np.eye(4), W, W, radius=radius)
    img, _ = ora.render(st, spec)
    g = img[..., 0].astype(np.int64)
    assert g[W // 2, W // 2] == 256
    for t in (g.T, g[::-1], g[:, ::-1]):
        assert np.array_equal(t, g)
    # brute-force weights of every pixel
    want = np.zeros_like(g)
    for iy in range(W):
        for ix in range(W):
            d = np.hypot(ix + 0.5 - px, iy + 0.5 - px)
            if d < radius + 1:
                want[iy, ix] = np.rint(256 * (1 - d / (radius + 1)) ** 2)
    assert np.array_equal(g, want)
