"""Pins of the unprojection / new-view rendering oracle (oracle.render):
closed forms for single points, the identity view, the z-test and its tie
rule, culling, and a point-by-point z-buffer loop on small random clouds."""
import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(313)
INTR = (64.0, 60.0, 31.5, 23.5)
IDENT = np.hstack([np.eye(3), np.zeros((3, 1))])


def _zbuffer_loop(points, rgb, pose, intr, H, W):
    """The same view by visiting points in index order with a strict z-test."""
    fx, fy, cx, cy = intr
    P = np.asarray(pose, dtype=np.float64).reshape(3, 4)
    best = np.full((H, W), np.inf)
    win = np.full((H, W), -1)
    pts = points.reshape(-1, 4)
    for n in range(pts.shape[0]):
        if pts[n, 3] <= 0:
            continue
        x, y, z = P[:, :3] @ pts[n, :3] + P[:, 3]
        if z <= 0:
            continue
        iu, iv = int(np.floor(fx * x / z + cx + 0.5)), int(np.floor(fy * y / z + cy + 0.5))
        if 0 <= iu < W and 0 <= iv < H and z < best[iv, iu]:
            best[iv, iu], win[iv, iu] = z, n
    return win


def test_unproject_closed_form():
    depth = np.zeros((48, 64), np.uint16)
    depth[10, 20] = 1500
    pts = oracle.unproject(depth, INTR)
    assert np.allclose(pts[10, 20], [(20 - 31.5) * 1500 / 64, (10 - 23.5) * 1500 / 60, 1500, 1])
    assert pts[0, 0, 3] == 0 and pts[0, 0, 2] == 0


def test_identity_view_reproduces_the_frame():
    depth = RNG.integers(500, 3000, (48, 64)).astype(np.uint16)
    depth[RNG.uniform(size=depth.shape) < 0.1] = 0
    rgb = RNG.integers(0, 256, (48, 64, 3), dtype=np.uint8)
    c, d, w = oracle.render_view(oracle.unproject(depth, INTR), rgb, IDENT, INTR, 48, 64)
    hole = depth == 0
    assert np.array_equal(d, depth) and np.array_equal(c[~hole], rgb[~hole]) and not c[hole].any()
    assert np.array_equal(w[~hole], np.flatnonzero(~hole.reshape(-1)))


def test_sideways_move_shifts_by_fx_t_over_z():
    depth = np.zeros((48, 64), np.uint16)
    depth[20, 30] = 1280
    rgb = np.zeros((48, 64, 3), np.uint8)
    rgb[20, 30] = (9, 8, 7)
    pose = IDENT.copy()
    pose[0, 3] = 100.0  # fx * 100 / 1280 = 5 pixels
    c, d, w = oracle.render_view(oracle.unproject(depth, INTR), rgb, pose, INTR, 48, 64)
    assert w[20, 35] == 20 * 64 + 30 and d[20, 35] == 1280 and tuple(c[20, 35]) == (9, 8, 7)
    assert (w >= 0).sum() == 1


def test_nearer_point_wins_and_ties_go_to_the_lower_index():
    pts = np.zeros((1, 4, 4))
    pts[0, 0] = (0, 0, 2000, 1)
    pts[0, 1] = (0, 0, 1000, 1)
    pts[0, 2] = (0, 0, 1000, 1)
    pts[0, 3] = (0, 0, 500, 0)  # not a measurement
    rgb = np.array([[[1, 1, 1], [2, 2, 2], [3, 3, 3], [4, 4, 4]]], np.uint8)
    c, d, w = oracle.render_view(pts, rgb, IDENT, (10.0, 10.0, 2.0, 2.0), 5, 5)
    assert w[2, 2] == 1 and d[2, 2] == 1000 and tuple(c[2, 2]) == (2, 2, 2)


def test_points_behind_the_camera_and_outside_are_dropped():
    depth = np.full((48, 64), 1000, np.uint16)
    flip = IDENT.copy()
    flip[2, 2] = -1.0  # every Z' < 0
    _, _, w = oracle.render_view(oracle.unproject(depth, INTR), np.zeros((48, 64, 3), np.uint8), flip, INTR, 48, 64)
    assert (w < 0).all()
    far = IDENT.copy()
    far[0, 3] = 1e6  # everything moves out of the frame
    _, _, w = oracle.render_view(oracle.unproject(depth, INTR), np.zeros((48, 64, 3), np.uint8), far, INTR, 48, 64)
    assert (w < 0).all()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_render_matches_a_point_by_point_zbuffer(seed):
    r = np.random.default_rng(seed)
    depth = r.integers(0, 3000, (20, 24)).astype(np.uint16)
    rgb = r.integers(0, 256, (20, 24, 3), dtype=np.uint8)
    a = r.uniform(-0.3, 0.3)
    pose = np.array([[np.cos(a), 0, np.sin(a), 150.0], [0, 1, 0, -80.0], [-np.sin(a), 0, np.cos(a), 300.0]])
    intr = (24.0, 24.0, 11.5, 9.5)
    pts = oracle.unproject(depth, intr)
    _, _, w = oracle.render_view(pts, rgb, pose, intr, 20, 24)
    assert np.array_equal(w, _zbuffer_loop(pts, rgb, pose, intr, 20, 24))
