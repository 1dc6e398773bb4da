"""FP64 oracle: RGB-D unprojection and z-buffered rendering of a new view.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes: an RGB-D frame pairs an image with a depth map and is
reconstructed in 3-D by projecting it into Cartesian space (Sec. 2); the
receiver renders the recovered RGB-D frames after recovery, a step it times
at about 3 ms (Sec. 5 microbenchmarks; App. latency breakdown).

Readings where the paper is silent: a pinhole camera with intrinsics (fx, fy,
cx, cy) in pixels and pixel centres at integer coordinates (the synthetic
scenes use fx = fy = W and the image centre); depth is the z coordinate in
mm, and depth 0 marks no measurement; unprojection gives an organised point
cloud, point (u, v) = ((u - cx) Z / fx, (v - cy) Z / fy, Z) with the pixel's
colour; a new view moves points by X' = R X + t (mm) and projects them with
the target intrinsics to the nearest pixel centre; points with Z' <= 0 or
outside the target frame are dropped; each target pixel shows the point of
smallest Z' (ties to the lower point index), its colour and its Z' rounded to
mm (half to even, clamped to u16); pixels no point reaches are 0.
"""
import numpy as np


def unproject(depth, intr):
    """depth [H, W] u16 mm -> points [H, W, 4] float64: (X, Y, Z, valid)."""
    fx, fy, cx, cy = (float(v) for v in intr)
    d = np.asarray(depth).astype(np.float64)
    H, W = d.shape
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    pts = np.zeros((H, W, 4))
    pts[..., 0] = (u - cx) * d / fx
    pts[..., 1] = (v - cy) * d / fy
    pts[..., 2] = d
    pts[..., 3] = (d > 0).astype(np.float64)
    return pts


def project(points, pose, intr):
    """Target-view coordinates of every point: (u', v', Z') float64 arrays
    over the points, with R = pose[:, :3] and t = pose[:, 3]."""
    fx, fy, cx, cy = (float(v) for v in intr)
    P = np.asarray(pose, dtype=np.float64).reshape(3, 4)
    X = points[..., :3].reshape(-1, 3)
    Xc = X @ P[:, :3].T + P[:, 3]
    z = Xc[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * Xc[:, 0] / z + cx
        v = fy * Xc[:, 1] / z + cy
    return u, v, z


def render_view(points, rgb, pose, intr, out_h, out_w):
    """Z-buffered splat of an organised point cloud into the target view:
    returns (rgb_out [out_h, out_w, 3] u8, depth_out [out_h, out_w] u16,
    winner [out_h, out_w] int64 point index or -1)."""
    u, v, z = project(points, pose, intr)
    cols = np.asarray(rgb).reshape(-1, 3)
    n_all = np.arange(u.shape[0])
    keep = (points[..., 3].reshape(-1) > 0) & (z > 0)
    with np.errstate(invalid="ignore"):
        iu, iv = np.floor(u + 0.5), np.floor(v + 0.5)
    keep &= (iu >= 0) & (iu < out_w) & (iv >= 0) & (iv < out_h)
    n = n_all[keep]
    pix = (iv[keep] * out_w + iu[keep]).astype(np.int64)
    # per target pixel, the smallest Z' and then the lowest index: sort by
    # (pixel, Z', index) and take each pixel's first entry
    order = np.lexsort((n, z[keep], pix))
    pix_s, n_s = pix[order], n[order]
    first = np.ones(pix_s.shape[0], dtype=bool)
    first[1:] = pix_s[1:] != pix_s[:-1]
    winner = np.full(out_h * out_w, -1, dtype=np.int64)
    winner[pix_s[first]] = n_s[first]
    winner = winner.reshape(out_h, out_w)
    best = np.full((out_h, out_w), np.inf)
    hit = winner >= 0
    best[hit] = z[winner[hit]]
    rgb_out = np.zeros((out_h, out_w, 3), dtype=np.uint8)
    depth_out = np.zeros((out_h, out_w), dtype=np.uint16)
    rgb_out[hit] = cols[winner[hit]]
    depth_out[hit] = np.clip(np.rint(best[hit]), 0, 65535).astype(np.uint16)
    return rgb_out, depth_out, winner
