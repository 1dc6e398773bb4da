"""Seeded RGB-D scene generator standing in for decoded talking-head frames.

The paper evaluates on face-cropped RGB-D video at 30 fps with limited motion
(Sec. 4 implementation and Sec. 5.1 setup); that dataset is not available, so
this generator produces frames with the same structure: an RGB frame (u8 HWC)
and a depth frame (u16 millimetres) per time step.

Scene: a pinhole camera (fx = fy = W, principal point at the image centre)
looks at three static planes (back wall 2600-3000 mm, floor, side wall) and
two spheres (centre depth 800-2000 mm, radius 150-400 mm) that translate by
1-3 px per frame.  Depth is the z of the nearest hit, clamped to [500, 3000]
mm.  Colour is a flat per-object base colour in [0.1, 0.9]^3 plus three
octaves of Perlin gradient noise (quintic fade, 32 px lattice, amplitude
+-0.1) in object coordinates.
"""
import numpy as np

_LATTICE = 32.0


def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def perlin2d(x, y, seed):
    """Improved gradient noise (Perlin 2002, quintic fade) at float coords.

    x, y: arrays of lattice-unit coordinates.  Returns values in about [-1, 1].
    """
    rng = np.random.default_rng(seed)
    perm = rng.permutation(256)
    perm = np.concatenate([perm, perm])
    ang = rng.uniform(0.0, 2.0 * np.pi, 256)
    gx, gy = np.cos(ang), np.sin(ang)
    xi = np.floor(x).astype(np.int64)
    yi = np.floor(y).astype(np.int64)
    xf, yf = x - xi, y - yi
    xi &= 255
    yi &= 255

    def grad(ix, iy, dx, dy):
        h = perm[perm[ix] + iy]
        return gx[h] * dx + gy[h] * dy

    n00 = grad(xi, yi, xf, yf)
    n10 = grad((xi + 1) & 255, yi, xf - 1.0, yf)
    n01 = grad(xi, (yi + 1) & 255, xf, yf - 1.0)
    n11 = grad((xi + 1) & 255, (yi + 1) & 255, xf - 1.0, yf - 1.0)
    u, v = _fade(xf), _fade(yf)
    nx0 = n00 + u * (n10 - n00)
    nx1 = n01 + u * (n11 - n01)
    return (nx0 + v * (nx1 - nx0)) * np.sqrt(2.0)


def _texture(u, v, seed):
    """Three octaves of gradient noise scaled to about +-0.1."""
    out = np.zeros_like(u)
    amp, freq, norm = 1.0, 1.0, 0.0
    for o in range(3):
        out += amp * perlin2d(u * freq / _LATTICE, v * freq / _LATTICE, seed + 7919 * o)
        norm += amp
        amp *= 0.5
        freq *= 2.0
    return 0.1 * np.clip(out / norm, -1.0, 1.0)


def _scene_params(seed):
    rng = np.random.default_rng(seed)
    p = {}
    p["back_z"] = rng.uniform(2600.0, 3000.0)
    p["floor_y"] = rng.uniform(600.0, 900.0)          # mm below the optical axis
    p["side_x"] = rng.uniform(-1400.0, -900.0)        # mm left of the axis
    p["colors"] = rng.uniform(0.1, 0.9, size=(5, 3))
    sph = []
    for _ in range(2):
        cz = rng.uniform(800.0, 2000.0)
        r = rng.uniform(150.0, 400.0)
        cu = rng.uniform(0.3, 0.7)                    # centre as a fraction of W
        cv = rng.uniform(0.3, 0.7)                    # centre as a fraction of H
        speed = rng.uniform(1.0, 3.0)
        ang = rng.uniform(0.0, 2.0 * np.pi)
        sph.append((cz, r, cu, cv, speed * np.cos(ang), speed * np.sin(ang)))
    p["spheres"] = sph
    p["tex_seed"] = int(rng.integers(0, 2**31 - 1))
    return p


def scene_frames(seed, height, width, frame_indices):
    """Render frames of one seeded scene.

    Returns (rgb u8 [F, H, W, 3], depth u16 [F, H, W]) for the given integer
    frame indices (spheres move linearly with the index).
    """
    p = _scene_params(seed)
    H, W = int(height), int(width)
    f = float(W)
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    vv, uu = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    dx = (uu - cx) / f
    dy = (vv - cy) / f
    inf = np.inf
    F = len(frame_indices)
    rgb = np.empty((F, H, W, 3), np.uint8)
    depth = np.empty((F, H, W), np.uint16)
    # static planes: z along each ray (ray = (dx, dy, 1) * z)
    z_back = np.full((H, W), p["back_z"])
    with np.errstate(divide="ignore", invalid="ignore"):
        z_floor = np.where(dy > 1e-9, p["floor_y"] / dy, inf)
        z_side = np.where(dx < -1e-9, p["side_x"] / dx, inf)
    plane_z = np.stack([z_back, z_floor, z_side])
    plane_id = np.argmin(plane_z, axis=0)
    plane_best = np.min(plane_z, axis=0)
    # texture coordinates on each plane: image coords on the back wall,
    # (u, distance-like v) on the floor and (v, distance-like u) on the side wall
    floor_v = 400.0 * np.minimum(1.0 / np.maximum(dy, 1e-3), 50.0)
    side_u = 400.0 * np.minimum(1.0 / np.maximum(-dx, 1e-3), 50.0)
    plane_tu = np.choose(plane_id, [uu, uu, vv])
    plane_tv = np.choose(plane_id, [vv, floor_v, side_u])
    plane_noise = None
    for fi, t in enumerate(frame_indices):
        z = plane_best.copy()
        obj = plane_id.copy()
        tu = plane_tu.copy()
        tv = plane_tv.copy()
        for si, (cz, r, cu, cv, vu, vvel) in enumerate(p["spheres"]):
            su = cu * W + vu * t
            sv = cv * H + vvel * t
            C = np.array([(su - cx) / f * cz, (sv - cy) / f * cz, cz])
            # ray d = (dx, dy, 1); solve |z d - C|^2 = r^2 for z
            a = dx * dx + dy * dy + 1.0
            b = -2.0 * (dx * C[0] + dy * C[1] + C[2])
            c = C @ C - r * r
            disc = b * b - 4.0 * a * c
            hit = disc >= 0.0
            zs = np.where(hit, (-b - np.sqrt(np.where(hit, disc, 0.0))) / (2.0 * a), inf)
            closer = zs < z
            z = np.where(closer, zs, z)
            obj = np.where(closer, 3 + si, obj)
            tu = np.where(closer, uu - su, tu)
            tv = np.where(closer, vv - sv, tv)
        base = p["colors"][obj]
        # the planes are static: their texture is computed once per call and
        # only sphere pixels are textured per frame (same values either way)
        if plane_noise is None:
            plane_noise = _texture(plane_tu, plane_tv, p["tex_seed"])
        noise = plane_noise.copy()
        on_sphere = obj >= 3
        if on_sphere.any():
            noise[on_sphere] = _texture(tu[on_sphere], tv[on_sphere], p["tex_seed"])
        col = np.clip(base + noise[..., None], 0.0, 1.0)
        rgb[fi] = np.rint(col * 255.0).astype(np.uint8)
        depth[fi] = np.rint(np.clip(z, 500.0, 3000.0)).astype(np.uint16)
    return rgb, depth
