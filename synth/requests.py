"""Seeded recovery requests: k clean reference frames plus one corrupted
target per modality, with its loss mask and frame indices.

The received target carries seeded random bytes at lost pixels (standing in
for decoder artefacts), so a consumer must zero-fill them itself.
"""
import numpy as np

from .scene import scene_frames
from .masks import stripe_mask, gilbert_elliott_masks


def make_request(scene_seed, mask_seed, height, width, k=5, delta=1, t_target=None,
                 loss=("stripes", 0.2), burst=4, separate_masks=False, mask_frame=0):
    """One request for both modalities.

    loss: ("stripes", p) or ("ge", mean_loss).  Refs are frames
    t_target-delta-(k-1) .. t_target-delta (oldest first).  Returns a dict of
    numpy arrays (see keys below).
    """
    H, W = int(height), int(width)
    t5 = int(t_target) if t_target is not None else k + delta + 3
    ref_idx = np.arange(t5 - delta - (k - 1), t5 - delta + 1, dtype=np.int64)
    idx = list(ref_idx) + [t5]
    rgb, depth = scene_frames(scene_seed, H, W, idx)

    def draw(seed):
        if loss[0] == "stripes":
            return stripe_mask(seed, H, W, loss[1])
        if loss[0] == "ge":
            return gilbert_elliott_masks(seed, H, W, mask_frame + 1, loss[1], burst)[mask_frame]
        if loss[0] == "none":
            return np.zeros((H, W), np.uint8)
        if loss[0] == "all":
            return np.ones((H, W), np.uint8)
        raise ValueError(loss)

    m_rgb = draw(mask_seed)
    m_d = draw(mask_seed + 1) if separate_masks else m_rgb.copy()
    junk = np.random.default_rng(mask_seed + 77)
    rgb_t = rgb[k].copy()
    d_t = depth[k].copy()
    lost = m_rgb.astype(bool)
    rgb_t[lost] = junk.integers(0, 256, size=(int(lost.sum()), 3), dtype=np.uint8)
    lost_d = m_d.astype(bool)
    d_t[lost_d] = junk.integers(0, 65536, size=int(lost_d.sum()), dtype=np.uint16)
    return dict(
        height=H, width=W, ref_idx=ref_idx, t_target=t5,
        rgb_refs=np.ascontiguousarray(rgb[:k]), depth_refs=np.ascontiguousarray(depth[:k]),
        rgb=rgb_t, depth=d_t, mask_rgb=m_rgb, mask_depth=m_d,
        rgb_clean=rgb[k], depth_clean=depth[k],
    )


def make_batch(config, n=None):
    """Requests for one of the named workloads.

    c1: 256x192, batch 1, stripes p=0.2       (scene 1001, mask 2008: seed 2001 draws no lost stripe)
    c2: 640x480, batch 1, G-E L=0.1 b=4       (scene 1002, mask 2002)
    c3: 1280x720, batch 4, G-E L=0.2 b=4      (scenes 1003-1006, masks 2003-2006)
    c4: 1280x720, batch 8, G-E L=0.3 b=4      (scenes 1007-1014, masks 2007-2014)
    """
    if config == "c1":
        reqs = [make_request(1001, 2008, 192, 256, loss=("stripes", 0.2))]
    elif config == "c2":
        reqs = [make_request(1002, 2002, 480, 640, loss=("ge", 0.1))]
    elif config == "c3":
        reqs = [make_request(1003 + i, 2003 + i, 720, 1280, loss=("ge", 0.2)) for i in range(4)]
    elif config == "c4":
        reqs = [make_request(1007 + i, 2007 + i, 720, 1280, loss=("ge", 0.3)) for i in range(8)]
    else:
        raise ValueError(config)
    return reqs if n is None else reqs[:n]


def make_calibration_set(height, width, n=32, mean_loss=0.3, scenes=4, k=5, burst=4):
    """n corrupted frames for FP8 calibration: `scenes` seeded scenes (seeds
    10000, 10001, ...), each with k clean references and n / scenes
    consecutive corrupted targets that reuse those references (as the frames
    of a GoP after a loss do), Gilbert-Elliott loss continuing across them."""
    H, W = int(height), int(width)
    per = -(-n // scenes)
    out = []
    for sc in range(scenes):
        ref_idx = np.arange(4, 4 + k, dtype=np.int64)
        targets = list(range(4 + k, 4 + k + per))
        rgb, depth = scene_frames(10000 + sc, H, W, list(ref_idx) + targets)
        mr = gilbert_elliott_masks(10100 + sc, H, W, per, mean_loss, burst)
        md = gilbert_elliott_masks(10200 + sc, H, W, per, mean_loss, burst)
        junk = np.random.default_rng(10300 + sc)
        for i, t in enumerate(targets):
            if len(out) == n:
                break
            rt, dt = rgb[k + i].copy(), depth[k + i].copy()
            lr, ld = mr[i] != 0, md[i] != 0
            rt[lr] = junk.integers(0, 256, size=(int(lr.sum()), 3), dtype=np.uint8)
            dt[ld] = junk.integers(0, 65536, size=int(ld.sum()), dtype=np.uint16)
            out.append(dict(height=H, width=W, ref_idx=ref_idx, t_target=t, scene=sc,
                            rgb_refs=np.ascontiguousarray(rgb[:k]), depth_refs=np.ascontiguousarray(depth[:k]),
                            rgb=rt, depth=dt, mask_rgb=mr[i], mask_depth=md[i],
                            rgb_clean=rgb[k + i], depth_clean=depth[k + i]))
    return out


def make_pretrain_batch(seed, batch, height, width, channels, k=5, mask_p=0.3):
    """Seeded pretraining samples of one modality (Sec. 3.4.2: frames with
    randomly masked pixels): per sample a scene (seed 50000 + 1000 seed + i),
    k clean references, the clean target frame and a per-pixel Bernoulli
    mask (1 = masked, probability mask_p) that the network's input zero-fills.
    channels 3 gives u8 RGB frames, 1 gives u16 depth frames in mm."""
    H, W = int(height), int(width)
    out = []
    for i in range(batch):
        s = 50000 + 1000 * seed + i
        ref_idx = np.arange(4, 4 + k, dtype=np.int64)
        t = 4 + k
        rgb, depth = scene_frames(s, H, W, list(ref_idx) + [t])
        frames = rgb if channels == 3 else depth
        mask = (np.random.default_rng(s + 500).random((H, W)) < mask_p).astype(np.uint8)
        out.append(dict(height=H, width=W, ref_idx=ref_idx, t_target=t, refs=np.ascontiguousarray(frames[:k]),
                        target=np.ascontiguousarray(frames[k]), mask=mask))
    return out
