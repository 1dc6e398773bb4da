"""Seeded generators: reproducibility, value ranges and loss statistics."""
import numpy as np

import synth


def test_scene_ranges_and_reproducible():
    rgb, d = synth.scene_frames(7, 96, 128, [0, 1, 2])
    assert rgb.dtype == np.uint8 and rgb.shape == (3, 96, 128, 3)
    assert d.dtype == np.uint16 and d.min() >= 500 and d.max() <= 3000
    rgb2, d2 = synth.scene_frames(7, 96, 128, [0, 1, 2])
    assert np.array_equal(rgb, rgb2) and np.array_equal(d, d2)
    assert not np.array_equal(rgb[0], rgb[2])          # spheres move


def test_stripe_mask_rate():
    rates = [synth.stripe_mask(s, 720, 16, 0.2)[::16, 0].mean() for s in range(400)]
    assert abs(np.mean(rates) - 0.2) < 0.01


def test_gilbert_elliott_statistics():
    L, b = 0.3, 4.0
    m = synth.gilbert_elliott_masks(5, 720, 4, 2000, L, b)[:, ::16, 0].reshape(-1)
    assert abs(m.mean() - L) < 0.02
    # mean burst length over runs of lost slices
    edges = np.diff(np.concatenate([[0], m.astype(int), [0]]))
    runs = np.flatnonzero(edges == -1) - np.flatnonzero(edges == 1)
    assert abs(runs.mean() - b) < 0.25
    p_gb, p_bg = synth.ge_params(0.2, 4)
    assert abs(p_gb - 0.0625) < 1e-12 and p_bg == 0.25


def test_partial_last_slice():
    m = synth.stripe_mask(3, 540, 8, 1.0)
    assert m.shape == (540, 8) and m.all()


def test_request_has_junk_at_lost_pixels():
    r = synth.make_request(1, 2, 64, 64, loss=("stripes", 0.5))
    lost = r["mask_rgb"] != 0
    assert lost.any()
    assert not np.array_equal(r["rgb"][lost], r["rgb_clean"][lost])
    assert np.array_equal(r["rgb"][~lost], r["rgb_clean"][~lost])
    assert list(r["ref_idx"]) == [4, 5, 6, 7, 8] and r["t_target"] == 9


def test_c1_has_loss():
    r = synth.make_batch("c1")[0]
    assert 0 < (r["mask_rgb"] != 0).mean() < 1
