"""Pins of the metric / loss oracle against closed forms and brute force.

Each check fixes one part of oracle.metrics by something other than its own
formula: SSIM by a per-window double loop with the 2-D Gaussian weights built
directly, and by its values on identical and on constant images; PSNR, MSE
and L1 by constant offsets; TV and the edge loss by ramps and checkerboards.
"""
import math

import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(11)


def _ssim_brute(x, y):
    """Mean SSIM by explicit windows: 2-D weights exp(-(a^2 + b^2) / (2 sigma^2))
    normalised over the 11 x 11 window, moments summed pixel by pixel."""
    r = 5
    a = np.arange(-r, r + 1)
    w2 = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / (2 * 1.5 ** 2))
    w2 /= w2.sum()
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    H, W = x.shape
    vals = []
    for i in range(H - 2 * r):
        for j in range(W - 2 * r):
            px, py = x[i:i + 11, j:j + 11], y[i:i + 11, j:j + 11]
            mx, my = (w2 * px).sum(), (w2 * py).sum()
            vx = (w2 * (px - mx) ** 2).sum()
            vy = (w2 * (py - my) ** 2).sum()
            cxy = (w2 * (px - mx) * (py - my)).sum()
            vals.append((2 * mx * my + c1) * (2 * cxy + c2) / ((mx * mx + my * my + c1) * (vx + vy + c2)))
    return np.array(vals).reshape(H - 2 * r, W - 2 * r)


def test_gaussian_window_is_the_normalised_sigma_1_5_gaussian():
    w = oracle.gaussian_window()
    assert w.shape == (11,) and abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w, w[::-1], rtol=0, atol=0)
    # neighbouring taps differ by exp((2k + 1) / (2 sigma^2)) around the centre
    assert math.isclose(w[5] / w[4], math.exp(1 / 4.5), rel_tol=1e-13)
    assert math.isclose(w[4] / w[3], math.exp(3 / 4.5), rel_tol=1e-13)


@pytest.mark.parametrize("H,W", [(11, 11), (14, 13), (19, 12)])
def test_ssim_map_matches_per_window_brute_force(H, W):
    x = RNG.uniform(0, 1, (H, W))
    y = np.clip(x + 0.2 * RNG.standard_normal((H, W)), 0, 1)
    got = oracle.ssim_map(x, y)
    ref = _ssim_brute(x, y)
    assert got.shape == ref.shape == (H - 10, W - 10)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_ssim_of_identical_frames_is_one_and_symmetric():
    x = RNG.integers(0, 256, (40, 37, 3), dtype=np.uint8)
    y = RNG.integers(0, 256, (40, 37, 3), dtype=np.uint8)
    assert abs(oracle.ssim(x, x) - 1.0) < 1e-12
    assert abs(oracle.ssim(x, y) - oracle.ssim(y, x)) < 1e-14


@pytest.mark.parametrize("a,b", [(0.2, 0.7), (0.0, 0.5), (0.9, 0.9)])
def test_ssim_of_constant_frames_is_the_luminance_term(a, b):
    # zero variances: the contrast-structure factor is C2 / C2
    x, y = np.full((16, 16), a), np.full((16, 16), b)
    c1 = 0.01 ** 2
    assert np.allclose(oracle.ssim_map(x, y), (2 * a * b + c1) / (a * a + b * b + c1), rtol=1e-12, atol=1e-14)


def test_psnr_mse_and_l1_of_a_constant_offset():
    gt = np.full((24, 30, 3), 100, np.uint8)
    pred = np.full((24, 30, 3), 110, np.uint8)
    m = oracle.frame_metrics(pred, gt)
    d = 10 / 255
    assert math.isclose(m["mse"], d * d, rel_tol=1e-13)
    assert math.isclose(m["l1"], d, rel_tol=1e-13)
    assert math.isclose(m["psnr"], 20 * math.log10(25.5), rel_tol=1e-13)
    assert oracle.frame_metrics(gt, gt)["psnr"] == math.inf


def test_total_variation_of_ramps_and_a_checkerboard():
    i, j = np.mgrid[0:20, 0:30].astype(np.float64)
    s = 0.03
    assert math.isclose(oracle.total_variation((s * j)[:, :, None]), s, rel_tol=1e-12)
    assert math.isclose(oracle.total_variation((-s * i)[:, :, None]), s, rel_tol=1e-12)
    cb = np.where((i + j) % 2 == 0, 0.25, -0.25)[:, :, None]
    assert math.isclose(oracle.total_variation(cb), 1.0, rel_tol=1e-12)


def test_edge_loss_of_ramps():
    i, j = np.mgrid[0:20, 0:30].astype(np.float64)
    s = 0.05
    zero = np.zeros_like(i)
    assert oracle.edge_loss((s * j)[:, :, None], zero[:, :, None]) == pytest.approx(s, rel=1e-12)
    # equal gradient magnitudes in different directions cost nothing
    assert oracle.edge_loss((s * j)[:, :, None], (s * i)[:, :, None]) == pytest.approx(0.0, abs=1e-15)
    # a diagonal ramp has |grad| = sqrt(2) s
    assert oracle.edge_loss((s * (i + j))[:, :, None], zero[:, :, None]) == pytest.approx(math.sqrt(2) * s, rel=1e-12)
    x = RNG.uniform(0, 1, (12, 17, 1))
    assert oracle.edge_loss(x, x) == 0.0


def test_depth_is_normalised_by_4000_mm():
    gt = np.full((16, 16), 2000, np.uint16)
    pred = np.full((16, 16), 2400, np.uint16)
    m = oracle.frame_metrics(pred, gt)
    assert math.isclose(m["l1"], 0.1, rel_tol=1e-13)
    assert math.isclose(m["l_depth"], 0.1 * 0.1 + 0.0 + (1 - m["ssim"]), rel_tol=1e-13)
    # constant frames 0.5 vs 0.6: SSIM is the luminance term
    c1 = 0.01 ** 2
    assert math.isclose(m["ssim"], (2 * 0.5 * 0.6 + c1) / (0.25 + 0.36 + c1), rel_tol=1e-12)


def test_l_rgb_is_mse_plus_tv_of_the_prediction():
    """L_RGB = MSE + alpha TV with alpha = 0.01 (Sec. 3.4.2 RGB loss, Sec. 4),
    TV taken on the prediction.  A horizontal ramp a*x against a zero ground
    truth has MSE = a^2 (W-1)(2W-1)/6 (mean of squares of 0..W-1) and TV = a
    (every horizontal step is a, every vertical one 0); swapping the two
    frames keeps the MSE and makes the prediction's TV zero."""
    H, W, a = 12, 17, 0.013
    ramp = np.broadcast_to((a * np.arange(W))[None, :, None], (H, W, 3)).copy()
    zero = np.zeros((H, W, 3))
    mse = a * a * (W - 1) * (2 * W - 1) / 6.0
    m = oracle.frame_metrics(ramp, zero)
    assert math.isclose(m["mse"], mse, rel_tol=1e-12)
    assert math.isclose(m["tv"], a, rel_tol=1e-12)
    assert math.isclose(m["l_rgb"], mse + 0.01 * a, rel_tol=1e-12)
    assert math.isclose(m["l_rgb"] - m["mse"], 0.01 * a, rel_tol=1e-9)
    swapped = oracle.frame_metrics(zero, ramp)
    assert math.isclose(swapped["mse"], mse, rel_tol=1e-12)
    assert swapped["tv"] == 0.0 and math.isclose(swapped["l_rgb"], mse, rel_tol=1e-12)


def test_l_depth_weights_on_flat_frames():
    """L_Depth = 0.1 L1 + L_edge + (1 - SSIM) (Sec. 3.4.2 depth loss, Sec. 4
    weights).  Two flat depth frames at u and v mm: L1 = |u - v| / 4000, no
    gradients so L_edge = 0, and SSIM is the luminance term alone,
    (2ab + C1) / (a^2 + b^2 + C1) with a = u/4000, b = v/4000, C1 = 1e-4."""
    u, v = 1200, 1700
    pred = np.full((20, 24), u, np.uint16)
    gt = np.full((20, 24), v, np.uint16)
    a, b = u / 4000.0, v / 4000.0
    lum = (2 * a * b + 1e-4) / (a * a + b * b + 1e-4)
    m = oracle.frame_metrics(pred, gt)
    assert math.isclose(m["l1"], abs(a - b), rel_tol=1e-12)
    assert m["edge"] == 0.0
    assert math.isclose(m["ssim"], lum, rel_tol=1e-12)
    # 1 - SSIM carries the float64 rounding of the filtered moments (~1e-17 against C2)
    assert math.isclose(m["l_depth"], 0.1 * abs(a - b) + (1.0 - lum), rel_tol=0, abs_tol=1e-12)
