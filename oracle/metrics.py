"""FP64 oracle: frame quality metrics and the per-modality training losses.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes: recovered frames are scored by SSIM (Wang et al.) and
PSNR against the originals (Sec. 5.1, metrics); the RGB model is trained on
MSE plus alpha times a total-variation term (Sec. 3.4.2, RGB loss equation)
and the depth model on alpha_r L_recon + alpha_e L_edge + alpha_s L_SSIM, with
L_recon an L1 reconstruction loss, L_SSIM a structural-similarity loss and
L_edge the mean difference of gradient magnitudes between prediction and
ground truth (Sec. 3.4.2, depth loss equation); alpha = 0.01, alpha_r = 0.1,
alpha_e = 1, alpha_s = 1 (Sec. 4, training details).

Readings where the paper is silent: all terms are taken on normalised values
(RGB u8 / 255, depth u16 / 4000 mm), so the data range is 1; SSIM uses the
11 x 11 Gaussian window with sigma 1.5, K1 = 0.01, K2 = 0.03, Gaussian-weighted
(biased) moments, valid positions only, averaged over positions and
channels; PSNR = 10 log10(1 / MSE); TV is anisotropic, the mean absolute
horizontal plus the mean absolute vertical forward difference of the
prediction; L_edge is the mean over pixels with both forward differences of
| |grad pred| - |grad gt| | with |grad| = sqrt(dx^2 + dy^2); L_SSIM = 1 - SSIM;
every mean runs over all channels.
"""
import math

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

SSIM_SIZE = 11
SSIM_SIGMA = 1.5
SSIM_K1 = 0.01
SSIM_K2 = 0.03
ALPHA_TV = 0.01                       # Sec. 4: alpha of the RGB loss
ALPHA_R, ALPHA_E, ALPHA_S = 0.1, 1.0, 1.0  # Sec. 4: depth loss weights


def normalise_frame(frame):
    """u8 -> /255, u16 -> /4000 (mm), float unchanged; always HWC float64."""
    a = np.asarray(frame)
    if a.dtype == np.uint8:
        x = a.astype(np.float64) / 255.0
    elif a.dtype == np.uint16:
        x = a.astype(np.float64) / 4000.0
    else:
        x = a.astype(np.float64)
    return x[:, :, None] if x.ndim == 2 else x


def gaussian_window(size=SSIM_SIZE, sigma=SSIM_SIGMA):
    """1-D Gaussian weights of the SSIM window, normalised to sum 1."""
    k = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    w = np.exp(-k * k / (2.0 * sigma * sigma))
    return w / w.sum()


def gaussian_filter_valid(x, w=None):
    """sum_{a,b} w[a] w[b] x[i+a, j+b] for every window inside the image:
    the 2-D window is the outer product of the 1-D one, applied along rows
    then columns."""
    w = gaussian_window() if w is None else w
    rows = sliding_window_view(x, len(w), axis=1) @ w
    return sliding_window_view(rows, len(w), axis=0) @ w


def ssim_map(x, y, data_range=1.0):
    """Wang et al.'s SSIM at every valid window position of one channel."""
    c1 = (SSIM_K1 * data_range) ** 2
    c2 = (SSIM_K2 * data_range) ** 2
    mx, my = gaussian_filter_valid(x), gaussian_filter_valid(y)
    sxx = gaussian_filter_valid(x * x) - mx * mx
    syy = gaussian_filter_valid(y * y) - my * my
    sxy = gaussian_filter_valid(x * y) - mx * my
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))


def ssim(pred, gt):
    """Mean SSIM over valid positions and channels of normalised HWC frames."""
    p, g = normalise_frame(pred), normalise_frame(gt)
    return float(np.mean([ssim_map(p[:, :, c], g[:, :, c]).mean() for c in range(p.shape[2])]))


def total_variation(x):
    """Anisotropic TV: mean |horizontal forward difference| + mean |vertical one|."""
    return float(np.abs(np.diff(x, axis=1)).mean() + np.abs(np.diff(x, axis=0)).mean())


def edge_loss(p, g):
    """Mean | |grad p| - |grad g| | over pixels with both forward differences."""
    def gmag(x):
        dx = x[:-1, 1:] - x[:-1, :-1]
        dy = x[1:, :-1] - x[:-1, :-1]
        return np.sqrt(dx * dx + dy * dy)
    return float(np.abs(gmag(p) - gmag(g)).mean())


def frame_metrics(pred, gt):
    """All per-frame values the GPU entry reports, from one prediction /
    ground-truth pair (u8 HWC RGB, u16 HW depth, or float HWC / HW)."""
    p, g = normalise_frame(pred), normalise_frame(gt)
    d = p - g
    mse = float(np.mean(d * d))
    l1 = float(np.mean(np.abs(d)))
    tv = total_variation(p)
    edge = edge_loss(p, g)
    s = ssim(pred, gt)
    psnr = math.inf if mse == 0.0 else 10.0 * math.log10(1.0 / mse)
    return {
        "mse": mse, "l1": l1, "tv": tv, "edge": edge, "ssim": s, "psnr": psnr,
        "l_rgb": mse + ALPHA_TV * tv,
        "l_depth": ALPHA_R * l1 + ALPHA_E * edge + ALPHA_S * (1.0 - s),
    }


METRIC_KEYS = ("mse", "l1", "tv", "edge", "ssim", "psnr", "l_rgb", "l_depth")
