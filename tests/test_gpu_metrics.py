"""revo_op_frame_metrics against the FP64 oracle (oracle.metrics): SSIM, PSNR,
MSE, L1, TV, edge loss, L_RGB and L_Depth (Sec. 3.4.2, Sec. 4, Sec. 5.1).

Tolerances, from the kernels' arithmetic: pixel terms are float32 per
element, summed in float32 within a workgroup and in float64 across
workgroups, so MSE, L1, TV and the edge loss are good to about 1e-6
relative (asserted at 1e-5).  SSIM takes float32 Gaussian moments: E[x^2] -
mu^2 carries about 2^-23 E[x^2] <= 1.2e-7 of rounding, which against C2 =
9e-4 moves one window's SSIM by at most about 3e-4 (asserted as the bound on
the frame mean, which is typically far below it).  PSNR follows MSE:
10 / ln 10 times its relative error."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

U8, U16, F32 = 0, 1, 2
RNG = np.random.default_rng(505)
TOL_REL = 1e-5
TOL_SSIM = 3e-4


def _lib():
    import paper_2604_27441_amd as pkg
    return pkg.lib


def _run(kind, pred, gt):
    """pred, gt: numpy [B, H, W(, C)] of the kind's dtype -> [B, 8] float64."""
    p, g = np.ascontiguousarray(pred), np.ascontiguousarray(gt)
    assert p.shape == g.shape and p.dtype == g.dtype
    B, H, W = p.shape[:3]
    C = p.shape[3] if p.ndim == 4 else 1
    pd, gd = torch.from_numpy(p).cuda(), torch.from_numpy(g).cuda()
    out = torch.full((B, 8), float("nan"), dtype=torch.float64, device="cuda")
    rc = _lib().revo_op_frame_metrics(kind, pd.data_ptr(), gd.data_ptr(), B, H, W, C, out.data_ptr(), None)
    assert rc == 0
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check(got, pred, gt):
    for b in range(pred.shape[0]):
        ref = oracle.frame_metrics(pred[b], gt[b])
        row = dict(zip(oracle.METRIC_KEYS, got[b]))
        for k in ("mse", "l1", "tv", "edge", "l_rgb"):
            assert abs(row[k] - ref[k]) <= TOL_REL * abs(ref[k]) + 1e-12, (b, k, row[k], ref[k])
        assert abs(row["ssim"] - ref["ssim"]) <= TOL_SSIM, (b, row["ssim"], ref["ssim"])
        assert abs(row["l_depth"] - ref["l_depth"]) <= TOL_SSIM + TOL_REL * abs(ref["l_depth"]), (b, row, ref)
        if math.isinf(ref["psnr"]):
            assert math.isinf(row["psnr"]) and row["psnr"] > 0
        else:
            assert abs(row["psnr"] - ref["psnr"]) <= 10 / math.log(10) * TOL_REL + 1e-9, (b, row["psnr"], ref["psnr"])


def _noisy(gt, sigma, lo, hi, dtype):
    return np.clip(gt.astype(np.float64) + sigma * RNG.standard_normal(gt.shape), lo, hi).round().astype(dtype)


@pytest.mark.parametrize("B,H,W", [(2, 48, 64), (1, 11, 11), (3, 77, 100)])
def test_rgb_u8(B, H, W):
    gt = RNG.integers(0, 256, (B, H, W, 3), dtype=np.uint8)
    pred = _noisy(gt, 12.0, 0, 255, np.uint8)
    _check(_run(U8, pred, gt), pred, gt)


@pytest.mark.parametrize("B,H,W", [(3, 77, 100), (1, 130, 21)])
def test_depth_u16(B, H, W):
    gt = RNG.integers(300, 4000, (B, H, W), dtype=np.uint16)
    pred = _noisy(gt, 40.0, 0, 65535, np.uint16)
    _check(_run(U16, pred, gt), pred, gt)


@pytest.mark.parametrize("C", [1, 3])
def test_float_frames(C):
    gt = RNG.uniform(-0.5, 1.5, (2, 37, 45, C)).astype(np.float32)
    pred = (gt + 0.05 * RNG.standard_normal(gt.shape)).astype(np.float32)
    _check(_run(F32, pred, gt), pred, gt)


def test_identical_frames():
    gt = RNG.integers(0, 256, (2, 40, 52, 3), dtype=np.uint8)
    got = _run(U8, gt, gt)
    for row in got:
        m = dict(zip(oracle.METRIC_KEYS, row))
        assert m["mse"] == 0.0 and m["l1"] == 0.0 and m["edge"] == 0.0
        assert abs(m["ssim"] - 1.0) < 1e-6 and math.isinf(m["psnr"])


def test_repeated_calls_start_from_zero():
    gt = RNG.integers(0, 256, (1, 33, 35, 3), dtype=np.uint8)
    pred = _noisy(gt, 20.0, 0, 255, np.uint8)
    a, b = _run(U8, pred, gt), _run(U8, pred, gt)
    assert np.allclose(a, b, rtol=1e-12, atol=0)


def test_rejects_frames_smaller_than_the_window():
    x = torch.zeros((1, 10, 40, 3), dtype=torch.uint8, device="cuda")
    out = torch.zeros((1, 8), dtype=torch.float64, device="cuda")
    assert _lib().revo_op_frame_metrics(U8, x.data_ptr(), x.data_ptr(), 1, 10, 40, 3, out.data_ptr(), None) != 0
    assert _lib().revo_op_frame_metrics(U16, x.data_ptr(), x.data_ptr(), 1, 40, 12, 3, out.data_ptr(), None) != 0


def test_720p_scene_frames():
    """Full 1280x720 frames with the synthetic scenes' structure: a frame
    against its successor, and a copy with a lost region replaced by noise."""
    rgb, depth = synth.scene_frames(1003, 720, 1280, [4, 5])
    lost = synth.gilbert_elliott_masks(2003, 720, 1280, 1, 0.2, 4)[0] != 0
    rp = rgb[1].copy()
    rp[lost] = RNG.integers(0, 256, (int(lost.sum()), 3), dtype=np.uint8)
    pred = np.stack([rgb[0], rp]); gt = np.stack([rgb[1], rgb[1]])
    _check(_run(U8, pred, gt), pred, gt)
    dp = depth[1].copy()
    dp[lost] = RNG.integers(0, 65536, int(lost.sum()), dtype=np.uint16)
    pred = np.stack([depth[0], dp]); gt = np.stack([depth[1], depth[1]])
    _check(_run(U16, pred, gt), pred, gt)
