"""Helpers for the GPU tests: drive the C ABI with torch device buffers."""
import numpy as np
import torch

import oracle


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def push_refs(rec, stream, req, device_ptrs=True, n_ref=None):
    """Submit a request's clean reference frames (oldest first) as clean frames."""
    H, W = req["height"], req["width"]
    refs = range(len(req["ref_idx"])) if n_ref is None else range(len(req["ref_idx"]) - n_ref, len(req["ref_idx"]))
    tickets = []
    for i in refs:
        rgb, d = req["rgb_refs"][i], req["depth_refs"][i]
        if device_ptrs:
            rgb, d = dev(rgb), dev(d)
        tickets.append(rec.submit(stream, int(req["ref_idx"][i]), W, H, rgb=rgb, depth=d, device_ptrs=device_ptrs))
    got = rec.wait(tickets)
    assert all(c.status == 0 for c in got.values()), got


def recover(rec, items, device_ptrs=True, hold=True):
    """Submit corrupted targets [(stream, req)] together; returns per item a dict
    with u8/u16 and float outputs (numpy) and the completion."""
    outs, tickets = [], []
    for n, (stream, req) in enumerate(items):
        H, W = req["height"], req["width"]
        o = dict(rgb=torch.zeros((H, W, 3), dtype=torch.uint8, device="cuda"),
                 depth=torch.zeros((H, W), dtype=torch.int16, device="cuda"),
                 rgb_f=torch.zeros((H, W, 3), dtype=torch.float32, device="cuda"),
                 depth_f=torch.zeros((H, W), dtype=torch.float32, device="cuda"))
        if device_ptrs:
            ins = [dev(req["rgb"]), dev(req["mask_rgb"]), dev(req["depth"]), dev(req["mask_depth"])]
            outs_ptr = (o["rgb"], o["depth"], o["rgb_f"], o["depth_f"])
        else:
            ins = [req["rgb"], req["mask_rgb"], req["depth"], req["mask_depth"]]
            o = {k: v.cpu().numpy() for k, v in o.items()}
            outs_ptr = (o["rgb"], o["depth"], o["rgb_f"], o["depth_f"])
        t = rec.submit(stream, int(req["t_target"]), W, H, rgb=ins[0], mask_rgb=ins[1], depth=ins[2],
                       mask_depth=ins[3], rgb_out=outs_ptr[0], depth_out=outs_ptr[1], rgb_out_f32=outs_ptr[2],
                       depth_out_f32=outs_ptr[3], device_ptrs=device_ptrs, hold=hold and n + 1 < len(items))
        tickets.append(t)
        outs.append((o, ins))
    got = rec.wait(tickets)
    res = []
    for t, (o, _) in zip(tickets, outs):
        if isinstance(o["rgb"], torch.Tensor):
            o = {k: v.cpu().numpy() for k, v in o.items()}
        o["depth"] = o["depth"].view(np.uint16)
        o["completion"] = got[t]
        res.append(o)
    return res


def psnr(a, b, peak=1.0):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10 * np.log10(peak * peak / mse)


def compare(req, gpu, ref):
    """Error figures of one GPU result against oracle outputs {mod: (pred, out_f, out_i)}."""
    lost_r = req["mask_rgb"] != 0
    lost_d = req["mask_depth"] != 0
    er = gpu["rgb_f"].astype(np.float64) - ref["rgb"][1]
    ed = gpu["depth_f"].astype(np.float64) - ref["depth"][1]
    return dict(
        rgb_psnr=psnr(gpu["rgb_f"], ref["rgb"][1]),
        rgb_psnr_lost=psnr(gpu["rgb_f"][lost_r], ref["rgb"][1][lost_r]) if lost_r.any() else float("inf"),
        rgb_maxabs=float(np.abs(er).max()),
        depth_maxabs=float(np.abs(ed).max()),
        depth_rms_lost=float(np.sqrt(np.mean(ed[lost_d] ** 2))) if lost_d.any() else 0.0,
        depth_p99=float(np.percentile(np.abs(ed[lost_d]), 99)) if lost_d.any() else 0.0,
    )


def check_received_and_codes(req, gpu):
    """Received pixels are copied bit-exactly; lost pixels' integer codes are
    the half-to-even rounding of the GPU's own float output (float32)."""
    keep_r = req["mask_rgb"] == 0
    keep_d = req["mask_depth"] == 0
    assert np.array_equal(gpu["rgb"][keep_r], req["rgb"][keep_r])
    assert np.array_equal(gpu["depth"][keep_d], req["depth"][keep_d])
    assert np.array_equal(gpu["rgb_f"][keep_r], (req["rgb"][keep_r].astype(np.float32) / np.float32(255)))
    assert np.array_equal(gpu["depth_f"][keep_d], req["depth"][keep_d].astype(np.float32))
    lr, ld = ~keep_r, ~keep_d
    q_r = np.rint(np.float32(255) * gpu["rgb_f"][lr].astype(np.float32)).astype(np.uint8)
    assert np.array_equal(gpu["rgb"][lr], q_r)
    assert np.array_equal(gpu["depth"][ld], np.rint(gpu["depth_f"][ld]).astype(np.uint16))
    assert gpu["rgb_f"].min() >= 0 and gpu["rgb_f"].max() <= 1
    assert gpu["depth_f"].min() >= 0 and gpu["depth_f"].max() <= 65535
