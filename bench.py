#!/usr/bin/env python3
"""Recovered RGB-D frame pairs per second at 1280x720 on one MI355X.

Workload: four 1280x720 conference streams, each with five clean reference
frames (RGB u8 + depth u16 mm) resident on the GPU and one corrupted frame
pair with a Gilbert-Elliott slice-loss mask (mean 20 %, bursts of 4 slices).
One step recovers the four corrupted pairs through the C ABI
(revo_recover_submit x 4, batched, then revo_recover_poll): tubelet
embedding, 12 encoder + 4 decoder blocks over all 10 800 tokens of each
request, target-frame head and mask composite, for the RGB and the depth
model.  The BF16 form is the headline; the FP32 form is timed beside it.

Prints one JSON line.  Also reports the roofline of the dominant kernel
(flash attention: algorithmic FLOPs / HIP-event time of its launches) and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "recovered RGB-D frames/sec at 1280x720 (BF16 vs FP32) + p50/p99 latency"
BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 MFMA
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 matrix
HBM_PEAK_GBPS = 8000.0      # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (packed FMA; unpacked code reaches half)
# frame metrics, per pixel and channel, separable SSIM: 5 moments x 11 taps
# along rows and along columns (220 FMA = 220 FLOP x 2), 3 products, about 15
# for the SSIM quotient and 12 for the pixel terms
METRIC_FLOP_PER_SAMPLE = 2 * 110 + 3 + 15 + 12


def model_flop_per_request(N, P, C, T=2, De=384, Dd=192, ne=12, nd=4):
    """Algorithmic FLOPs of one request: embedding, blocks (linear + attention),
    encoder-to-decoder projection, head on the target time slot.  The last
    decoder block only needs the target tubelet's P queries (K and V of all
    N tokens, Q, projection and MLP of P rows, attention P x N): the path
    prunes that block's attention to them, and counts only what is needed."""
    L = T * 256 * C
    f = 2.0 * N * L * De
    f += ne * (24.0 * N * De * De + 4.0 * N * N * De)
    f += 2.0 * N * De * Dd
    f += (nd - 1) * (24.0 * N * Dd * Dd + 4.0 * N * N * Dd)
    f += 4.0 * N * Dd * Dd + 20.0 * P * Dd * Dd + 4.0 * N * P * Dd
    f += 2.0 * P * Dd * 256 * C
    return f


def run_form(precision, reqs, blobs, steps, warmup, log, one_stream=False, profile="attention"):
    import torch
    from paper_2604_27441_amd import Recoverer
    from tests.gpu_util import dev, push_refs

    rec = Recoverer(blobs[0], blobs[1], precision=precision, device=0, max_batch_tokens=4 * 10800 + 64,
                    max_batch=8, profile=profile, one_stream=one_stream)
    for s, r in enumerate(reqs):
        push_refs(rec, s, r)
    H, W = reqs[0]["height"], reqs[0]["width"]
    ins = [(dev(r["rgb"]), dev(r["mask_rgb"]), dev(r["depth"]), dev(r["mask_depth"])) for r in reqs]
    outs = [(torch.empty((H, W, 3), dtype=torch.uint8, device="cuda"), torch.empty((H, W), dtype=torch.int16, device="cuda"))
            for _ in reqs]
    torch.cuda.synchronize()

    def step():
        tickets = []
        for i, r in enumerate(reqs):
            t = rec.submit(i, int(r["t_target"]), W, H, rgb=ins[i][0], mask_rgb=ins[i][1], depth=ins[i][2],
                           mask_depth=ins[i][3], rgb_out=outs[i][0], depth_out=outs[i][1], device_ptrs=True,
                           hold=i + 1 < len(reqs))
            tickets.append(t)
        got = rec.wait(tickets)
        bad = [c for c in got.values() if c.status != 0]
        if bad:
            raise RuntimeError(f"recovery failed: {bad}")
        return got

    for i in range(warmup):
        step()
        log(f"warmup step {i + 1}/{warmup} done")
    rec.stats(reset=True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        got = step()
        lat += [(c.done_ns - c.submit_ns) * 1e-6 for c in got.values()]
        if (i + 1) % max(1, steps // 4) == 0:
            log(f"timed step {i + 1}/{steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = rec.stats()
    rec.close()
    lat.sort()
    pct = lambda p: lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))]
    return dict(seconds=dt, pairs=steps * len(reqs), ms_per_step=1e3 * dt / steps,
                p50_ms=pct(50), p99_ms=pct(99), stats=st, outputs=outs)


def render_bench(reqs, outs, log, iters=20):
    """The receiver's rendering step on the recovered frames of the timed run:
    revo_op_unproject then revo_op_render_view into a view turned 5 degrees
    and moved 10 cm (Sec. 2, Sec. 5), timed with HIP events on the launching
    stream.  Algorithmic traffic per source pixel: depth 2 B + point 16 B
    written (unprojection); z-buffer clear 8 B, point read 16 B, one 8-byte
    atomic, resolve 8 + 3 + 3 + 2 B (rendering at the source size) = 66 B."""
    import math
    import numpy as np
    import torch
    from paper_2604_27441_amd import lib
    B, H, W = len(reqs), reqs[0]["height"], reqs[0]["width"]
    rgb = torch.stack([o[0] for o in outs])
    depth = torch.stack([o[1] for o in outs])
    assert rgb.shape == (B, H, W, 3) and depth.shape == (B, H, W) and rgb.is_contiguous() and depth.is_contiguous()
    pts = torch.empty((B, H, W, 4), dtype=torch.float32, device="cuda")
    zbuf = torch.empty((B, H, W), dtype=torch.int64, device="cuda")
    co = torch.empty((B, H, W, 3), dtype=torch.uint8, device="cuda")
    do = torch.empty((B, H, W), dtype=torch.int16, device="cuda")
    intr = np.array([W, W, (W - 1) / 2, (H - 1) / 2], dtype=np.float32)   # the synthetic scenes' camera
    a = math.radians(5.0)
    pose = np.array([[math.cos(a), 0, math.sin(a), 100.0], [0, 1, 0, 0.0], [-math.sin(a), 0, math.cos(a), 0.0]],
                    dtype=np.float32)

    def call():
        r1 = lib.revo_op_unproject(depth.data_ptr(), B, H, W, intr.ctypes.data, pts.data_ptr(), None)
        r2 = lib.revo_op_render_view(pts.data_ptr(), rgb.data_ptr(), B, H, W, pose.ctypes.data, intr.ctypes.data,
                                     H, W, zbuf.data_ptr(), co.data_ptr(), do.data_ptr(), None)
        return r1 or r2
    for _ in range(3):
        assert call() == 0
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    nbytes = 66 * B * H * W
    gbs = nbytes / (ms * 1e-3) / 1e9
    filled = float((zbuf != -1).float().mean())
    log(f"render: {ms * 1e3:.1f} us for {B} frames (unproject + new view), {gbs:.0f} GB/s algorithmic; "
        f"{100 * filled:.1f} % of target pixels hit")
    return {"ms_per_call": ms, "frames": B, "bytes_per_call": nbytes,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBPS},
            "target_pixels_hit": filled, "view": "yaw 5 degrees, 100 mm sideways, same intrinsics"}


LINEAR_SHAPES = [(43200, 1152, 384, 0), (43200, 384, 384, 1), (43200, 1536, 384, 2), (43200, 384, 1536, 1),
                 (43200, 576, 192, 0), (43200, 192, 768, 1)]


def linear_shapes_bench(log, iters=10):
    """The encoder and decoder products at 43200 tokens (BF16) through
    revo_op_linear, one after another, timed with HIP events: the workload of
    the GEMM counter profiles."""
    import torch
    from paper_2604_27441_amd import lib
    rows = []
    for (M, N, K, epi) in LINEAR_SHAPES:
        torch.manual_seed(0)
        x = torch.randn(M, K, device="cuda").to(torch.bfloat16)
        w = (torch.randn(N, K, device="cuda") * 0.05).to(torch.bfloat16)
        b = torch.zeros(N, device="cuda")
        out = torch.zeros(M, N, device="cuda", dtype=torch.float32 if epi == 1 else torch.bfloat16)
        assert x.shape == (M, K) and w.shape == (N, K) and out.shape == (M, N)
        call = lambda: lib.revo_op_linear(1, epi, x.data_ptr(), w.data_ptr(), b.data_ptr(), out.data_ptr(), M, N, K, None)
        assert call() == 0
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(iters):
            call()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / iters * 1e3
        rows.append({"M": M, "N": N, "K": K, "epilogue": ["store", "residual", "gelu"][epi], "us": us,
                     "tflops": 2 * M * N * K / (us * 1e-6) / 1e12})
        log(f"linear {M}x{N}x{K} {rows[-1]['epilogue']}: {us:.1f} us, {rows[-1]['tflops']:.0f} TFLOP/s")
    return rows


def attention_only_bench(log, iters=10):
    """revo_op_attention_noalloc (BF16) on one 1280x720 encoder layer of the 4-request
    batch laid out as 24 heads of one 10800-token request (the same work as
    4 requests x 6 heads), timed with HIP events: the workload of the
    attention counter profiles."""
    import torch
    from paper_2604_27441_amd import lib
    heads, ntok = 24, 10800
    ld = (ntok + 64 + 15) // 16 * 16
    torch.manual_seed(0)
    q = (torch.randn(heads, ld, 64, device="cuda") * 0.2).to(torch.bfloat16)
    k = torch.randn(heads, ld, 64, device="cuda").to(torch.bfloat16)
    vt = torch.randn(heads, 64, ld, device="cuda").to(torch.bfloat16)
    o = torch.zeros(ntok, heads * 64, device="cuda", dtype=torch.bfloat16)
    assert q.shape == (heads, ld, 64) and vt.shape == (heads, 64, ld) and ld >= ntok + 64 and ld % 16 == 0
    # the entry point without allocations: its request descriptor and work
    # list are written by a small kernel on the stream, so nothing on the host
    # (no allocation, copy or synchronisation) sits between the timed launches
    call = lambda: lib.revo_op_attention_noalloc(1, q.data_ptr(), k.data_ptr(), vt.data_ptr(), o.data_ptr(), heads, ntok,
                                                 ld, None)
    assert call() == 0
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        call()
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / iters * 1e3
    tf = 4.0 * ntok * ntok * 64 * heads / (us * 1e-6) / 1e12
    log(f"attention 24 heads x {ntok} tokens: {us:.1f} us per call (descriptor kernel included), {tf:.0f} TFLOP/s")
    return {"heads": heads, "tokens": ntok, "us": us, "tflops": tf}


def metrics_bench(reqs, outs, log, iters=20):
    """Quality metrics and training losses of the recovered frames against the
    clean targets through revo_op_frame_metrics (SSIM, PSNR, L_RGB, L_Depth;
    Sec. 3.4.2, Sec. 5.1), timed with HIP events on the launching stream.
    Algorithmic traffic: each prediction and ground-truth byte read once."""
    import numpy as np
    import torch
    from paper_2604_27441_amd import lib
    B, H, W = len(reqs), reqs[0]["height"], reqs[0]["width"]
    res = {}
    for name, kind, C, pred, gt in (
            ("rgb", 0, 3, torch.stack([o[0] for o in outs]),
             torch.from_numpy(np.stack([r["rgb_clean"] for r in reqs])).cuda()),
            ("depth", 1, 1, torch.stack([o[1] for o in outs]),
             torch.from_numpy(np.stack([r["depth_clean"] for r in reqs]).view(np.int16)).cuda())):
        assert pred.shape == gt.shape and pred.is_contiguous() and gt.is_contiguous()
        assert pred.numel() == B * H * W * C and pred.element_size() == gt.element_size()
        o = torch.empty((B, 8), dtype=torch.float64, device="cuda")
        call = lambda: lib.revo_op_frame_metrics(kind, pred.data_ptr(), gt.data_ptr(), B, H, W, C, o.data_ptr(), None)
        for _ in range(3):
            assert call() == 0
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(iters):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / iters
        nbytes = 2 * pred.numel() * pred.element_size()
        flop = METRIC_FLOP_PER_SAMPLE * B * H * W * C
        v = o.cpu().numpy().mean(axis=0)
        gbs = nbytes / (ms * 1e-3) / 1e9
        tf = flop / (ms * 1e-3) / 1e12
        res[name] = {"ms_per_call": ms, "frames": B, "bytes_per_call": nbytes, "achieved_GBps": gbs,
                     "hbm_frac": gbs / HBM_PEAK_GBPS, "flop_per_call": flop,
                     "roofline": {"bound": "alu", "achieved": tf, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": tf / FP32_VECTOR_PEAK_TFLOPS},
                     "ssim": float(v[4]), "psnr_db": float(v[5]), "loss": float(v[6] if name == "rgb" else v[7])}
        log(f"frame metrics {name}: {ms * 1e3:.1f} us per call of {B} frames, {gbs:.0f} GB/s; "
            f"SSIM {v[4]:.4f}, PSNR {v[5]:.2f} dB")
    res["note"] = ("recovered frames of the timed BF16 run against the clean targets; the weights are random, so "
                   "the quality values only exercise the path; loss = L_RGB for rgb, L_Depth for depth")
    return res


SERVE_RES = [(480, 640)] * 16 + [(540, 960)] * 16 + [(720, 1280)] * 32   # 1 : 1 : 2


def serve_bench(blobs, streams, seconds, warm_seconds, cap_tokens, log, seed=0):
    """Serving loop: `streams` conference streams with Poisson arrivals at
    30 fps each, mixed resolutions, per-stream Gilbert-Elliott loss (mean
    U[0.05, 0.40], bursts of 4 slices, independent RGB and depth chains), a
    deadline of arrival + 1/30 s, BF16 graph launches, deadline shedding.
    A frame of a modality with no lost slice is a clean reference update."""
    import numpy as np
    import torch

    import synth
    from paper_2604_27441_amd import Recoverer

    rng = np.random.default_rng(40000 + seed)
    res = [SERVE_RES[(i * len(SERVE_RES)) // streams] for i in range(streams)]
    # shared content per resolution: 5 references + 1 target frame pair
    content = {}
    for (H, W) in sorted(set(res)):
        rgb, dep = synth.scene_frames(20000 + H, H, W, list(range(6)))
        content[(H, W)] = [(torch.from_numpy(rgb[i]).cuda(), torch.from_numpy(dep[i]).cuda()) for i in range(6)]
    # per-stream loss chains over 15 frames (cycled), uploaded as device masks
    F = 15
    masks = []
    for i in range(streams):
        H, W = res[i]
        L = rng.uniform(0.05, 0.40)
        mr = synth.gilbert_elliott_masks(30000 + 2 * i, H, W, F, L, 4)
        md = synth.gilbert_elliott_masks(30001 + 2 * i, H, W, F, L, 4)
        masks.append([(torch.from_numpy(mr[f]).cuda() if mr[f].any() else None,
                       torch.from_numpy(md[f]).cuda() if md[f].any() else None) for f in range(F)])
    outs = {r: (torch.empty((r[0], r[1], 3), dtype=torch.uint8, device="cuda"),
                torch.empty(r, dtype=torch.int16, device="cuda")) for r in set(res)}
    rec = Recoverer(blobs[0], blobs[1], precision=1, device=0, max_batch_tokens=cap_tokens, max_batch=16,
                    max_streams=streams, shed=True, graphs=True, fps=30.0)
    t_ids = []
    for i in range(streams):
        H, W = res[i]
        for f in range(5):
            t_ids.append(rec.submit(i, f, W, H, rgb=content[(H, W)][f][0], depth=content[(H, W)][f][1],
                                    device_ptrs=True))
    rec.wait(t_ids)
    # Poisson arrival schedule
    total = warm_seconds + seconds
    arrivals = []
    for i in range(streams):
        t = rng.exponential(1 / 30.0)
        while t < total:
            arrivals.append((t, i))
            t += rng.exponential(1 / 30.0)
    arrivals.sort()
    frame_no = [5] * streams
    info = {}
    lat, done = [], []
    t0 = time.perf_counter()
    t0_ns = time.clock_gettime_ns(time.CLOCK_MONOTONIC)
    pending = 0

    def drain(timeout_us):
        nonlocal pending
        for c in rec.poll(256, timeout_us):
            pending -= 1
            done.append((c, info.pop(c.ticket)))

    for (ta, i) in arrivals:
        while True:
            now = time.perf_counter() - t0
            if now >= ta:
                break
            drain(int(min(ta - now, 0.002) * 1e6))
        H, W = res[i]
        f = frame_no[i]
        frame_no[i] += 1
        mr, md = masks[i][f % F]
        arr_ns = t0_ns + int(ta * 1e9)
        t = rec.submit(i, f, W, H, rgb=content[(H, W)][5][0], mask_rgb=mr, depth=content[(H, W)][5][1],
                       mask_depth=md, rgb_out=outs[(H, W)][0], depth_out=outs[(H, W)][1], device_ptrs=True,
                       deadline_ns=arr_ns + int(1e9 / 30.0))
        if t is None:  # queue full: the frame is dropped like a shed one
            continue
        pending += 1
        info[t] = (ta, (H, W), mr is not None or md is not None, arr_ns)
        drain(0)
    while pending > 0:
        drain(1_000_000)
    rec.close()
    # measured window: arrivals after the warm-up
    served = [(c, x) for c, x in done if x[0] >= warm_seconds and x[2]]
    n_rec = len(served)
    ok = [(c, x) for c, x in served if c.status == 0]
    shed = sum(1 for c, _ in served if c.status == 1)
    lat = sorted((c.done_ns - x[3]) * 1e-6 for c, x in ok)
    pct = lambda v, p: v[min(len(v) - 1, int(round(p / 100 * (len(v) - 1))))] if v else None
    per_res = {}
    for r in sorted(set(res)):
        lr = sorted((c.done_ns - x[3]) * 1e-6 for c, x in ok if x[1] == r)
        nr = sum(1 for _, x in served if x[1] == r)
        per_res[f"{r[1]}x{r[0]}"] = {"served_per_s": len(lr) / seconds, "offered_per_s": nr / seconds,
                                     "p50_ms": pct(lr, 50), "p99_ms": pct(lr, 99)}
    # per stream: served fraction of its recoveries, the longest run of shed
    # recoveries, and whether some window of 30 frames (one GoP) that holds
    # recoveries has none served (the stream frozen on its last good frame)
    by_stream = {}
    for c, x in served:
        by_stream.setdefault(c.stream_id, []).append((c.frame_index, c.status == 0))
    fracs, runs, frozen = [], [], 0
    for sid, seq in by_stream.items():
        seq.sort()
        fracs.append(sum(hit for _, hit in seq) / len(seq))
        run = best = 0
        for _, hit in seq:
            run = 0 if hit else run + 1
            best = max(best, run)
        runs.append(best)
        good = [f for f, hit in seq if hit]
        for f, _ in seq:
            # the window of 30 frames ending at this recovery
            if not any(f - 29 <= g <= f for g in good) and seq[0][0] <= f - 29:
                frozen += 1
                break
    out = {
        "streams": streams, "seconds": seconds, "offered_recoveries_per_s": n_rec / seconds,
        "served_pairs_per_s": len(ok) / seconds, "shed_fraction": shed / max(1, n_rec),
        "failed": sum(1 for c, _ in served if c.status == 2),
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
        "deadline_met_fraction": (sum(1 for v in lat if v <= 1000 / 30.0) / len(lat)) if lat else None,
        "per_resolution": per_res, "batch_token_cap": cap_tokens,
        "fairness": {
            "min_stream_served_fraction": min(fracs) if fracs else None,
            "max_shed_run": max(runs) if runs else None,
            "streams_frozen_for_a_gop": frozen,
            "note": "per stream over the measured window: fraction of its recoveries served, longest run of shed "
                    "recoveries, and streams with a 30-frame window of recoveries none of which was served",
        },
    }
    log(f"serving {streams} streams: {out['served_pairs_per_s']:.1f} pairs/s served, shed {100 * out['shed_fraction']:.1f} %,"
        f" p50 {out['p50_ms']} ms, p99 {out['p99_ms']} ms, max shed run {out['fairness']['max_shed_run']}")
    return out


def _time_batches(rec, reqs, base_stream, steps, warmup):
    """Time `steps` submissions of the whole batch `reqs` (device pointers)."""
    import torch
    from tests.gpu_util import dev
    H, W = reqs[0]["height"], reqs[0]["width"]
    ins = [(dev(r["rgb"]), dev(r["mask_rgb"]), dev(r["depth"]), dev(r["mask_depth"])) for r in reqs]
    outs = [(torch.empty((H, W, 3), dtype=torch.uint8, device="cuda"),
             torch.empty((H, W), dtype=torch.int16, device="cuda")) for _ in reqs]

    def step():
        ts = [rec.submit(base_stream + i, int(r["t_target"]), W, H, rgb=ins[i][0], mask_rgb=ins[i][1],
                         depth=ins[i][2], mask_depth=ins[i][3], rgb_out=outs[i][0], depth_out=outs[i][1],
                         device_ptrs=True, hold=i + 1 < len(reqs)) for i, r in enumerate(reqs)]
        got = rec.wait(ts)
        assert all(c.status == 0 for c in got.values()), got
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def fp8_bench(blobs, c3, steps, log):
    """FP8-E4M3 form at 1280x720, batch 8, Gilbert-Elliott loss 30 %:
    calibration on 32 seeded frames through the ABI, throughput, error
    against the BF16 form on the same batch, and against the FP64 oracle on
    the sampled 1280x720 outputs of tests/golden (request 0 of the batch-4
    workload)."""
    import numpy as np

    import synth
    from paper_2604_27441_amd import Recoverer
    from tests.gpu_util import psnr, push_refs, recover

    t = time.perf_counter()
    c4 = synth.make_batch("c4")
    calib = synth.make_calibration_set(720, 1280, 32, 0.3)
    log(f"fp8 inputs ready ({time.perf_counter() - t:.1f} s)")
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "c3_720p_samples.json")))
    res = {}
    outs = {}
    for prec, name in ((2, "fp8"), (1, "bf16")):
        rec = Recoverer(blobs[0], blobs[1], precision=prec, device=0, max_batch_tokens=8 * 10816,
                        max_batch=8, max_streams=32, profile="attention" if prec == 2 else False)
        for s, r in enumerate(c4):
            push_refs(rec, s, r)
        for s, r in enumerate(c3):
            push_refs(rec, 8 + s, r)
        if prec == 2:
            for sc in range(4):
                push_refs(rec, 12 + sc, next(x for x in calib if x["scene"] == sc))
            t = time.perf_counter()
            rec.calibrate(1)
            for i in range(0, len(calib), 8):
                recover(rec, [(12 + x["scene"], x) for x in calib[i:i + 8]])
            rec.calibrate(0)
            res["calibration_seconds"] = time.perf_counter() - t
            rec.stats(reset=True)
            dt = _time_batches(rec, c4, 0, steps, 1)
            st = rec.stats()
            res.update(value=len(c4) * steps / dt, ms_per_step=1e3 * dt / steps, steps=steps,
                       attn_tflops=st["attn_flop"] / (st["attn_ms"] * 1e-3) / 1e12 if st["attn_ms"] else None)
        outs[name] = (recover(rec, list(enumerate(c4))), recover(rec, [(8, c3[0])])[0])
        rec.close()
    # FP8 against BF16 on the batch of 8
    a, b = outs["fp8"][0], outs["bf16"][0]
    er = np.concatenate([(x["rgb_f"].astype(np.float64) - y["rgb_f"]).ravel() for x, y in zip(a, b)])
    ed = np.concatenate([(x["depth_f"].astype(np.float64) - y["depth_f"]).ravel() for x, y in zip(a, b)])
    res["vs_bf16"] = {"rgb_psnr_db": float(10 * np.log10(1.0 / max(np.mean(er ** 2), 1e-30))),
                      "depth_maxabs_mm": float(np.abs(ed).max()),
                      "depth_rms_mm": float(np.sqrt(np.mean(ed ** 2)))}
    # FP8 and BF16 against FP64 on the sampled 1280x720 outputs (lost pixels)
    for name in ("fp8", "bf16"):
        o = outs[name][1]
        g = {}
        for mod, key in (("rgb", "rgb_f"), ("depth", "depth_f")):
            y, x = np.array(golden[mod]["y"][:1536]), np.array(golden[mod]["x"][:1536])
            ref = np.array(golden[mod]["oracle"][:1536], np.float64)
            g[mod] = o[key][y, x].astype(np.float64) - ref
        res[f"{name}_vs_fp64_samples"] = {"rgb_psnr_db": psnr(g["rgb"], 0.0),
                                          "rgb_maxabs": float(np.abs(g["rgb"]).max()),
                                          "depth_rms_mm": float(np.sqrt(np.mean(g["depth"] ** 2))),
                                          "depth_maxabs_mm": float(np.abs(g["depth"]).max())}
    log(f"fp8: {res['value']:.1f} pairs/s at batch 8; vs bf16 {res['vs_bf16']}; vs fp64 {res['fp8_vs_fp64_samples']}")
    return res


def sweep_kt(log, reps=3):
    """Per-frame recovery latency at 1280x720 (one RGB-D pair, BF16) over
    k in 1..7 clean references and tubelet T in {1, 2, 3}: the shape of the
    paper's latency-versus-k and k x T ablations (App. B.3), here with
    seeded weights.  k + 1 frames are padded up to whole tubelets by
    repeating the oldest reference (at most 9 frames: k = 7 at T = 3)."""
    import synth
    from paper_2604_27441_amd import Recoverer
    from tests.gpu_util import push_refs, recover
    rows = []
    for T in (1, 2, 3):
        blobs = synth.make_weights(0, tubelet=T)
        for k in range(1, 8):
            nframes = -(-(k + 1) // T) * T
            if nframes > 9:
                continue
            req = synth.make_request(1003, 2003, 720, 1280, k=k, loss=("ge", 0.2))
            rec = Recoverer(blobs[0], blobs[1], precision=1, device=0, k=k, tubelet=T,
                            max_batch_tokens=(nframes // T) * 3600 + 64, max_batch=1)
            push_refs(rec, 0, req)
            recover(rec, [(0, req)])
            lat = []
            for _ in range(reps):
                c = recover(rec, [(0, req)])[0]["completion"]
                lat.append((c.done_ns - c.submit_ns) * 1e-6)
            rec.close()
            lat.sort()
            rows.append({"k": k, "T": T, "tokens": (nframes // T) * 3600, "median_ms": lat[len(lat) // 2]})
            log(f"k={k} T={T}: {rows[-1]['median_ms']:.2f} ms per RGB-D pair")
    return rows


def attention_traffic():
    """HBM bytes per attention launch from the committed counter record, or
    None when the kernel source changed since the counters were taken."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", "attn_bf16_720p_b4_traffic.json")
    try:
        rec = json.load(open(rec_path))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return rec["bytes_per_launch"]


def train_flop_per_sample(N, P, C, T=2, De=384, Dd=192, ne=12, nd=4):
    """Algorithmic FLOPs of one pretraining sample: the forward pass over all
    tokens (no pruning: every block's queries are needed for the gradient of
    the next), and the backward pass: two products (dX and dW) per forward
    product, and five N x N x 64 products per head in attention (the scores
    again, dP, dV, dK, dQ) against the forward's two."""
    L = T * 256 * C
    lin = 2.0 * N * L * De + ne * 24.0 * N * De * De + 2.0 * N * De * Dd + nd * 24.0 * N * Dd * Dd + 2.0 * P * Dd * 256 * C
    att = ne * 4.0 * N * N * De + nd * 4.0 * N * N * Dd
    return 3.0 * lin + 3.5 * att


def train_bench(log, steps=5, warmup=1, batch=8, height=192, width=256):
    """Pretraining step (Sec. 3.4.2 / Sec. 4): FP32 forward, L_RGB, backward of
    every layer and Adam on seeded 256x192 frames with 30 % of the pixels
    masked, batch 8, one trainer per modality, 12 + 4 blocks."""
    import numpy as np
    import torch

    import synth
    from paper_2604_27441_amd import Trainer

    out = {"workload": f"{width}x{height} pretraining, batch {batch}, 12+4 blocks, FP32, L_RGB = MSE + 0.01 TV, "
                       "Adam lr 2e-4, per-pixel masks p = 0.3",
           "data": "synthetic"}
    blobs = synth.make_weights(0)
    gy, gx = -(-height // 16), -(-width // 16)
    P = gy * gx
    N = 3 * P
    total_flop, total_s = 0.0, 0.0
    data = {}
    for C, name in ((3, "rgb"), (1, "depth")):
        batches = []
        for i in range(warmup + steps):
            sm = synth.make_pretrain_batch(100 + i, batch, height, width, C)
            refs = np.stack([x["refs"] for x in sm])
            tgt = np.stack([x["target"] for x in sm])
            if C == 1:
                refs, tgt = refs.view(np.int16), tgt.view(np.int16)
            batches.append((torch.from_numpy(np.ascontiguousarray(refs)).cuda(),
                            torch.from_numpy(np.ascontiguousarray(tgt)).cuda(),
                            torch.from_numpy(np.ascontiguousarray(np.stack([x["mask"] for x in sm]))).cuda(),
                            np.stack([x["ref_idx"] for x in sm]), np.array([x["t_target"] for x in sm])))
        data[name] = batches
        with Trainer(blobs[0 if C == 3 else 1], C, batch, height, width) as tr:
            losses = [tr.step(*batches[i]) for i in range(warmup)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(steps):
                losses.append(tr.step(*batches[warmup + i]))
            dt = time.perf_counter() - t0
        flop = train_flop_per_sample(N, P, C) * batch
        total_flop += flop * steps
        total_s += dt
        out[name] = {"ms_per_step": 1e3 * dt / steps, "samples_per_s": batch * steps / dt,
                     "tflops": flop * steps / dt / 1e12, "losses": losses}
        log(f"train {name}: {1e3 * dt / steps:.2f} ms per step of {batch}, {flop * steps / dt / 1e12:.1f} TFLOP/s, "
            f"losses {['%.4f' % v for v in losses]}")
    out["flop_per_sample"] = {"rgb": train_flop_per_sample(N, P, 3), "depth": train_flop_per_sample(N, P, 1)}
    out["tflops"] = total_flop / total_s / 1e12
    out["frac_of_fp32_peak"] = out["tflops"] / FP32_PEAK_TFLOPS

    # both models at once: each trainer stepped by its own host thread (the
    # library call releases the interpreter lock), so their kernels share the
    # GPU; the same batches and starting weights as above
    import threading
    trs = [Trainer(blobs[0], 3, batch, height, width), Trainer(blobs[1], 1, batch, height, width)]
    try:
        names = ("rgb", "depth")
        for tr, name in zip(trs, names):
            for i in range(warmup):
                tr.step(*data[name][i])
        torch.cuda.synchronize()
        errors = []

        def run(tr, name):
            try:
                for i in range(steps):
                    tr.step(*data[name][warmup + i])
            except Exception as e:  # re-raised below on the main thread
                errors.append(e)

        threads = [threading.Thread(target=run, args=(tr, name)) for tr, name in zip(trs, names)]
        t0 = time.perf_counter()
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        dt = time.perf_counter() - t0
        if errors:
            raise errors[0]
    finally:
        for tr in trs:
            tr.close()
    flop = (train_flop_per_sample(N, P, 3) + train_flop_per_sample(N, P, 1)) * batch
    out["both_models_concurrent"] = {"ms_per_step_pair": 1e3 * dt / steps, "samples_per_s": 2 * batch * steps / dt,
                                     "tflops": flop * steps / dt / 1e12}
    log(f"train rgb + depth at once: {1e3 * dt / steps:.2f} ms per pair of steps, {flop * steps / dt / 1e12:.1f} TFLOP/s")
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def small_configs_bench(blobs, log, steps=20, oracle_runs=True):
    """The plain FP32 form at 256x192 (stripes, p = 0.2) and at 640x480
    (Gilbert-Elliott loss 10, 30 and 50 %, burst 4), batch 1: frames/s and
    p50 latency through the ABI, and at 256x192 and 640x480 / 30 % the error
    against the FP64 oracle (the 10 % draw of that mask seed loses no slice), whose own seconds per pair (both modalities,
    full network) are timed beside it."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import oracle
    import synth
    from tests.gpu_util import compare

    threads = sum(i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas") or os.cpu_count()
    cases = [("256x192", synth.make_batch("c1")[0], True)]
    for L in (0.1, 0.3, 0.5):
        cases.append((f"640x480 loss {int(L * 100)}%", synth.make_request(1002, 2002, 480, 640, loss=("ge", L)),
                      L == 0.3))
    rows = {}
    for name, req, with_oracle in cases:
        r = run_form(0, [req], blobs, steps, 3, lambda m: None, profile=False)
        o = r.pop("outputs")
        row = {"frames_per_s": r["pairs"] / r["seconds"], "ms_per_pair": r["ms_per_step"], "p50_ms": r["p50_ms"],
               "p99_ms": r["p99_ms"], "lost_fraction_rgb": float(np.mean(req["mask_rgb"] != 0))}
        if with_oracle and oracle_runs:
            t = time.perf_counter()
            ref = oracle.recover(req, blobs)
            row["oracle_seconds_per_pair"] = time.perf_counter() - t
            row["oracle_threads"] = int(threads)
            # one more recovery with float outputs for the error figures
            from paper_2604_27441_amd import Recoverer
            from tests.gpu_util import push_refs, recover
            with Recoverer(blobs[0], blobs[1], precision=0, device=0, max_batch_tokens=10800 + 64) as rec:
                push_refs(rec, 0, req)
                got = recover(rec, [(0, req)])[0]
            e = compare(req, got, ref)
            row["fp32_vs_fp64"] = {"rgb_psnr_db": e["rgb_psnr"], "rgb_maxabs": e["rgb_maxabs"],
                                   "depth_maxabs_mm": e["depth_maxabs"], "depth_rms_lost_mm": e["depth_rms_lost"]}
        rows[name] = row
        log(f"fp32 {name}: {row['frames_per_s']:.1f} pairs/s"
            + (f", oracle {row['oracle_seconds_per_pair']:.1f} s per pair, error {row['fp32_vs_fp64']}"
               if "oracle_seconds_per_pair" in row else ""))
    return rows


def cpu_baseline(req, log):
    """FP64 oracle on a bounded sample of one 1280x720 request.

    Sample: the full RGB forward pass with 1 encoder + 1 decoder block, plus
    one more encoder block and one more decoder block timed on their own;
    a pair takes about 2 x (t_11 + 11 t_enc + 3 t_dec) (depth costs the same
    up to the small embedding and head)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import oracle
    import synth

    blobs1 = synth.make_weights(0, enc_depth=1, dec_depth=1)
    arch1 = oracle.Arch(channels=3, enc_depth=1, dec_depth=1)
    p1 = oracle.unpack_weights(blobs1[0], arch1)
    t = time.perf_counter()
    oracle.forward(req["rgb_refs"], req["ref_idx"], req["rgb"], req["t_target"], req["mask_rgb"], p1, arch1)
    t11 = time.perf_counter() - t
    log(f"cpu baseline: 1+1-block forward {t11:.1f} s")
    N = 3 * 45 * 80
    rng = np.random.default_rng(0)
    t = time.perf_counter()
    oracle.transformer_block(rng.standard_normal((N, 384)), p1, "enc0.", 6)
    t_enc = time.perf_counter() - t
    t = time.perf_counter()
    oracle.transformer_block(rng.standard_normal((N, 192)), p1, "dec0.", 3)
    t_dec = time.perf_counter() - t
    pair_s = 2.0 * (t11 + 11 * t_enc + 3 * t_dec)
    threads = sum(i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas") or os.cpu_count()
    log(f"cpu baseline: enc block {t_enc:.1f} s, dec block {t_dec:.1f} s -> {pair_s:.0f} s per pair")
    return {
        "value": 1.0 / pair_s, "unit": "RGB-D frame pairs/s", "cores": int(threads), "kind": "oracle",
        "sample": ("FP64 NumPy oracle on one 1280x720 request: RGB forward with 1 encoder + 1 decoder block "
                   f"({t11:.1f} s) plus one encoder block ({t_enc:.1f} s) and one decoder block ({t_dec:.1f} s) "
                   "timed alone; pair = 2 x (t11 + 11 enc + 3 dec)"),
        "seconds_per_pair": pair_s,
        "cpu_model": cpu_model(),
        "logical_cpus": os.cpu_count(),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp32-steps", type=int, default=3)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--one-stream", action="store_true",
                    help="run RGB and depth one after the other on one stream (clean per-kernel times)")
    ap.add_argument("--no-sweep-kt", action="store_true", help="skip the latency sweep over k = 1..7, T = 1..3")
    ap.add_argument("--no-small", action="store_true", help="skip the FP32 256x192 and 640x480 lines")
    ap.add_argument("--no-fp8", action="store_true", help="skip the FP8 form (batch 8)")
    ap.add_argument("--fp8-steps", type=int, default=5)
    ap.add_argument("--serve-seconds", type=float, default=6.0, help="measured serving window (0 = skip)")
    ap.add_argument("--serve-warmup", type=float, default=2.0)
    ap.add_argument("--serve-streams", type=int, default=64)
    ap.add_argument("--serve-cap", type=int, default=21600, help="tokens per batch per modality when serving")
    ap.add_argument("--serve-sweep-seconds", type=float, default=3.0,
                    help="measured window of each point of the 4, 8, 16, 32-stream sweep (0 = no sweep)")
    ap.add_argument("--attention-only", action="store_true",
                    help="only time revo_op_attention on one encoder layer's work (attention profiles)")
    ap.add_argument("--linear-shapes", action="store_true",
                    help="only time the encoder/decoder products through revo_op_linear (GEMM profiles)")
    ap.add_argument("--no-train", action="store_true", help="skip the pretraining step")
    ap.add_argument("--train-only", action="store_true", help="only time the pretraining step (profiles)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB (a kernel of known traffic "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the recovery path has no multi-GPU form here "
              "(streams would shard across GPUs by stream id with no collective)", file=sys.stderr)
        sys.exit(2)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.copy_calibration > 0:
        import torch
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {n} bytes read + {n} bytes written")
        del src, dst

    if args.attention_only:
        print(json.dumps({"attention": attention_only_bench(log), "dtype": "bf16", "data": "synthetic"}), flush=True)
        return
    if args.train_only:
        print(json.dumps({"train": train_bench(log), "dtype": "fp32", "data": "synthetic"}), flush=True)
        return
    if args.linear_shapes:
        print(json.dumps({"linear_shapes": linear_shapes_bench(log), "dtype": "bf16", "data": "synthetic"}), flush=True)
        return

    import synth
    t = time.perf_counter()
    reqs = synth.make_batch("c3")
    blobs = synth.make_weights(0)
    log(f"inputs ready ({time.perf_counter() - t:.1f} s)")

    # timed region: HIP events around the attention launches only (the
    # roofline kernel); a short untimed pass with every kernel timed, on one
    # stream so that kernels do not overlap, gives the per-class split
    bf = run_form(1, reqs, blobs, args.steps, args.warmup, log, args.one_stream)
    log(f"bf16: {bf['ms_per_step']:.2f} ms/step")
    bf_outs = bf.pop("outputs")
    fm = metrics_bench(reqs, bf_outs, log)
    rv = render_bench(reqs, bf_outs, log)
    split = run_form(1, reqs, blobs, 3, 1, log, True, profile=True)
    sst = split["stats"]
    fp = None
    if not args.no_fp32:
        fp = run_form(0, reqs, blobs, args.fp32_steps, 1, log, args.one_stream)
        log(f"fp32: {fp['ms_per_step']:.2f} ms/step")

    N, P = 10800, 3600
    flop_pair = model_flop_per_request(N, P, 3) + model_flop_per_request(N, P, 1)
    value = bf["pairs"] / bf["seconds"]
    st = bf["stats"]
    attn_tflops = st["attn_flop"] / (st["attn_ms"] * 1e-3) / 1e12 if st["attn_ms"] > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "RGB-D frame pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": bf["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": "1280x720 RGB-D loss recovery, 4 streams per step, BF16 MFMA with FP32 accumulation",
            "batch": len(reqs), "height": 720, "width": 1280, "tokens_per_request": N, "k": 5, "tubelet": 2,
            "encoder": "384x12 (6 heads)", "decoder": "192x4 (3 heads)", "patch": 16,
            "loss": "Gilbert-Elliott, mean 20%, burst 4 slices", "weights": "He-normal, seed 0",
            "parallelism": "single GPU",
            "streams": 1 if args.one_stream else 2,
        },
        "p50_ms": bf["p50_ms"],
        "p99_ms": bf["p99_ms"],
        "latency_note": "submit-to-poll of each request in a batch of 4",
        "flop_per_pair": flop_pair,
        "path_tflops": flop_pair * value / 1e12,
        "path_frac_of_bf16_peak": flop_pair * value / 1e12 / BF16_PEAK_TFLOPS,
        "roofline": {
            "kernel": "attn_kernel<OpBF16> (flash attention)",
            "bound": "mfma",
            "achieved": attn_tflops,
            "peak": BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": attn_tflops / BF16_PEAK_TFLOPS,
            "traffic": attention_traffic(),
            "traffic_unit": "bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, copy-calibrated)",
            "launches": st["attn_launches"],
            "avg_launch_ms": st["attn_ms"] / max(1, st["attn_launches"]),
            "flop_per_launch": st["attn_flop"] / max(1, st["attn_launches"]),
            "one_stream": {
                "achieved": sst["attn_flop"] / (sst["attn_ms"] * 1e-3) / 1e12 if sst["attn_ms"] > 0 else 0.0,
                "frac": sst["attn_flop"] / (sst["attn_ms"] * 1e-3) / 1e12 / BF16_PEAK_TFLOPS if sst["attn_ms"] > 0 else 0.0,
                "note": "the same kernel in the split pass (one stream, no overlap); in the timed region the RGB "
                        "and depth networks share the GPU, so one attention launch often runs beside another "
                        "and its span includes that sharing",
            },
        },
        "gpu_time_ms_per_step": {
            "note": "every kernel timed, one stream, 3 steps outside the timed region",
            "attention": sst["attn_ms"] / 3, "linear": sst["gemm_ms"] / 3,
            "other": sst["other_ms"] / 3, "forward": sst["forward_ms"] / 3,
        },
        "linear_tflops": sst["gemm_flop"] / (sst["gemm_ms"] * 1e-3) / 1e12 if sst["gemm_ms"] > 0 else 0.0,
    }
    out["frame_metrics"] = fm
    out["render"] = rv
    if fp:
        fv = fp["pairs"] / fp["seconds"]
        fst = fp["stats"]
        out["fp32"] = {
            "value": fv, "ms_per_step": fp["ms_per_step"], "p50_ms": fp["p50_ms"], "p99_ms": fp["p99_ms"],
            "steps": args.fp32_steps, "bf16_speedup": value / fv,
            "attn_tflops": fst["attn_flop"] / (fst["attn_ms"] * 1e-3) / 1e12 if fst["attn_ms"] > 0 else 0.0,
            "path_frac_of_fp32_peak": flop_pair * fv / 1e12 / FP32_PEAK_TFLOPS,
        }
    if not args.no_fp8:
        out["fp8"] = fp8_bench(blobs, reqs, args.fp8_steps, log)
    if not args.no_sweep_kt:
        out["k_t_sweep"] = sweep_kt(log)
    if not args.no_train:
        out["train"] = train_bench(log)
    if not args.no_small:
        out["fp32_small"] = small_configs_bench(blobs, log, oracle_runs=not args.no_cpu_baseline)
    if args.serve_seconds > 0:
        out["serving"] = serve_bench(blobs, args.serve_streams, args.serve_seconds, args.serve_warmup,
                                     args.serve_cap, log)
        if args.serve_sweep_seconds > 0:
            # the stream-count knee: where shedding starts
            sweep = [serve_bench(blobs, n, args.serve_sweep_seconds, 1.0, args.serve_cap, log) for n in (4, 8, 16, 32)]
            out["serving_sweep"] = [
                {k: v[k] for k in ("streams", "offered_recoveries_per_s", "served_pairs_per_s", "shed_fraction",
                                   "p50_ms", "p99_ms", "fairness")} for v in sweep + [out["serving"]]]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(reqs[0], log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
