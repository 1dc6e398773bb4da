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


def model_flop_per_request(N, P, C, T=2, De=384, Dd=192, ne=12, nd=4):
    """Algorithmic FLOPs of one request: embedding, blocks (linear + attention),
    encoder-to-decoder projection, head on the target time slot."""
    L = T * 256 * C
    f = 2.0 * N * L * De
    f += ne * (24.0 * N * De * De + 4.0 * N * N * De)
    f += 2.0 * N * De * Dd
    f += nd * (24.0 * N * Dd * Dd + 4.0 * N * N * Dd)
    f += 2.0 * P * Dd * 256 * C
    return f


def run_form(precision, reqs, blobs, steps, warmup, log, one_stream=False):
    import torch
    from paper_2604_27441_amd import Recoverer
    from tests.gpu_util import dev, push_refs

    rec = Recoverer(blobs[0], blobs[1], precision=precision, device=0, max_batch_tokens=4 * 10800 + 64,
                    max_batch=8, profile=True, one_stream=one_stream)
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
                p50_ms=pct(50), p99_ms=pct(99), stats=st)


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

    import synth
    t = time.perf_counter()
    reqs = synth.make_batch("c3")
    blobs = synth.make_weights(0)
    log(f"inputs ready ({time.perf_counter() - t:.1f} s)")

    bf = run_form(1, reqs, blobs, args.steps, args.warmup, log, args.one_stream)
    log(f"bf16: {bf['ms_per_step']:.2f} ms/step")
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
        },
        "gpu_time_ms_per_step": {
            "attention": st["attn_ms"] / args.steps, "linear": st["gemm_ms"] / args.steps,
            "other": st["other_ms"] / args.steps, "forward": st["forward_ms"] / args.steps,
        },
        "linear_tflops": st["gemm_flop"] / (st["gemm_ms"] * 1e-3) / 1e12 if st["gemm_ms"] > 0 else 0.0,
    }
    if fp:
        fv = fp["pairs"] / fp["seconds"]
        fst = fp["stats"]
        out["fp32"] = {
            "value": fv, "ms_per_step": fp["ms_per_step"], "p50_ms": fp["p50_ms"], "p99_ms": fp["p99_ms"],
            "steps": args.fp32_steps, "bf16_speedup": value / fv,
            "attn_tflops": fst["attn_flop"] / (fst["attn_ms"] * 1e-3) / 1e12 if fst["attn_ms"] > 0 else 0.0,
            "path_frac_of_fp32_peak": flop_pair * fv / 1e12 / FP32_PEAK_TFLOPS,
        }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(reqs[0], log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
