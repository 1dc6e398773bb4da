"""Write the sampled-output fixtures of the 1280x720 workloads.

Only the seeded generators (synth) and the oracle are called.  He-normal
weights from seed 0, k=5, T=2, 12 + 4 blocks, both modalities.

  c3     tests/golden/c3_720p_samples.json: request 0 of the four-request
         BF16 batch (scene 1003, Gilbert-Elliott loss 20 %, burst 4).
  c3r1   tests/golden/c3_720p_request1_samples.json: request 1 of that batch
         (scene 1004, mask 2004).
  s540   tests/golden/s540_bf16_samples.json: one 960x540 pair (6120 tokens;
         the last patch row is 12 pixels high), 2 + 1 blocks with the perturbed
         seed-3 weights (non-zero biases and gains), Gilbert-Elliott loss 30 %,
         under the BF16-rounding oracle: the serving loop's 540p shape.
  c4fp8  tests/golden/c4_720p_fp8_samples.json: request 0 of the eight-request
         FP8 batch (scene 1007, loss 30 %), under the FP8-rounding oracle whose
         activation scales come from its own calibration pass (per-site absmax
         / 448, exact arithmetic) over the first 8 frames of the seeded
         calibration set at 1280x720 (scenes 10000-10003, two consecutive
         corrupted frames each, loss 30 %, burst 4).

Stored per modality: 2048 seeded sample pixels (1536 lost, 512 received),
the oracle's float output there, the rounding oracle's float output there
(BF16 rounding for c3/c3r1, FP8 rounding for c4fp8), and full-frame error
figures of the rounding oracle against the exact one.

Run: python tests/golden/make_golden.py [c3|c3r1|s540|c4fp8 ...]
(several minutes per 1280x720 forward on 8 cores; c4fp8 runs ten)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
CALIB_FRAMES = 8


def _timed(what, fn):
    t = time.time()
    r = fn()
    print(f"{what} {time.time() - t:.0f} s", flush=True)
    return r


def _samples(req, exact, emu, seed, emu_key, workload, extra=None):
    rng = np.random.default_rng(seed)
    out = {"workload": workload, "generator": "tests/golden/make_golden.py (synth + oracle only)"}
    if extra:
        out.update(extra)
    for mod, key in (("rgb", "mask_rgb"), ("depth", "mask_depth")):
        lost = np.argwhere(req[key] != 0)
        kept = np.argwhere(req[key] == 0)
        pick = np.concatenate([lost[rng.choice(len(lost), 1536, replace=False)],
                               kept[rng.choice(len(kept), 512, replace=False)]])
        ys, xs = pick[:, 0], pick[:, 1]
        ef, qf = exact[mod][1], emu[mod][1]
        lmask = req[key] != 0
        d = qf - ef
        out[mod] = {
            "y": ys.tolist(), "x": xs.tolist(),
            "oracle": np.round(ef[ys, xs], 9).tolist(),
            emu_key: np.round(qf[ys, xs], 9).tolist(),
            emu_key.replace("oracle_", "") + "_vs_oracle_full_frame": {
                "max_abs": float(np.abs(d).max()),
                "rms_lost": float(np.sqrt(np.mean(d[lmask] ** 2))),
                "psnr_db": float(10 * np.log10((1.0 if mod == "rgb" else 65535.0 ** 2) / np.mean(d ** 2)))
                if mod == "rgb" else None,
            },
            "lost_fraction": float(lmask.mean()),
        }
    return out


def _write(path, out):
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"wrote {path} ({os.path.getsize(path)} bytes)")


def c3(index, path, seed):
    req = synth.make_batch("c3")[index]
    blobs = synth.make_weights(0)
    exact = _timed("fp64 oracle", lambda: oracle.recover(req, blobs))
    emu = _timed("bf16-rounding oracle", lambda: oracle.recover(req, blobs, rnd=oracle.Rounding(oracle.bf16_round)))
    wl = (f"1280x720 batch of 4, request {index}: scene {1003 + index}, mask {2003 + index}, G-E loss 20% burst 4, "
          "weights He-normal seed 0, k=5, T=2, 12+4 blocks")
    _write(path, _samples(req, exact, emu, seed, "oracle_bf16_rounding", wl))


def s540(path, seed):
    small = dict(enc_depth=2, dec_depth=1)
    req = synth.make_request(501, 502, 540, 960, loss=("ge", 0.3))
    blobs = synth.make_weights(3, perturb_seed=4, **small)
    exact = _timed("fp64 oracle", lambda: oracle.recover(req, blobs, **small))
    emu = _timed("bf16-rounding oracle", lambda: oracle.recover(req, blobs, rnd=oracle.Rounding(oracle.bf16_round),
                                                                **small))
    wl = ("960x540 pair: scene 501, mask 502, G-E loss 30% burst 4, weights synth.make_weights(3, perturb_seed=4), "
          "k=5, T=2, 2+1 blocks")
    _write(path, _samples(req, exact, emu, seed, "oracle_bf16_rounding", wl))


def c4fp8(path, seed):
    req = synth.make_batch("c4", n=1)[0]
    blobs = synth.make_weights(0)
    calib = synth.make_calibration_set(720, 1280, n=CALIB_FRAMES)
    scales = {}
    for mod in ("rgb", "depth"):
        rec = oracle.AbsMaxRecorder()
        for i, r in enumerate(calib):
            _timed(f"calibration {mod} frame {i}", lambda: oracle.recover(r, blobs, rnd=rec, modalities=(mod,)))
        scales[mod] = rec.scales()
    exact = _timed("fp64 oracle", lambda: oracle.recover(req, blobs))
    emu = {}
    for mod in ("rgb", "depth"):
        emu.update(_timed(f"fp8-rounding oracle {mod}",
                          lambda: oracle.recover(req, blobs, rnd=oracle.FP8Rounding(scales[mod]), modalities=(mod,))))
    wl = ("1280x720 batch of 8, request 0: scene 1007, mask 2007, G-E loss 30% burst 4, weights He-normal seed 0, "
          "k=5, T=2, 12+4 blocks; FP8 E4M3 block products and encoder-to-decoder projection")
    extra = {"calibration": f"synth.make_calibration_set(720, 1280, n={CALIB_FRAMES}): scenes 10000-10003, "
                            "two corrupted frames each, G-E loss 30% burst 4; per-site absmax / 448",
             "scales": scales}
    _write(path, _samples(req, exact, emu, seed, "oracle_fp8_rounding", wl, extra))


def main(argv):
    jobs = argv or ["c3", "c3r1", "s540", "c4fp8"]
    for j in jobs:
        if j == "c3":
            c3(0, os.path.join(HERE, "c3_720p_samples.json"), 424242)
        elif j == "c3r1":
            c3(1, os.path.join(HERE, "c3_720p_request1_samples.json"), 424243)
        elif j == "s540":
            s540(os.path.join(HERE, "s540_bf16_samples.json"), 424245)
        elif j == "c4fp8":
            c4fp8(os.path.join(HERE, "c4_720p_fp8_samples.json"), 424244)
        else:
            raise SystemExit(f"unknown fixture {j}")


if __name__ == "__main__":
    main(sys.argv[1:])
