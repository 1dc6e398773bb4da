"""Write tests/golden/c3_720p_samples.json: sampled outputs of the FP64 oracle
(and of its BF16-rounding mode) on the 1280x720 workload.

Only the seeded generators (synth) and the oracle are called.  The full
network runs on request 0 of the four-request 1280x720 batch (scene 1003,
Gilbert-Elliott loss 20 %, burst 4), both modalities, 12 + 4 blocks,
He-normal weights from seed 0.  Stored per modality: 2048 seeded sample
pixels (1536 lost, 512 received), the oracle's float output there, the
BF16-rounding oracle's float output there, and full-frame error figures of
the BF16-rounding oracle against the exact one.

Run: python tests/golden/make_golden.py   (several minutes on 8 cores)
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_720p_samples.json")


def main():
    req = synth.make_batch("c3", n=1)[0]
    blobs = synth.make_weights(0)
    t = time.time()
    exact = oracle.recover(req, blobs)
    print(f"fp64 oracle {time.time() - t:.0f} s", flush=True)
    t = time.time()
    emu = oracle.recover(req, blobs, rnd=oracle.Rounding(oracle.bf16_round))
    print(f"bf16-rounding oracle {time.time() - t:.0f} s", flush=True)
    rng = np.random.default_rng(424242)
    out = {"workload": "1280x720 batch of 4, request 0: scene 1003, mask 2003, G-E loss 20% burst 4, "
                       "weights He-normal seed 0, k=5, T=2, 12+4 blocks",
           "generator": "tests/golden/make_golden.py (synth + oracle only)"}
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
            "oracle_bf16_rounding": np.round(qf[ys, xs], 9).tolist(),
            "bf16_rounding_vs_oracle_full_frame": {
                "max_abs": float(np.abs(d).max()),
                "rms_lost": float(np.sqrt(np.mean(d[lmask] ** 2))),
                "psnr_db": float(10 * np.log10((1.0 if mod == "rgb" else 65535.0 ** 2) / np.mean(d ** 2)))
                if mod == "rgb" else None,
            },
            "lost_fraction": float(lmask.mean()),
        }
    with open(OUT, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"wrote {OUT} ({os.path.getsize(OUT)} bytes)")


if __name__ == "__main__":
    main()
