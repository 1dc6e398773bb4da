"""The largest accepted frame, 4096 x 4096 (196 608 tokens per request at
T = 2, 1536 query tiles per head): one recovery per form runs every kernel
at its largest offsets.  The oracle cannot run at this size, so the checks
are properties that hold at any size: received pixels come back exact and
lost ones are the rounding of the GPU's own float output; the BF16 form
stays within the BF16 budget of the FP32 form (whose parity with the oracle
the smaller tests establish); a 4097-pixel frame is refused.  The frames are
a 512 x 512 synthetic request tiled 8 x 8 (content does not matter here)."""
import numpy as np
import pytest

import synth
from tests.gpu_util import check_received_and_codes, psnr, push_refs, recover

pytestmark = pytest.mark.gpu

SMALL = dict(enc_depth=2, dec_depth=1)
SIDE = 4096


def _tiled():
    base = synth.make_request(71, 72, 512, 512, loss=("stripes", 0.5))
    rep = SIDE // 512
    t2 = lambda a: np.ascontiguousarray(np.tile(a, (rep, rep) + (1,) * (a.ndim - 2)))
    t3 = lambda a: np.ascontiguousarray(np.tile(a, (1, rep, rep) + (1,) * (a.ndim - 3)))
    req = dict(base)
    req.update(height=SIDE, width=SIDE, rgb=t2(base["rgb"]), depth=t2(base["depth"]), mask_rgb=t2(base["mask_rgb"]),
               mask_depth=t2(base["mask_depth"]), rgb_refs=t3(base["rgb_refs"]), depth_refs=t3(base["depth_refs"]))
    assert req["rgb"].shape == (SIDE, SIDE, 3) and req["rgb_refs"].shape[1:] == (SIDE, SIDE, 3)
    assert req["depth_refs"].shape[1:] == (SIDE, SIDE) and req["mask_rgb"].any() and req["mask_depth"].any()
    return req


def _run(prec, req, blobs):
    from paper_2604_27441_amd import Recoverer
    tokens = 3 * (SIDE // 16) ** 2
    with Recoverer(blobs[0], blobs[1], precision=prec, max_batch_tokens=tokens + 64, max_batch=1, max_streams=2,
                   **SMALL) as rec:
        push_refs(rec, 0, req)
        out = recover(rec, [(0, req)])[0]
    assert out["completion"].status == 0, out["completion"]
    return out


def test_largest_frame_bf16_against_fp32():
    req = _tiled()
    blobs = synth.make_weights(3, perturb_seed=4, **SMALL)
    f32 = _run(0, req, blobs)
    b16 = _run(1, req, blobs)
    for out in (f32, b16):
        check_received_and_codes(req, out)
        assert np.isfinite(out["rgb_f"]).all() and np.isfinite(out["depth_f"]).all()
    lr, ld = req["mask_rgb"] != 0, req["mask_depth"] != 0
    p = psnr(b16["rgb_f"][lr], f32["rgb_f"][lr])
    d = b16["depth_f"][ld].astype(np.float64) - f32["depth_f"][ld]
    rms = float(np.sqrt(np.mean(d * d)))
    print(f"4096x4096 bf16 vs fp32: lost-pixel rgb psnr {p:.1f} dB, depth rms {rms:.1f} mm, max {np.abs(d).max():.0f} mm")
    # the BF16 form against FP32 at 1280x720 and 12 + 4 blocks: 47 dB and 25 mm rms (against FP64)
    assert p >= 40.0 and rms <= 100.0


def test_frames_past_the_largest_are_refused():
    from paper_2604_27441_amd import Recoverer
    from paper_2604_27441_amd._lib import RevoError
    import torch
    blobs = synth.make_weights(3, perturb_seed=4, **SMALL)
    with Recoverer(blobs[0], blobs[1], precision=1, max_batch_tokens=4096, **SMALL) as rec:
        rgb = torch.zeros((16, SIDE + 1, 3), dtype=torch.uint8, device="cuda")
        with pytest.raises(RevoError):
            rec.submit(0, 1, SIDE + 1, 16, rgb=rgb, device_ptrs=True)
