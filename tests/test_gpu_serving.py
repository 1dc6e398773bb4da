"""Serving semantics of the C ABI on the GPU: admission by HBM budget
(REVO_ENOMEM at create, REVO_EAGAIN at submit), deadline shedding (the
display repeats its last frame, Sec. 3.3) with the shed request's clean
modality still entering the reference ring (Sec. 3.4.1 reference reuse),
REVO_ENOREF before any clean frame, ordering after the caller's stream, and
reference frames dropped by a resolution change staying intact for a batch
already in flight."""
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import dev, push_refs, recover

pytestmark = pytest.mark.gpu

FP32 = 0
SMALL = dict(enc_depth=2, dec_depth=1)
H, W = 48, 64


def _rec(blobs, **kw):
    from paper_2604_27441_amd import Recoverer
    kw.setdefault("max_batch_tokens", 4096)
    kw.setdefault("precision", FP32)
    return Recoverer(blobs[0], blobs[1], **SMALL, **kw)


def _r4k(n):
    return (n + 4095) & ~4095


def _outs(h=H, w=W):
    return dict(rgb=torch.zeros((h, w, 3), dtype=torch.uint8, device="cuda"),
                depth=torch.zeros((h, w), dtype=torch.int16, device="cuda"),
                rgb_f=torch.zeros((h, w, 3), dtype=torch.float32, device="cuda"),
                depth_f=torch.zeros((h, w), dtype=torch.float32, device="cuda"))


def _submit(rec, stream, r, o, hold=False, deadline_ns=0, rgb_lost=True, depth_lost=True):
    ins = [dev(r["rgb"]), dev(r["mask_rgb"]), dev(r["depth"]), dev(r["mask_depth"])]
    return rec.submit(stream, int(r["t_target"]), r["width"], r["height"], rgb=ins[0],
                      mask_rgb=ins[1] if rgb_lost else None, depth=ins[2], mask_depth=ins[3] if depth_lost else None,
                      rgb_out=o["rgb"], depth_out=o["depth"], rgb_out_f32=o["rgb_f"], depth_out_f32=o["depth_f"],
                      device_ptrs=True, hold=hold, deadline_ns=deadline_ns)


def _np(o):
    g = {k: v.cpu().numpy() for k, v in o.items()}
    g["depth"] = g["depth"].view(np.uint16)
    return g


def test_budget_below_the_weights_and_workspaces_fails_create():
    from paper_2604_27441_amd._lib import RevoError
    blobs = synth.make_weights(3, **SMALL)
    with pytest.raises(RevoError) as e:
        _rec(blobs, hbm_budget_bytes=1 << 20)
    assert e.value.code == -12
    with _rec(blobs) as rec:
        fixed = rec.stats()["hbm_fixed_bytes"]
    assert fixed > (1 << 20)
    with pytest.raises(RevoError) as e:
        _rec(blobs, hbm_budget_bytes=fixed - 4096)        # fixed workspace size, budget just below
    assert e.value.code == -12


def test_submit_waits_for_budget_then_succeeds():
    """A budget that holds the weights, workspaces and references but only
    one recovery's staging and prediction buffers: a second recovery
    submitted while the first is still queued gets REVO_EAGAIN, and succeeds
    once poll has handed the first back.  Both results equal the unbudgeted
    ones."""
    blobs = synth.make_weights(3, perturb_seed=4, **SMALL)
    a = synth.make_request(121, 122, H, W, loss=("stripes", 0.5))
    b = synth.make_request(121, 123, H, W, loss=("stripes", 0.5))
    b["rgb_refs"], b["depth_refs"] = a["rgb_refs"], a["depth_refs"]
    with _rec(blobs) as rec:
        fixed = rec.stats()["hbm_fixed_bytes"]
        push_refs(rec, 0, a)
        alone = [recover(rec, [(0, r)])[0] for r in (a, b)]
    px = H * W
    ring = 5 * (_r4k(3 * px) + _r4k(2 * px))
    one = _r4k(3 * px) + _r4k(px) + _r4k(12 * px) + _r4k(2 * px) + _r4k(px) + _r4k(4 * px)
    with _rec(blobs, hbm_budget_bytes=fixed + ring + one + one // 2) as rec:
        assert rec.stats()["hbm_fixed_bytes"] == fixed
        push_refs(rec, 0, a)
        oa, ob = _outs(), _outs()
        # a is held in the queue (REVO_HOLD keeps it for up to 2 ms), so its
        # staging is still charged when b arrives
        ta = _submit(rec, 0, a, oa, hold=True)
        assert ta is not None
        assert _submit(rec, 0, b, ob) is None             # REVO_EAGAIN
        got = rec.wait([ta])
        assert got[ta].status == 0
        tb = _submit(rec, 0, b, ob)
        assert tb is not None
        assert rec.wait([tb])[tb].status == 0
        assert rec.stats()["hbm_pool_bytes"] <= ring + one + one // 2
    for o, al in ((oa, alone[0]), (ob, alone[1])):
        g = _np(o)
        for key in ("rgb", "depth", "rgb_f", "depth_f"):
            assert np.array_equal(g[key], al[key]), key


def test_expired_deadline_is_shed_and_its_clean_depth_still_becomes_a_reference():
    blobs = synth.make_weights(3, perturb_seed=4, **SMALL)
    req = synth.make_request(125, 126, H, W, loss=("stripes", 0.5))
    nxt = synth.make_request(125, 127, H, W, t_target=req["t_target"] + 1, loss=("stripes", 0.5))
    assert req["mask_rgb"].any() and nxt["mask_depth"].any()
    with _rec(blobs, shed=True) as rec:
        push_refs(rec, 0, req)
        o = _outs()
        # RGB lost, depth intact, deadline long past: shed, nothing written
        t = _submit(rec, 0, req, o, deadline_ns=1, rgb_lost=True, depth_lost=False)
        c = rec.wait([t])[t]
        assert c.status == 1
        g = _np(o)
        assert not g["rgb"].any() and not g["depth"].any() and not g["rgb_f"].any()
        # a depth recovery with time to spare runs against the new reference set
        o2 = _outs()
        t2 = _submit(rec, 0, nxt, o2, deadline_ns=time.clock_gettime_ns(time.CLOCK_MONOTONIC) + 10**10,
                     rgb_lost=False, depth_lost=True)
        c2 = rec.wait([t2])[t2]
        assert c2.status == 0
        st = rec.stats()
        # the five clean references and the depth recovery
        assert st["shed"] == 1 and st["served"] == len(req["ref_idx"]) + 1
    g2 = _np(o2)
    r2 = dict(nxt)
    r2["depth_refs"] = list(req["depth_refs"][1:]) + [req["depth"]]
    r2["ref_idx"] = list(req["ref_idx"][1:]) + [req["t_target"]]
    rb = oracle.recover(r2, blobs, modalities=("depth",), **SMALL)["depth"]
    assert np.abs(g2["depth_f"] - rb[1]).max() <= 0.5
    assert np.array_equal(g2["rgb"], nxt["rgb"])          # the clean RGB is copied


def test_recovery_before_any_clean_frame_is_refused_at_submit():
    from paper_2604_27441_amd._lib import RevoError
    blobs = synth.make_weights(3, **SMALL)
    req = synth.make_request(81, 82, 32, 48, loss=("stripes", 0.5))
    with _rec(blobs) as rec:
        with pytest.raises(RevoError) as e:
            _submit(rec, 5, req, _outs(32, 48))
        assert e.value.code == -61
        push_refs(rec, 5, req)
        o = _outs(32, 48)
        t = _submit(rec, 5, req, o)
        assert rec.wait([t])[t].status == 0
        # a different size has no reference yet
        other = synth.make_request(83, 84, 48, 64, loss=("stripes", 0.5))
        with pytest.raises(RevoError) as e:
            _submit(rec, 5, other, _outs())
        assert e.value.code == -61


def test_reference_frames_dropped_by_a_resolution_change_outlive_the_batch_reading_them():
    """A recovery, then at once a clean frame of the same stream at a new size
    (its old references leave the ring) and clean frames of other streams at
    the old size (whose staging would reuse freed memory): the recovery still
    reads its own references."""
    blobs = synth.make_weights(3, perturb_seed=4, **SMALL)
    req = synth.make_request(131, 132, H, W, loss=("stripes", 0.5))
    big = synth.make_request(133, 134, 64, 80, loss=("stripes", 0.5))
    rng = np.random.default_rng(135)
    with _rec(blobs, max_streams=8) as rec:
        push_refs(rec, 0, req)
        for s in range(1, 5):
            push_refs(rec, s, req)
        alone = recover(rec, [(0, req)])[0]
        o = _outs()
        t = _submit(rec, 0, req, o)
        rec.submit(0, int(req["t_target"]) + 1, 80, 64, rgb=dev(big["rgb"]), depth=dev(big["depth"]),
                   device_ptrs=True)
        for s in range(1, 5):
            for f in range(3):
                rgb = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
                dep = rng.integers(500, 3000, (H, W), dtype=np.uint16)
                rec.submit(s, 100 + f, W, H, rgb=dev(rgb), depth=dev(dep), device_ptrs=True)
        c = rec.wait([t])[t]
        assert c.status == 0
        while rec.poll(64, 200_000):
            pass
    g = _np(o)
    for key in ("rgb", "depth", "rgb_f", "depth_f"):
        assert np.array_equal(g[key], alone[key]), key


def test_input_copies_follow_the_callers_stream():
    """With hip_stream set, submit orders its input copies after the work the
    caller already enqueued there: inputs written on that stream behind a
    spin of a few milliseconds are read as written."""
    blobs = synth.make_weights(3, perturb_seed=4, **SMALL)
    req = synth.make_request(141, 142, H, W, loss=("stripes", 0.5))
    s = torch.cuda.Stream()
    with _rec(blobs, hip_stream=s.cuda_stream) as rec:
        push_refs(rec, 0, req)
        alone = recover(rec, [(0, req)])[0]
        src = [dev(req["rgb"]), dev(req["mask_rgb"]), dev(req["depth"]), dev(req["mask_depth"])]
        dst = [torch.zeros_like(x) for x in src]
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            torch.cuda._sleep(20_000_000)
            for d_, s_ in zip(dst, src):
                d_.copy_(s_)
        o = _outs()
        t = rec.submit(0, int(req["t_target"]), W, H, rgb=dst[0], mask_rgb=dst[1], depth=dst[2], mask_depth=dst[3],
                       rgb_out=o["rgb"], depth_out=o["depth"], rgb_out_f32=o["rgb_f"], depth_out_f32=o["depth_f"],
                       device_ptrs=True)
        assert rec.wait([t])[t].status == 0
    g = _np(o)
    for key in ("rgb", "depth", "rgb_f", "depth_f"):
        assert np.array_equal(g[key], alone[key]), key


def test_malformed_requests_are_refused_and_the_context_stays_usable():
    """REVO_EINVAL at submit for a request with no frame, a mask without its
    frame, a stream id past max_streams, a frame below 16 x 16, and host
    memory passed as device pointers; none of them disturbs a later recovery."""
    from paper_2604_27441_amd._lib import RevoError
    blobs = synth.make_weights(3, **SMALL)
    req = synth.make_request(85, 86, H, W, loss=("stripes", 0.5))
    rgb, mask = dev(req["rgb"]), dev(req["mask_rgb"])
    bad = [
        dict(stream_id=0, width=W, height=H),                                          # no frame at all
        dict(stream_id=0, width=W, height=H, mask_depth=mask),                         # mask without its frame
        dict(stream_id=64, width=W, height=H, rgb=rgb, mask_rgb=mask),                 # stream id >= max_streams
        dict(stream_id=0, width=15, height=H, rgb=rgb, mask_rgb=mask),                 # narrower than one patch
        dict(stream_id=0, width=W, height=H, rgb=req["rgb"], mask_rgb=req["mask_rgb"]),  # host memory
    ]
    with _rec(blobs, max_streams=64) as rec:
        push_refs(rec, 0, req)
        for kw in bad:
            sid, w_, h_ = kw.pop("stream_id"), kw.pop("width"), kw.pop("height")
            with pytest.raises(RevoError) as e:
                rec.submit(sid, int(req["t_target"]), w_, h_, device_ptrs=True, **kw)
            assert e.value.code == -22, (kw.keys(), e.value.code)
        o = _outs()
        t = _submit(rec, 0, req, o)
        c = rec.wait([t])[t]
        assert c.status == 0
        ref = oracle.recover(req, blobs, **SMALL)
        g = _np(o)
        assert np.abs(g["rgb_f"].astype(np.float64) - ref["rgb"][1]).max() <= 1e-4
