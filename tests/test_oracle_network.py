"""Whole-network pins of the FP64 oracle: an independent library-routine
statement of the network, invariants of compositing and zero-fill, and the
shapes the paper fixes (k = 5 clean frames + 1 target, T = 2, Sec. 3.4.1 and
App. B.3)."""
import numpy as np
import pytest

import oracle
import synth
from tests import torch_reference

TINY = dict(enc_dim=24, enc_depth=2, enc_heads=2, dec_dim=12, dec_depth=1, dec_heads=2)


def _tiny_blobs(T=2, seed=5):
    return synth.make_weights(seed, tubelet=T, enc_depth=2, dec_depth=1, enc_dim=24, dec_dim=12, perturb_seed=seed + 1)


@pytest.mark.parametrize("C", [3, 1])
@pytest.mark.parametrize("k,T,n_ref", [(5, 2, 5), (4, 2, 4), (5, 2, 2), (5, 3, 5), (3, 1, 3)])
def test_tiny_network_matches_library_statement(C, k, T, n_ref):
    req = synth.make_request(11, 12, 40, 32, k=k, loss=("stripes", 0.5))
    blobs = _tiny_blobs(T)
    blob = blobs[0] if C == 3 else blobs[1]
    arch = oracle.Arch(channels=C, k=k, tubelet=T, **TINY)
    params = oracle.unpack_weights(blob, arch)
    refs = (req["rgb_refs"] if C == 3 else req["depth_refs"])[k - n_ref:]
    ridx = req["ref_idx"][k - n_ref:]
    tgt = req["rgb"] if C == 3 else req["depth"]
    ours = oracle.forward(refs, ridx, tgt, req["t_target"], req["mask_rgb"], params, arch)
    ref = torch_reference.predict(refs, ridx, tgt, req["t_target"], req["mask_rgb"], blob, C, k=k, T=T,
                                  De=24, ne=2, heads_e=2, Dd=12, nd=1, heads_d=2)
    assert ours.shape == (40, 32, C)
    assert np.allclose(ours, ref, rtol=0, atol=1e-11)


@pytest.mark.slow
def test_full_model_c1_matches_library_statement():
    req = synth.make_batch("c1")[0]
    blobs = synth.make_weights(0)
    for C in (3, 1):
        arch = oracle.Arch(channels=C)
        params = oracle.unpack_weights(blobs[0] if C == 3 else blobs[1], arch)
        refs = req["rgb_refs"] if C == 3 else req["depth_refs"]
        tgt = req["rgb"] if C == 3 else req["depth"]
        ours = oracle.forward(refs, req["ref_idx"], tgt, req["t_target"], req["mask_rgb"], params, arch)
        ref = torch_reference.predict(refs, req["ref_idx"], tgt, req["t_target"], req["mask_rgb"],
                                      blobs[0] if C == 3 else blobs[1], C)
        assert np.allclose(ours, ref, rtol=0, atol=1e-9)


def test_weight_counts_match_model_size():
    # 24.03 M parameters for RGB, 23.44 M for depth at patch 16, T = 2
    assert synth.weight_count(3) == 24034752
    assert synth.weight_count(1) == 23443904
    a = oracle.Arch(channels=3)
    p = oracle.unpack_weights(np.zeros(24034752, np.float32), a)
    assert p["emb.w"].shape == (384, 1536) and p["head.w"].shape == (1536, 192)
    with pytest.raises(ValueError):
        oracle.unpack_weights(np.zeros(24034751, np.float32), a)


def test_he_normal_scale():
    rgb, _ = synth.make_weights(0, enc_depth=1, dec_depth=1)
    p = oracle.unpack_weights(rgb, oracle.Arch(channels=3, enc_depth=1, dec_depth=1))
    for name, fan_in in [("emb.w", 1536), ("enc0.fc2.w", 1536), ("e2d.w", 384), ("head.w", 192)]:
        assert abs(p[name].std() / np.sqrt(2.0 / fan_in) - 1) < 0.02
    assert np.all(p["enc0.qkv.b"] == 0) and np.all(p["enc0.ln1.g"] == 1)


def _run(req, blobs, **kw):
    return oracle.recover(req, blobs, enc_depth=2, dec_depth=1, **kw)


def test_clean_frame_is_copied_exactly():
    req = synth.make_request(21, 22, 40, 48, loss=("none", 0))
    out = _run(req, synth.make_weights(3, enc_depth=2, dec_depth=1))
    assert np.array_equal(out["rgb"][2], req["rgb"])
    assert np.array_equal(out["depth"][2], req["depth"])


def test_all_lost_returns_clamped_prediction():
    req = synth.make_request(21, 22, 40, 48, loss=("all", 0))
    out = _run(req, synth.make_weights(3, enc_depth=2, dec_depth=1))
    pred, of, oi = out["rgb"]
    assert np.allclose(of, np.clip(pred, 0, 1))
    pred, of, oi = out["depth"]
    assert np.allclose(of, np.clip(4000 * pred[..., 0], 0, 65535))


def test_lost_pixel_values_do_not_matter():
    req = synth.make_request(21, 22, 40, 48, loss=("stripes", 0.5))
    blobs = synth.make_weights(3, enc_depth=2, dec_depth=1)
    a = _run(req, blobs)
    req2 = dict(req)
    req2["rgb"] = req["rgb"].copy()
    req2["rgb"][req["mask_rgb"] != 0] = 255 - req2["rgb"][req["mask_rgb"] != 0]
    b = _run(req2, blobs, modalities=("rgb",))
    assert np.array_equal(a["rgb"][0], b["rgb"][0])


def test_temporal_distance_changes_prediction():
    """Reusing the same references for a later target (Sec. 3.4.1, error
    propagation in a GoP) changes only the temporal-distance embedding."""
    blobs = synth.make_weights(3, enc_depth=2, dec_depth=1)
    req = synth.make_request(21, 22, 40, 48, loss=("stripes", 0.5))
    a = _run(req, blobs, modalities=("rgb",))
    req2 = dict(req)
    req2["t_target"] = req["t_target"] + 3
    b = _run(req2, blobs, modalities=("rgb",))
    assert not np.allclose(a["rgb"][0], b["rgb"][0])


def test_token_count_and_padding():
    # 540 rows pad to 544: N = 3 * 34 * 60 = 6120 tokens at 960x540
    gy, gx = -(-540 // 16), -(-960 // 16)
    assert 3 * gy * gx == 6120
    U = oracle.tubelet_vectors(np.zeros((6, 48, 32, 3)), 2)
    assert U.shape == (3 * 3 * 2, 1536)
