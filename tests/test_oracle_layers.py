"""Pins of the FP64 oracle's layers against library routines, closed forms,
invariants and direct loops (architecture of Sec. 3.4.1 / App. B.1)."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle

RNG = np.random.default_rng(1234)


def test_bf16_round_known_values():
    one = 1.0
    ulp = 2.0 ** -7
    assert oracle.bf16_round(np.array([one]))[0] == 1.0
    assert oracle.bf16_round(np.array([one + ulp / 2]))[0] == 1.0            # tie -> even
    assert oracle.bf16_round(np.array([one + 1.5 * ulp]))[0] == one + 2 * ulp  # tie -> even
    assert oracle.bf16_round(np.array([one + ulp / 2 + 2.0 ** -20]))[0] == one + ulp
    assert oracle.bf16_round(np.array([-(one + 1.5 * ulp)]))[0] == -(one + 2 * ulp)


def test_bf16_round_matches_torch():
    x = RNG.standard_normal(100000) * np.exp(RNG.uniform(-20, 20, 100000))
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.bf16_round(x), ref)


def test_gelu_closed_form_and_library():
    z = np.linspace(-6, 6, 1001)
    direct = np.array([0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in z])
    assert np.allclose(oracle.gelu(z), direct, rtol=0, atol=1e-15)
    lib = F.gelu(torch.tensor(z), approximate="none").numpy()
    assert np.allclose(oracle.gelu(z), lib, rtol=0, atol=1e-14)
    assert oracle.gelu(np.array([0.0]))[0] == 0.0
    # GELU(1) = Phi(1), GELU(-1) = -Phi(-1)
    assert abs(oracle.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert abs(oracle.gelu(np.array([-1.0]))[0] + 0.15865525393145707) < 1e-15
    assert abs(oracle.gelu(np.array([20.0]))[0] - 20.0) < 1e-12


def test_layer_norm_library_and_moments():
    x = RNG.standard_normal((37, 24)) * 3 + 1.5
    g = 1 + 0.1 * RNG.standard_normal(24)
    b = 0.1 * RNG.standard_normal(24)
    ours = oracle.layer_norm(x, g, b)
    lib = F.layer_norm(torch.tensor(x), (24,), torch.tensor(g), torch.tensor(b), eps=1e-6).numpy()
    assert np.allclose(ours, lib, rtol=0, atol=1e-13)
    plain = oracle.layer_norm(x, np.ones(24), np.zeros(24))
    assert np.allclose(plain.mean(axis=1), 0, atol=1e-14)
    # biased variance with eps: var(out) = var / (var + eps)
    v = x.var(axis=1)
    assert np.allclose(plain.var(axis=1), v / (v + 1e-6), atol=1e-13)


def _attention_loops(q, k, v):
    n, d = q.shape
    out = np.zeros((n, v.shape[1]))
    for i in range(n):
        s = [sum(q[i, t] * k[j, t] for t in range(d)) / math.sqrt(d) for j in range(k.shape[0])]
        m = max(s)
        e = [math.exp(x - m) for x in s]
        z = sum(e)
        for c in range(v.shape[1]):
            out[i, c] = sum(e[j] * v[j, c] for j in range(k.shape[0])) / z
    return out


def test_attention_direct_loops():
    q, k, v = (RNG.standard_normal((9, 6)) for _ in range(3))
    assert np.allclose(oracle.attention_head(q, k, v), _attention_loops(q, k, v), atol=1e-13)


def test_attention_library_and_chunking():
    q, k, v = (RNG.standard_normal((300, 64)) * 2 for _ in range(3))
    lib = F.scaled_dot_product_attention(torch.tensor(q)[None], torch.tensor(k)[None], torch.tensor(v)[None]).numpy()[0]
    assert np.allclose(oracle.attention_head(q, k, v), lib, atol=1e-12)
    assert np.allclose(oracle.attention_head(q, k, v, chunk=7), lib, atol=1e-12)


def test_attention_special_cases():
    v = RNG.standard_normal((1, 8))
    q, k = RNG.standard_normal((1, 8)), RNG.standard_normal((1, 8))
    assert np.allclose(oracle.attention_head(q, k, v), v)                     # N = 1 -> V
    q = RNG.standard_normal((5, 8))
    kk = np.tile(RNG.standard_normal((1, 8)), (11, 1))
    v = RNG.standard_normal((11, 8))
    assert np.allclose(oracle.attention_head(q, kk, v), np.tile(v.mean(0), (5, 1)))  # equal keys
    assert np.allclose(oracle.attention_head(np.zeros((3, 8)), RNG.standard_normal((11, 8)), v),
                       np.tile(v.mean(0), (3, 1)))                              # zero query
    q, k, v = (RNG.standard_normal((13, 8)) for _ in range(3))
    perm = RNG.permutation(13)
    base = oracle.attention_head(q, k, v)
    assert np.allclose(oracle.attention_head(q[perm], k, v), base[perm])         # equivariant in queries
    assert np.allclose(oracle.attention_head(q, k[perm], v[perm]), base)         # invariant to key order


def test_sinusoid_closed_form():
    d = 128
    e0 = oracle.sinusoid(d, 0.0)
    assert np.array_equal(e0[0::2], np.zeros(64)) and np.array_equal(e0[1::2], np.ones(64))
    s = 7.0
    e = oracle.sinusoid(d, s)
    assert abs(e[0] - math.sin(7.0)) < 1e-15 and abs(e[1] - math.cos(7.0)) < 1e-15
    assert abs(e[126] - math.sin(7.0 * 10000.0 ** (-126.0 / 128))) < 1e-15
    assert np.allclose(e[0::2] ** 2 + e[1::2] ** 2, 1.0)
    pe = oracle.positional_embedding(384, 3.0, 5.0, 9.0)
    assert np.allclose(pe[:128], oracle.sinusoid(128, 3.0))
    assert np.allclose(pe[128:256], oracle.sinusoid(128, 5.0))
    assert np.allclose(pe[256:], oracle.sinusoid(128, 9.0))
    assert not np.allclose(oracle.positional_embedding(384, 1.0, 0, 0), oracle.positional_embedding(384, 2.0, 0, 0))


def test_sequence_frames():
    slots, times = oracle.sequence_frames([4, 5, 6, 7, 8], 9, 5, 2)
    assert slots == [0, 1, 2, 3, 4, 5] and times == [4, 5, 6, 7, 8, 9]
    slots, times = oracle.sequence_frames([7, 8], 9, 5, 2)        # stream start: repeat oldest
    assert slots == [0, 0, 0, 0, 1, 2] and times == [7, 7, 7, 7, 8, 9]
    slots, times = oracle.sequence_frames([1, 2, 3, 4], 6, 4, 2)  # k+1 odd: pad at the old end
    assert slots == [0, 0, 1, 2, 3, 4] and times == [1, 1, 2, 3, 4, 6]
    with pytest.raises(ValueError):
        oracle.sequence_frames([], 3, 5, 2)


def test_tubelet_vectors_index_map():
    T, C, Hp, Wp = 2, 3, 32, 48
    f, r, c_, ch = np.meshgrid(np.arange(4), np.arange(Hp), np.arange(Wp), np.arange(C), indexing="ij")
    frames = (f * 1e6 + r * 1e3 + c_ + ch * 0.1).astype(np.float64)
    U = oracle.tubelet_vectors(frames, T)
    gy, gx = Hp // 16, Wp // 16
    assert U.shape == (2 * gy * gx, T * 256 * C)
    for n in [0, 5, 6, 11]:
        j, y, x = n // (gy * gx), (n % (gy * gx)) // gx, n % gx
        for t, py, px, ci in [(0, 0, 0, 0), (1, 15, 3, 2), (0, 7, 15, 1), (1, 0, 0, 1)]:
            e = ((t * 16 + py) * 16 + px) * C + ci
            assert U[n, e] == frames[j * T + t, 16 * y + py, 16 * x + px, ci]


def test_tubelet_embedding_is_conv3d():
    """Tubelet embedding == Conv3d with kernel = stride = (T, 16, 16)."""
    T, C, F_, Hp, Wp, D = 2, 3, 6, 32, 48, 12
    frames = RNG.random((F_, Hp, Wp, C))
    w = RNG.standard_normal((D, T * 256 * C)) * 0.05
    b = RNG.standard_normal(D)
    ours = oracle.linear(oracle.tubelet_vectors(frames, T), w, b)
    vid = torch.tensor(frames).permute(3, 0, 1, 2)[None]                   # [1, C, F, H, W]
    wt = torch.tensor(w).view(D, T, 16, 16, C).permute(0, 4, 1, 2, 3)       # [D, C, T, 16, 16]
    lib = F.conv3d(vid, wt, torch.tensor(b), stride=(T, 16, 16))[0]          # [D, J, gy, gx]
    lib = lib.permute(1, 2, 3, 0).reshape(-1, D).numpy()
    assert np.allclose(ours, lib, atol=1e-12)


def test_composite_rules():
    H, W = 4, 5
    pred = RNG.standard_normal((H, W, 3))
    recv = RNG.integers(0, 256, (H, W, 3), dtype=np.uint8)
    mask = (RNG.random((H, W)) < 0.5).astype(np.uint8)
    of, oi = oracle.composite(pred, recv, mask, 3)
    keep = mask == 0
    assert np.array_equal(oi[keep], recv[keep])
    assert np.array_equal(of[keep], recv[keep] / 255.0)
    assert np.allclose(of[~keep], np.clip(pred[~keep], 0, 1))
    assert np.array_equal(oi[~keep], np.rint(255 * np.clip(pred[~keep], 0, 1)).astype(np.uint8))
    # ties round to even: 1.5 -> 2, 2.5 -> 2
    p = np.array([[[1.5 / 255, 2.5 / 255, 0.0]]])
    _, q = oracle.composite(p, np.zeros((1, 1, 3), np.uint8), np.ones((1, 1), np.uint8), 3)
    assert list(q[0, 0]) == [2, 2, 0]
    dp = np.array([[[-1.0], [0.25], [100.0]]])           # -4000 mm, 1000 mm, 400 km
    recv_d = np.array([[7, 8, 9]], np.uint16)
    df, di = oracle.composite(dp, recv_d, np.ones((1, 3), np.uint8), 1)
    assert list(df[0]) == [0.0, 1000.0, 65535.0] and list(di[0]) == [0, 1000, 65535]
    df, di = oracle.composite(dp, recv_d, np.zeros((1, 3), np.uint8), 1)
    assert list(di[0]) == [7, 8, 9] and list(df[0]) == [7.0, 8.0, 9.0]


def test_e4m3_round_matches_torch_and_saturates():
    x = RNG.standard_normal(200000) * np.exp(RNG.uniform(-12, 6, 200000))
    x = x[np.abs(x) <= 448]
    ref = torch.tensor(x, dtype=torch.float64).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(oracle.e4m3_round(x), ref)
    assert list(oracle.e4m3_round(np.array([448.0, 460.0, 1e6, -1e6]))) == [448.0, 448.0, 448.0, -448.0]
    sub = 2.0 ** -9
    assert list(oracle.e4m3_round(np.array([sub, sub / 2, 1.5 * sub, 0.0]))) == [sub, 0.0, 2 * sub, 0.0]
    assert list(oracle.e4m3_round(np.array([1.0625, 1.1875, -2.5]))) == [1.0, 1.25, -2.5]


def test_fp8_rounding_scales():
    w = RNG.standard_normal((7, 33))
    r = oracle.FP8Rounding({"enc0.qkv": 0.01})
    wq = r.weight(w, "enc0.qkv")
    assert np.allclose(np.abs(wq).max(axis=1), np.abs(w).max(axis=1))      # row max maps to 448 exactly
    assert np.all(np.abs(wq - w) <= np.abs(w).max(axis=1, keepdims=True) / 448 * 16 + 1e-15)
    x = RNG.standard_normal((5, 33))
    assert np.array_equal(r.act(x, "enc0.qkv"), oracle.e4m3_round(x / 0.01) * 0.01)
    assert np.array_equal(r.weight(w, "head"), oracle.bf16_round(w))
    # without FP8 attention, attention operands stay bf16
    r16 = oracle.FP8Rounding({"enc0.attn.k1": 0.01}, fp8_attention=False)
    assert np.array_equal(r16.act(x, "enc0.attn.k1"), oracle.bf16_round(x))
    assert np.array_equal(r16.act(np.abs(x), "enc0.attn.p"), oracle.bf16_round(np.abs(x)))


def test_fp8_attention_operand_rounding():
    """Attention operands of the FP8 form: per-head power-of-two scales (the
    smallest power of two >= absmax / 448), Q rounded as the kernels hold it
    (times log2(e) / 8), probabilities with unit scale."""
    assert oracle.pow2_scale(0.3) == 0.5 and oracle.pow2_scale(0.25) == 0.25 and oracle.pow2_scale(0.0) == 1.0
    assert oracle.pow2_scale(3.0) == 4.0 and oracle.pow2_scale(1e-3) == 2.0 ** -9
    x = RNG.standard_normal((6, 64)) * 3
    sc = {"dec0.attn.q2": 2.9 / 448, "dec0.attn.k2": 5.0 / 448, "dec0.attn.v2": 0.7 / 448}
    r = oracle.FP8Rounding(sc)
    c = oracle.QK_LOG2
    sq = 2.0 ** math.ceil(math.log2(2.9 / 448 * c))
    assert np.array_equal(r.act(x, "dec0.attn.q2"), oracle.e4m3_round(x * c / sq) * sq / c)
    sk = 2.0 ** math.ceil(math.log2(5.0 / 448))
    assert np.array_equal(r.act(x, "dec0.attn.k2"), oracle.e4m3_round(x / sk) * sk)
    assert sk == 2.0 ** -6                                                 # 5/448 = 0.01116 -> 1/64
    sv = 2.0 ** -9                                                         # 0.7/448 = 0.00156 -> 1/512
    assert np.array_equal(r.act(x, "dec0.attn.v2"), oracle.e4m3_round(x / sv) * sv)
    p = np.exp(-np.abs(x))
    assert np.array_equal(r.act(p, "dec0.attn.p"), oracle.e4m3_round(p))
    assert r.attn_operand("enc11.attn.q5") == "q" and r.attn_operand("enc11.qkv") is None


def test_absmax_recorder_sites():
    import synth
    req = synth.make_request(5, 6, 32, 48, loss=("stripes", 0.5))
    blobs = synth.make_weights(2, enc_depth=2, dec_depth=1)
    rec = oracle.AbsMaxRecorder()
    oracle.recover(req, blobs, enc_depth=2, dec_depth=1, rnd=rec, modalities=("rgb",))
    sites = set(rec.absmax)
    blocks = [(f"enc{i}.", 6) for i in range(2)] + [("dec0.", 3)]
    want = {"emb", "e2d", "head"} | {f"{b}{k}" for b, _ in blocks for k in ("qkv", "proj", "fc1", "fc2", "attn.p")}
    want |= {f"{b}attn.{t}{h}" for b, heads in blocks for t in "qkv" for h in range(heads)}
    assert sites == want
    assert all(v > 0 for v in rec.absmax.values())
    exact = oracle.recover(req, blobs, enc_depth=2, dec_depth=1, modalities=("rgb",))
    again = oracle.recover(req, blobs, enc_depth=2, dec_depth=1, rnd=oracle.AbsMaxRecorder(), modalities=("rgb",))
    assert np.array_equal(exact["rgb"][0], again["rgb"][0])                 # recording changes nothing


@pytest.mark.parametrize("gy,gx,T,C", [(2, 3, 2, 3), (3, 2, 2, 1), (1, 4, 3, 3), (2, 2, 1, 1)])
def test_head_placement_is_the_index_bijection(gy, gx, T, C):
    """Head outputs tagged (token id, output index) land pixel by pixel where
    the tubelet layout puts them: token y*gx + x, slot T-1, (py, px, c)."""
    P, L = gy * gx, T * 256 * C
    o = np.arange(P)[:, None] * 100000.0 + np.arange(L)[None, :]
    frame = oracle.place_target_slot(o, gy, gx, T, C)
    assert frame.shape == (16 * gy, 16 * gx, C)
    for Y in range(16 * gy):
        for X in range(16 * gx):
            for c in range(C):
                tok = (Y // 16) * gx + (X // 16)
                idx = (((T - 1) * 16 + Y % 16) * 16 + X % 16) * C + c
                assert frame[Y, X, c] == tok * 100000.0 + idx
    # a bijection onto the target slot's outputs
    used = np.sort(frame.ravel())
    want = np.sort((np.arange(P)[:, None] * 100000.0 + ((T - 1) * 256 * C + np.arange(256 * C))[None, :]).ravel())
    assert np.array_equal(used, want)


def test_absmax_recorder_scale_values():
    """Calibration scales are max |activation| over every call of a site,
    divided by 448 (the E4M3 maximum), and 1 for a site that only saw zeros;
    with such a scale the largest activation maps onto 448 exactly."""
    rec = oracle.AbsMaxRecorder()
    x1 = np.array([[0.5, -2.0], [1.0, 0.25]])
    x2 = np.array([[-3.5, 0.0, 1.5]])
    assert rec.act(x1, "enc0.qkv") is x1                      # exact arithmetic passes through
    rec.act(x2, "enc0.qkv")
    rec.act(np.zeros((3, 4)), "enc0.proj")
    rec.act(np.array([[7.0]]), "dec0.fc2")
    rec.act(np.array([[-1.0]]), "dec0.fc2")
    s = rec.scales()
    assert s == {"enc0.qkv": 3.5 / 448.0, "enc0.proj": 1.0, "dec0.fc2": 7.0 / 448.0}
    r = oracle.FP8Rounding(s)
    q = r.act(x2, "enc0.qkv")
    assert q[0, 0] == -3.5 and q[0, 1] == 0.0                 # -absmax -> -448 -> back exactly
