"""Each HIP kernel on its own, through revo_op_*, against the FP64 oracle's
same layer (linear, LayerNorm, GELU, attention of Sec. 3.4.1 / App. B.1)."""
import math

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

FP32, BF16 = 0, 1
RNG = np.random.default_rng(77)


def _lib():
    import paper_2604_27441_amd as pkg
    return pkg.lib


def _dt(prec):
    return torch.float32 if prec == FP32 else torch.bfloat16


def _as_op(a, prec):
    """Host operand rounded to the kernel's operand type, and its exact float64 value."""
    t = torch.tensor(a, dtype=torch.float32).to(_dt(prec))
    return t.cuda(), t.to(torch.float64).numpy()


# FP32 products of at most 256 workgroups of 64-wide tiles run 8-wave
# workgroups that split each stage's k steps; 12800 x 384 (600 tiles of 64)
# and 4608 x 1536 (432 tiles of 128) take the 4-wave forms
@pytest.mark.parametrize("prec", [FP32, BF16])
@pytest.mark.parametrize("M,N,K", [(1, 64, 64), (300, 192, 384), (1000, 1152, 384), (257, 384, 1536), (77, 64, 192),
                                   (200, 256, 320), (12800, 384, 384), (4608, 1536, 384)])
@pytest.mark.parametrize("epi", [0, 1, 2])
def test_linear(prec, M, N, K, epi):
    x = RNG.standard_normal((M, K))
    w = RNG.standard_normal((N, K)) * math.sqrt(2.0 / K)
    b = 0.1 * RNG.standard_normal(N)
    xd, x64 = _as_op(x, prec)
    wd, w64 = _as_op(w, prec)
    bd = torch.tensor(b, dtype=torch.float32).cuda()
    b64 = bd.double().cpu().numpy()
    ref = oracle.linear(x64, w64, b64)
    if epi == 1:
        res = RNG.standard_normal((M, N)).astype(np.float32)
        out = torch.tensor(res).cuda()
        ref = ref + res
    else:
        out = torch.zeros((M, N), dtype=torch.float32 if prec == FP32 or epi == 1 else torch.bfloat16).cuda()
        if epi == 2:
            ref = oracle.gelu(ref)
    rc = _lib().revo_op_linear(prec, epi, xd.data_ptr(), wd.data_ptr(), bd.data_ptr(), out.data_ptr(), M, N, K, None)
    assert rc == 0
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    # accumulation in FP32 over K terms; a BF16 result is additionally rounded once (2^-9 relative)
    scale = np.abs(ref).max() + 1e-30
    tol = 2e-6 * math.sqrt(K) * scale if (prec == FP32 or epi == 1) else 4e-3 * np.abs(ref) + 2e-6 * math.sqrt(K) * scale
    assert np.all(np.abs(got - ref) <= tol + 1e-7), float(np.abs(got - ref).max())


@pytest.mark.parametrize("prec", [FP32, BF16])
@pytest.mark.parametrize("rows,D", [(1, 384), (1000, 384), (333, 192), (5, 24)])
def test_layernorm(prec, rows, D):
    x = (RNG.standard_normal((rows, D)) * 3 + 2).astype(np.float32)
    g = (1 + 0.1 * RNG.standard_normal(D)).astype(np.float32)
    b = (0.1 * RNG.standard_normal(D)).astype(np.float32)
    y = torch.zeros((rows, D), dtype=_dt(prec)).cuda()
    xd, gd, bd = torch.tensor(x).cuda(), torch.tensor(g).cuda(), torch.tensor(b).cuda()  # alive across the launch
    rc = _lib().revo_op_layernorm(prec, xd.data_ptr(), gd.data_ptr(), bd.data_ptr(), y.data_ptr(), rows, D, None)
    assert rc == 0
    torch.cuda.synchronize()
    ref = oracle.layer_norm(x.astype(np.float64), g.astype(np.float64), b.astype(np.float64))
    got = y.double().cpu().numpy()
    tol = 1e-5 if prec == FP32 else 4e-3 * np.abs(ref) + 1e-5
    assert np.all(np.abs(got - ref) <= tol), float(np.abs(got - ref).max())


def _swap23(n):
    """Column order of the BF16 V^T operand: token index with bits 2 and 3 swapped."""
    c = np.arange(n)
    return (c & ~12) | ((c & 4) << 1) | ((c & 8) >> 1)


def _attn_inputs(heads, ntok, prec, scale=1.0, ld=None):
    ld = ld or ((ntok + 64 + 15) // 16 * 16)
    q = RNG.standard_normal((heads, ntok, 64)) * scale
    k = RNG.standard_normal((heads, ntok, 64)) * scale
    v = RNG.standard_normal((heads, ntok, 64))
    dt = _dt(prec)
    # operand values as the kernel sees them
    q_op = torch.tensor(q * (math.log2(math.e) / 8), dtype=torch.float32).to(dt)
    k_op = torch.tensor(k, dtype=torch.float32).to(dt)
    v_op = torch.tensor(v, dtype=torch.float32).to(dt)
    qd = torch.zeros((heads, ld, 64), dtype=dt)
    kd = torch.zeros((heads, ld, 64), dtype=dt)
    vt = torch.zeros((heads, 64, ld), dtype=dt)
    qd[:, :ntok] = q_op
    kd[:, :ntok] = k_op
    vt[:, :, :ntok] = v_op.transpose(1, 2)
    if prec == BF16:
        vt = vt[:, :, _swap23(ld)]   # the BF16 kernel's V^T column order
    q64 = q_op.double().numpy() / (math.log2(math.e) / 8)
    return qd.cuda(), kd.cuda(), vt.cuda(), q64, k_op.double().numpy(), v_op.double().numpy(), ld


@pytest.mark.parametrize("prec", [FP32, BF16])
@pytest.mark.parametrize("heads,ntok", [(1, 1), (2, 63), (2, 64), (1, 128), (6, 576), (3, 1000), (1, 4099)])
def test_attention(prec, heads, ntok):
    qd, kd, vt, q64, k64, v64, ld = _attn_inputs(heads, ntok, prec, scale=1.5)
    o = torch.zeros((ntok, heads * 64), dtype=_dt(prec)).cuda()
    rc = _lib().revo_op_attention(prec, qd.data_ptr(), kd.data_ptr(), vt.data_ptr(), o.data_ptr(), heads, ntok, ld, None)
    assert rc == 0
    got = o.double().cpu().numpy()
    for h in range(heads):
        ref = oracle.attention_head(q64[h], k64[h], v64[h])
        g = got[:, h * 64:(h + 1) * 64]
        if prec == FP32:
            assert np.abs(g - ref).max() < 2e-5 * np.abs(v64[h]).max(), float(np.abs(g - ref).max())
        else:
            # probabilities rounded to bf16 (2^-9 relative) and the output rounded once more
            err = np.abs(g - ref)
            assert err.max() < 1.5e-2 * np.abs(v64[h]).max(), float(err.max())
            assert np.sqrt(np.mean(err ** 2)) < 4e-3 * np.sqrt(np.mean(ref ** 2)) + 1e-3


@pytest.mark.parametrize("prec", [FP32, BF16])
@pytest.mark.parametrize("direction,amp", [(1, 60.0), (-1, 60.0), (1, 6.0)])
def test_attention_drifting_max(prec, direction, amp):
    """Scores that rise (or fall) steadily over the keys, by amp * 5 in
    natural-log units end to end.  A rise of 300 raises the running max many
    times (BF16: the first pass, which keeps the first block's max,
    overflows and the row is recomputed with running maxima); a fall leaves
    the first block's max in place; a rise of 30 (43 in log2 units) keeps
    the first pass, with probabilities up to about 2^43.  The result must be
    the softmax average in every case."""
    heads, ntok = 2, 2000
    qd, kd, vt, q64, k64, v64, ld = _attn_inputs(heads, ntok, prec, scale=0.3)
    u = np.zeros(64)
    u[0] = 1.0
    ramp = np.linspace(0.0, 1.0, ntok) if direction > 0 else np.linspace(1.0, 0.0, ntok)
    kk = k64 + amp * ramp[None, :, None] * u
    qq = q64 + 40.0 * u
    dt = _dt(prec)
    k_op = torch.tensor(kk, dtype=torch.float32).to(dt)
    q_op = torch.tensor(qq * (math.log2(math.e) / 8), dtype=torch.float32).to(dt)
    kd[:, :ntok] = k_op.cuda()
    qd[:, :ntok] = q_op.cuda()
    q64 = q_op.double().numpy() / (math.log2(math.e) / 8)
    k64 = k_op.double().numpy()
    o = torch.zeros((ntok, heads * 64), dtype=dt).cuda()
    assert _lib().revo_op_attention(prec, qd.data_ptr(), kd.data_ptr(), vt.data_ptr(), o.data_ptr(), heads, ntok, ld, None) == 0
    got = o.double().cpu().numpy()
    for h in range(heads):
        ref = oracle.attention_head(q64[h], k64[h], v64[h])
        err = np.abs(got[:, h * 64:(h + 1) * 64] - ref)
        # a float32 score s (log2 units) is off by a few ulp(s): each
        # probability moves by about 2^-23 |s| relative, times a few
        smax = (np.abs(q64[h]) @ np.abs(k64[h]).T).max() / 8 * math.log2(math.e)
        bound = 2e-5 + 1e-6 * smax if prec == FP32 else 1.5e-2
        assert err.max() < bound * np.abs(v64[h]).max(), (float(err.max()), smax)


def test_attention_overflow_in_some_tiles():
    """BF16: only the queries aligned with the rising keys overflow the first
    pass, so only their workgroups (query tiles 0, 4 and 5 of 128) repeat the
    rows in the safe pass; every row must match the oracle."""
    heads, ntok = 2, 1000
    qd, kd, vt, q64, k64, v64, ld = _attn_inputs(heads, ntok, BF16, scale=0.3)
    u = np.zeros(64)
    u[0] = 1.0
    kk = k64 + 60.0 * np.linspace(0.0, 1.0, ntok)[None, :, None] * u
    hot = np.zeros(ntok, dtype=bool)
    hot[:100] = True
    hot[600:700] = True
    qq = q64 + 40.0 * hot[None, :, None] * u
    k_op = torch.tensor(kk, dtype=torch.float32).to(torch.bfloat16)
    q_op = torch.tensor(qq * (math.log2(math.e) / 8), dtype=torch.float32).to(torch.bfloat16)
    kd[:, :ntok] = k_op.cuda()
    qd[:, :ntok] = q_op.cuda()
    q64 = q_op.double().numpy() / (math.log2(math.e) / 8)
    k64 = k_op.double().numpy()
    o = torch.zeros((ntok, heads * 64), dtype=torch.bfloat16).cuda()
    assert _lib().revo_op_attention(BF16, qd.data_ptr(), kd.data_ptr(), vt.data_ptr(), o.data_ptr(), heads, ntok, ld, None) == 0
    got = o.double().cpu().numpy()
    for h in range(heads):
        ref = oracle.attention_head(q64[h], k64[h], v64[h])
        err = np.abs(got[:, h * 64:(h + 1) * 64] - ref)
        assert err.max() < 1.5e-2 * np.abs(v64[h]).max(), float(err.max())


def test_attention_uniform_keys_average_values():
    """Equal keys give the mean of V exactly up to rounding (softmax is uniform)."""
    heads, ntok = 2, 300
    qd, kd, vt, q64, k64, v64, ld = _attn_inputs(heads, ntok, FP32)
    kd[:, :ntok] = kd[:, :1].clone()
    o = torch.zeros((ntok, heads * 64), dtype=torch.float32).cuda()
    assert _lib().revo_op_attention(FP32, qd.data_ptr(), kd.data_ptr(), vt.data_ptr(), o.data_ptr(), heads, ntok, ld, None) == 0
    got = o.double().cpu().numpy()
    for h in range(heads):
        assert np.allclose(got[:, h * 64:(h + 1) * 64], v64[h].mean(0), atol=2e-6)


def test_convert_bf16_rounding():
    x = (RNG.standard_normal(100003) * np.exp(RNG.uniform(-30, 30, 100003))).astype(np.float32)
    y = torch.zeros(x.size, dtype=torch.bfloat16).cuda()
    xd = torch.tensor(x).cuda()
    assert _lib().revo_op_convert(BF16, xd.data_ptr(), y.data_ptr(), x.size, None) == 0
    torch.cuda.synchronize()
    assert np.array_equal(y.double().cpu().numpy(), oracle.bf16_round(x))


FP8 = 2


def _fp8_group_loss(a8, b8):
    """Bound on what the FP8 MFMA drops when it sums products: it adds each
    group of 8 consecutive k products after aligning them to the group's
    largest product, keeping about 14 bits below that product's leading bit
    (measured on gfx950: 448*448 + 4 gives 448*448, 448*448 + 8 is exact;
    across groups the sum is FP32).  Per product the loss is below both |p|
    and 2^(E - 13), E = floor(log2 max |p|) of its group (a factor 2 of
    margin over the measured window).  a8 [M][K], b8 [N][K] in code units."""
    # products of two E4M3 values are exact in float32
    a8, b8 = np.abs(a8).astype(np.float32), np.abs(b8).astype(np.float32)
    loss = np.zeros((a8.shape[0], b8.shape[0]))
    for g in range(0, a8.shape[1], 8):
        p = a8[:, None, g:g + 8] * b8[None, :, g:g + 8]
        _, e = np.frexp(p.max(axis=2))            # max = f * 2^e, f in [0.5, 1)
        win = np.ldexp(np.float32(1), e - 14)      # 2^(floor(log2 max) - 13)
        loss += np.minimum(p, win[..., None]).sum(axis=2)
    return loss


def _fp8_bytes(v):
    """E4M3 bytes of values that are already E4M3 numbers (exact in torch)."""
    return torch.tensor(v, dtype=torch.float32).to(torch.float8_e4m3fn).view(torch.uint8)


def test_convert_fp8_rounding():
    x = (RNG.standard_normal(100003) * np.exp(RNG.uniform(-14, 8, 100003))).astype(np.float32)
    x[:4] = [448.0, 460.0, 1e6, -3e4]
    xd = torch.tensor(x).cuda()
    y = torch.zeros(x.size, dtype=torch.uint8).cuda()
    assert _lib().revo_op_convert(FP8, xd.data_ptr(), y.data_ptr(), x.size, None) == 0
    torch.cuda.synchronize()
    got = y.cpu().view(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(got, oracle.e4m3_round(x))


@pytest.mark.parametrize("M,N,K", [(1, 64, 64), (300, 576, 192), (1000, 1152, 384), (257, 384, 1536), (200, 192, 256)])
@pytest.mark.parametrize("epi", [0, 1, 2])
def test_linear_fp8(M, N, K, epi):
    x = RNG.standard_normal((M, K)) * 3
    w = RNG.standard_normal((N, K)) * math.sqrt(2.0 / K)
    b = 0.1 * RNG.standard_normal(N)
    rnd = oracle.FP8Rounding({"l.qkv": float(np.abs(x).max() / 448)})
    xs = rnd.scales["l.qkv"]
    xq = rnd.act(x, "l.qkv")                       # dequantised operands the kernel sees
    wq = rnd.weight(w, "l.qkv")
    ws = np.abs(w).max(axis=1) / 448.0
    x8 = _fp8_bytes(xq / xs).cuda()
    w8 = _fp8_bytes(wq / ws[:, None]).cuda()
    wsd = torch.tensor(ws, dtype=torch.float32).cuda()
    xsd = torch.tensor([xs], dtype=torch.float32).cuda()
    bd = torch.tensor(b, dtype=torch.float32).cuda()
    ref = xq @ wq.T + bd.double().cpu().numpy()
    # the kernel's scales are float32 copies of the oracle's
    ref_scale_err = 2 * 2.0 ** -24 * np.abs(xq).sum(1, keepdims=True) @ np.abs(wq).max(1, keepdims=True).T
    ref_scale_err = ref_scale_err + _fp8_group_loss(xq / xs, wq / ws[:, None]) * ws[None, :] * xs
    osd = torch.tensor([0.05], dtype=torch.float32).cuda()
    if epi == 1:
        res = RNG.standard_normal((M, N)).astype(np.float32)
        out = torch.tensor(res).cuda()
        ref = ref + res
    elif epi == 0:
        out = torch.zeros((M, N), dtype=torch.bfloat16).cuda()
    else:
        out = torch.zeros((M, N), dtype=torch.uint8).cuda()
    rc = _lib().revo_op_linear_fp8(epi, x8.data_ptr(), w8.data_ptr(), wsd.data_ptr(), xsd.data_ptr(), bd.data_ptr(),
                                   out.data_ptr(), osd.data_ptr(), M, N, K, None)
    assert rc == 0
    torch.cuda.synchronize()
    scale = np.abs(ref).max() + 1e-30
    tol = 2e-6 * math.sqrt(K) * scale + ref_scale_err      # on the pre-activation value
    if epi == 2:
        got = out.cpu().view(torch.float8_e4m3fn).to(torch.float64).numpy() * 0.05
        want = oracle.e4m3_round(oracle.gelu(ref) / 0.05) * 0.05
        # |GELU'| <= 1.13, so the pre-activation tolerance moves GELU by at
        # most 1.13 tol; each side then rounds to E4M3 (half a step each,
        # bounded by the step at the larger of the two magnitudes)
        big = np.maximum(np.abs(want), np.abs(got)) / 0.05
        step = np.exp2(np.maximum(np.floor(np.log2(np.maximum(big, 1e-30))), -6) - 3) * 0.05
        bad = np.argwhere(np.abs(got - want) > step + 1.13 * tol + 1e-12)
        assert bad.size == 0, [(tuple(i), float(ref[tuple(i)]), float(got[tuple(i)] / 0.05),
                                float(want[tuple(i)] / 0.05)) for i in bad[:8]]
        assert np.sum(got != want) <= max(2, 0.01 * got.size)   # codes away from rounding midpoints agree
        return
    got = out.double().cpu().numpy()
    if epi == 0:
        tol = tol + 4e-3 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= tol + 1e-7), float(np.abs(got - ref).max())


def _fp8_vt_col(t):
    """Column of key t in the FP8 attention kernel's V^T (a permutation inside
    each aligned group of 64 keys)."""
    t = np.asarray(t)
    return (t & ~63) | (((t >> 2) & 1) << 5) | (((t >> 5) & 1) << 4) | (((t >> 3) & 3) << 2) | (t & 3)


def _e4m3_bytes(x):
    return torch.tensor(np.asarray(x, np.float32)).to(torch.float8_e4m3fn).view(torch.uint8)


@pytest.mark.parametrize("heads,ntok", [(1, 64), (3, 130), (2, 1000), (1, 4099)])
def test_attention_fp8(heads, ntok):
    """FP8 attention (the FP8 form) against FP64 on the exact operands, within
    the error budget of the FP8-rounding oracle (E4M3 Q, K, V with per-head
    power-of-two scales, E4M3 probabilities): twice its MSE, four times its
    max error."""
    rng = np.random.default_rng(4242 + ntok)
    c = oracle.QK_LOG2
    ld = (ntok + 64 + 63) // 64 * 64
    q = rng.standard_normal((heads, ntok, 64)) * 1.5
    k = rng.standard_normal((heads, ntok, 64)) * 1.5
    v = rng.standard_normal((heads, ntok, 64))
    q8 = torch.zeros((heads, ld, 64), dtype=torch.uint8)
    k8 = torch.zeros((heads, ld, 64), dtype=torch.uint8)
    vt8 = torch.zeros((heads, 64, ld), dtype=torch.uint8)
    exps, rounded = [], []
    for h in range(heads):
        sq = oracle.pow2_scale(np.abs(q[h] * c).max() / 448)
        sk = oracle.pow2_scale(np.abs(k[h]).max() / 448)
        sv = oracle.pow2_scale(np.abs(v[h]).max() / 448)
        exps.append((int(round(math.log2(sq))), int(round(math.log2(sk))), int(round(math.log2(sv)))))
        q8[h, :ntok] = _e4m3_bytes(q[h] * c / sq)
        k8[h, :ntok] = _e4m3_bytes(k[h] / sk)
        vb = _e4m3_bytes(v[h] / sv)                               # [ntok][64]
        vt8[h][:, torch.from_numpy(_fp8_vt_col(np.arange(ntok)))] = vb.T.contiguous()
        rounded.append((oracle.e4m3_round(q[h] * c / sq) * sq / c, oracle.e4m3_round(k[h] / sk) * sk,
                        oracle.e4m3_round(v[h] / sv) * sv))
    ex = np.array([e[0] for e in exps] + [e[1] for e in exps] + [e[2] for e in exps], dtype=np.int32)
    o = torch.zeros((ntok, heads * 64), dtype=torch.bfloat16).cuda()
    qd, kd, vd = q8.cuda(), k8.cuda(), vt8.cuda()
    rc = _lib().revo_op_attention_fp8(qd.data_ptr(), kd.data_ptr(), vd.data_ptr(), o.data_ptr(), heads, ntok, ld,
                                      ex.ctypes.data, None)
    assert rc == 0
    got = o.double().cpu().numpy()
    p_round = oracle.FP8Rounding({})
    for h in range(heads):
        exact = oracle.attention_head(q[h], k[h], v[h])
        emu = oracle.attention_head(*rounded[h], rnd=p_round, site="x.attn.p")
        g = got[:, h * 64:(h + 1) * 64]
        e_gpu, e_emu = g - exact, emu - exact
        rms, rms_emu = np.sqrt(np.mean(e_gpu ** 2)), np.sqrt(np.mean(e_emu ** 2))
        print(f"fp8 attention heads {heads} ntok {ntok} h {h}: rms {rms:.3g} (oracle {rms_emu:.3g}), "
              f"max {np.abs(e_gpu).max():.3g} (oracle {np.abs(e_emu).max():.3g})")
        assert rms <= np.sqrt(2.0) * rms_emu, (h, rms, rms_emu)
        assert np.abs(e_gpu).max() <= 4.0 * np.abs(e_emu).max(), h
