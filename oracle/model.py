"""FP64 oracle: ReVo's post-decode neural loss-recovery forward pass.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes (Sec. 3.4.1, App. B.1, App. B.3): a ViViT / VideoMAE
style encoder-decoder that takes the k closest clean frames plus the current
corrupted frame and outputs one reconstructed frame; tubelets of T
consecutive frames and a patch form one token; both visible and corrupted
pixels are fed; no token shuffling; the same encoder-decoder at inference as
in pretraining; scaled dot-product attention inside the Transformer blocks;
positional embeddings encode the temporal distance between references and
the corrupted target; separate RGB and depth models.  k = 5, T = 2.

Where the paper is silent this oracle takes these readings: patch 16;
encoder 384 wide x 12 blocks x 6 heads (MLP 1536), decoder 192 x 4 x 3 (MLP
768); pre-LN blocks, LayerNorm eps 1e-6, exact-erf GELU, qkv bias; RGB /255,
depth /4000 mm; lost target pixels zero-filled in every channel; no mask
channel; a fixed three-axis sinusoidal positional embedding (temporal
distance, patch row, patch column) added after the embedding and after the
encoder-to-decoder projection; joint space-time attention over all tokens of
one request; a head emitting the full tubelet, of which the target frame's
time slot is kept; clamp to the valid range; received (unlost) pixels copied
through and only lost pixels replaced by the prediction.
"""
import math
from dataclasses import dataclass

import numpy as np
from scipy.special import erf

PATCH = 16


# --------------------------------------------------------------------------
# architecture description and weight unpacking
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Arch:
    """Shapes of one modality's model (C = 3 for RGB, 1 for depth)."""
    channels: int
    k: int = 5
    tubelet: int = 2
    enc_dim: int = 384
    enc_depth: int = 12
    enc_heads: int = 6
    dec_dim: int = 192
    dec_depth: int = 4
    dec_heads: int = 3

    @property
    def tub_len(self):
        return self.tubelet * PATCH * PATCH * self.channels


def unpack_weights(blob, arch):
    """Split a flat FP32 blob into named float64 arrays (matrices [out][in]).

    Order: emb, encoder blocks (ln1, qkv, proj, ln2, fc1, fc2), enc_norm,
    e2d, decoder blocks, dec_norm, head; each matrix is followed by its bias.
    """
    blob = np.asarray(blob)
    p = {}
    pos = 0

    def take(name, shape):
        nonlocal pos
        n = int(np.prod(shape))
        if pos + n > blob.size:
            raise ValueError("weight blob too short")
        p[name] = blob[pos:pos + n].astype(np.float64).reshape(shape)
        pos += n

    De, Dd = arch.enc_dim, arch.dec_dim
    take("emb.w", (De, arch.tub_len))
    take("emb.b", (De,))
    for i in range(arch.enc_depth):
        _take_block(take, f"enc{i}.", De)
    take("enc_norm.g", (De,))
    take("enc_norm.b", (De,))
    take("e2d.w", (Dd, De))
    take("e2d.b", (Dd,))
    for i in range(arch.dec_depth):
        _take_block(take, f"dec{i}.", Dd)
    take("dec_norm.g", (Dd,))
    take("dec_norm.b", (Dd,))
    take("head.w", (arch.tub_len, Dd))
    take("head.b", (arch.tub_len,))
    if pos != blob.size:
        raise ValueError(f"weight blob has {blob.size} values, layout needs {pos}")
    return p


def _take_block(take, pre, D):
    take(pre + "ln1.g", (D,))
    take(pre + "ln1.b", (D,))
    take(pre + "qkv.w", (3 * D, D))
    take(pre + "qkv.b", (3 * D,))
    take(pre + "proj.w", (D, D))
    take(pre + "proj.b", (D,))
    take(pre + "ln2.g", (D,))
    take(pre + "ln2.b", (D,))
    take(pre + "fc1.w", (4 * D, D))
    take(pre + "fc1.b", (4 * D,))
    take(pre + "fc2.w", (D, 4 * D))
    take(pre + "fc2.b", (D,))


# --------------------------------------------------------------------------
# operand rounding (error budgeting only; identity for the FP64 oracle)
# --------------------------------------------------------------------------
def bf16_round(x):
    """Round to the nearest bfloat16 value, ties to even, via float32.

    The value is first rounded to float32 (as a float32 producer would hold
    it), then its low 16 mantissa bits are rounded off.
    """
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def e4m3_round(x):
    """Round to the nearest OCP FP8 E4M3 value (bias 7, 3 mantissa bits,
    subnormal quantum 2^-9), ties to even, saturating at +-448."""
    x = np.asarray(x, np.float64)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.abs(x)))
    q = np.exp2(np.maximum(e, -6.0) - 3.0)
    return np.clip(np.rint(x / q) * q, -448.0, 448.0)


class Rounding:
    """Where a reduced-precision GPU form rounds matrix-multiply operands.

    Every matrix product names its call site ("emb", "<blk>.qkv",
    "<blk>.proj", "<blk>.fc1", "<blk>.fc2", "e2d", "head", and "attn" for
    Q/K/V and the probabilities); ``act`` rounds the activation operand and
    ``weight`` the weight operand.  ``Rounding()`` (the default) is exact
    FP64.  ``Rounding(bf16_round)`` rounds every operand the same way while
    sums, normalisation statistics, the residual stream and the composite
    stay in FP64.  It never reorders any computation.
    """

    def __init__(self, fn=None):
        self.fn = fn

    def act(self, x, site):
        return x if self.fn is None else self.fn(x)

    def weight(self, w, site):
        return w if self.fn is None else self.fn(w)


def pow2_scale(s):
    """Smallest power of two >= s (1 for s <= 0): the attention operands'
    scales, so that a scaled product is exact in the exponent."""
    return 2.0 ** math.ceil(math.log2(s)) if s > 0 else 1.0


QK_LOG2 = math.log2(math.e) / 8.0   # the kernels hold Q multiplied by log2(e) / sqrt(64)


class FP8Rounding(Rounding):
    """The FP8 form: the four block products and the encoder-to-decoder
    projection take E4M3 operands, activations with a per-tensor scale
    (absmax over a calibration set / 448) and weights with a per-output-row
    scale (row absmax / 448).  With fp8_attention, attention's Q, K and V
    are E4M3 with per-head power-of-two scales (the smallest power of two
    >= absmax / 448; Q as the kernels hold it, times log2(e) / 8) and the
    probabilities exp(s - row max) E4M3 with unit scale.  Embedding and
    head stay BF16 (and attention, without fp8_attention)."""

    FP8_KINDS = ("qkv", "proj", "fc1", "fc2", "e2d")

    def __init__(self, act_scales, fp8_attention=True):
        super().__init__(bf16_round)
        self.scales = dict(act_scales)
        self.fp8_attention = fp8_attention

    @classmethod
    def is_fp8(cls, site):
        return site.rsplit(".", 1)[-1] in cls.FP8_KINDS

    @staticmethod
    def attn_operand(site):
        """'q', 'k', 'v' or 'p' for an attention site ('<blk>.attn.q<h>', ...)."""
        parts = site.rsplit(".", 2)
        if len(parts) >= 2 and parts[-2] == "attn":
            return parts[-1][0]
        return None

    def act(self, x, site):
        kind = self.attn_operand(site) if self.fp8_attention else None
        if kind == "p":
            return e4m3_round(x)
        if kind in ("q", "k", "v"):
            x = np.asarray(x)
            if kind == "q":
                s = pow2_scale(self.scales[site] * QK_LOG2)
                return e4m3_round(x * QK_LOG2 / s) * s / QK_LOG2
            s = pow2_scale(self.scales[site])
            return e4m3_round(x / s) * s
        if not self.is_fp8(site):
            return bf16_round(x)
        s = self.scales[site]
        return e4m3_round(np.asarray(x) / s) * s

    def weight(self, w, site):
        if not self.is_fp8(site):
            return bf16_round(w)
        sw = np.abs(w).max(axis=1, keepdims=True) / 448.0
        sw = np.where(sw > 0, sw, 1.0)
        return e4m3_round(w / sw) * sw


class AbsMaxRecorder(Rounding):
    """Exact arithmetic that records max |activation operand| per call site
    (the calibration pass of the FP8 form)."""

    def __init__(self):
        super().__init__(None)
        self.absmax = {}

    def act(self, x, site):
        m = float(np.abs(x).max()) if np.size(x) else 0.0
        self.absmax[site] = max(self.absmax.get(site, 0.0), m)
        return x

    def scales(self):
        return {k: (v / 448.0 if v > 0 else 1.0) for k, v in self.absmax.items()}


EXACT = Rounding()


# --------------------------------------------------------------------------
# input preparation (Sec. 3.3 zero-filled partial frames; Sec. 3.4.1 inputs)
# --------------------------------------------------------------------------
def normalise(frame, channels):
    """Map a decoded frame to model units: RGB u8/255, depth u16 mm / 4000."""
    if channels == 3:
        return np.asarray(frame, np.float64) / 255.0
    return np.asarray(frame, np.float64)[..., None] / 4000.0


def zero_fill(x, mask):
    """Set every channel of lost pixels (mask == 1) to zero."""
    out = x.copy()
    out[np.asarray(mask) != 0] = 0.0
    return out


def sequence_frames(ref_idx, t_target, k, T):
    """Indices (into refs + [target]) and frame times of the model's input.

    The k references are oldest first and the target comes last.  With fewer
    than k references the oldest is repeated; the sequence is then padded at
    the old end, again with the oldest frame, up to a multiple of T.
    """
    n_ref = len(ref_idx)
    if n_ref == 0:
        raise ValueError("no clean reference frame")
    slots = [0] * (k - n_ref) + list(range(n_ref))
    slots = slots + [n_ref]                       # the target
    pad = (-len(slots)) % T
    slots = [0] * pad + slots
    times = [int(ref_idx[s]) if s < n_ref else int(t_target) for s in slots]
    return slots, times


def tubelet_vectors(frames, T):
    """Cut F frames [F, H', W', C] into tubelet vectors.

    Token n = j*P + y*(W'/16) + x for tubelet j (frames jT .. jT+T-1), patch
    row y and column x; its vector element ((t*16 + py)*16 + px)*C + c holds
    frame jT+t at pixel (16y+py, 16x+px), channel c.
    """
    F, Hp, Wp, C = frames.shape
    J = F // T
    gy, gx = Hp // PATCH, Wp // PATCH
    U = np.empty((J * gy * gx, T * PATCH * PATCH * C))
    for j in range(J):
        for y in range(gy):
            for x in range(gx):
                blk = frames[j * T:(j + 1) * T, y * PATCH:(y + 1) * PATCH, x * PATCH:(x + 1) * PATCH, :]
                U[j * gy * gx + y * gx + x] = blk.reshape(-1)
    return U


def sinusoid(d, s):
    """Length-d sinusoid of a scalar position s: sin at even, cos at odd slots.

    Element 2i is sin(s * 10000^(-2i/d)) and element 2i+1 the cosine.
    """
    out = np.empty(d)
    for i in range(d // 2):
        w = 10000.0 ** (-2.0 * i / d)
        out[2 * i] = math.sin(s * w)
        out[2 * i + 1] = math.cos(s * w)
    return out


def positional_embedding(D, tau, y, x):
    """Fixed embedding of a token's temporal distance tau to the target and
    its patch row and column: three length-D/3 sinusoids, concatenated."""
    d = D // 3
    return np.concatenate([sinusoid(d, tau), sinusoid(d, y), sinusoid(d, x)])


def token_positions(D, taus, gy, gx):
    """PE rows for every token of a request, in token order."""
    rows = []
    for tau in taus:
        for y in range(gy):
            for x in range(gx):
                rows.append(positional_embedding(D, tau, y, x))
    return np.stack(rows)


# --------------------------------------------------------------------------
# network layers
# --------------------------------------------------------------------------
def linear(x, w, b, rnd=EXACT, site=""):
    """x W^T + b with W stored [out][in]."""
    return rnd.act(x, site) @ rnd.weight(w, site).T + b


def layer_norm(x, g, b, eps=1e-6):
    """Per-row (x - mean) / sqrt(biased variance + eps) * g + b."""
    mu = x.mean(axis=-1, keepdims=True)
    var = ((x - mu) ** 2).mean(axis=-1, keepdims=True)
    return (x - mu) / np.sqrt(var + eps) * g + b


def gelu(z):
    """Exact GELU: z * Phi(z) = z/2 * (1 + erf(z / sqrt(2)))."""
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def attention_head(q, k, v, rnd=EXACT, chunk=2048, site="attn.p"):
    """softmax(q k^T / sqrt(d)) v over all keys, rows processed in chunks
    (rows are independent, so chunking changes nothing).  The probabilities
    exp(s - row max) are the product operand (call site `site`); the row sum
    divides afterwards."""
    d = q.shape[1]
    out = np.empty((q.shape[0], v.shape[1]))
    for r0 in range(0, q.shape[0], chunk):
        s = q[r0:r0 + chunk] @ k.T / math.sqrt(d)
        s -= s.max(axis=1, keepdims=True)
        e = np.exp(s)
        denom = e.sum(axis=1, keepdims=True)
        out[r0:r0 + chunk] = (rnd.act(e, site) @ v) / denom
    return out


def self_attention(a, p, pre, heads, rnd=EXACT):
    """Multi-head self-attention: qkv projection (columns Q | K | V, each
    head-major with contiguous heads), per-head attention, output projection.
    Each head's Q, K and V are product operands (call sites
    '<blk>.attn.q<h>', '.k<h>', '.v<h>'), and so are its probabilities
    ('<blk>.attn.p')."""
    N, D = a.shape
    dh = D // heads
    qkv = linear(a, p[pre + "qkv.w"], p[pre + "qkv.b"], rnd, pre + "qkv")
    o = np.empty((N, D))
    for h in range(heads):
        sl = slice(h * dh, (h + 1) * dh)
        q = rnd.act(qkv[:, sl], f"{pre}attn.q{h}")
        k = rnd.act(qkv[:, D + h * dh:D + (h + 1) * dh], f"{pre}attn.k{h}")
        v = rnd.act(qkv[:, 2 * D + h * dh:2 * D + (h + 1) * dh], f"{pre}attn.v{h}")
        o[:, sl] = attention_head(q, k, v, rnd, site=f"{pre}attn.p")
    return linear(o, p[pre + "proj.w"], p[pre + "proj.b"], rnd, pre + "proj")


def transformer_block(h, p, pre, heads, rnd=EXACT):
    """Pre-LN block: h + Attn(LN1(h)), then + FC2(GELU(FC1(LN2(.))))."""
    h = h + self_attention(layer_norm(h, p[pre + "ln1.g"], p[pre + "ln1.b"]), p, pre, heads, rnd)
    a = layer_norm(h, p[pre + "ln2.g"], p[pre + "ln2.b"])
    z = gelu(linear(a, p[pre + "fc1.w"], p[pre + "fc1.b"], rnd, pre + "fc1"))
    return h + linear(z, p[pre + "fc2.w"], p[pre + "fc2.b"], rnd, pre + "fc2")


# --------------------------------------------------------------------------
# whole forward pass and compositing
# --------------------------------------------------------------------------
def forward(refs, ref_idx, target, t_target, mask, params, arch, rnd=EXACT):
    """Prediction of the target frame in model units, [H, W, C], unclamped.

    refs: [n_ref, H, W(, 3)] clean frames oldest first; target: the received
    frame; mask: [H, W] with 1 = lost.
    """
    C, T = arch.channels, arch.tubelet
    H, W = np.asarray(target).shape[:2]
    Hp, Wp = PATCH * -(-H // PATCH), PATCH * -(-W // PATCH)
    gy, gx = Hp // PATCH, Wp // PATCH
    slots, times = sequence_frames(ref_idx, t_target, arch.k, T)
    seq = np.zeros((len(slots), Hp, Wp, C))
    for i, s in enumerate(slots):
        if s < len(ref_idx):
            fr = normalise(refs[s], C)
        else:
            fr = zero_fill(normalise(target, C), mask)
        seq[i, :H, :W, :] = fr
    J = len(slots) // T
    taus = [t_target - times[j * T] for j in range(J)]
    U = tubelet_vectors(seq, T)
    h = linear(U, params["emb.w"], params["emb.b"], rnd, "emb")
    h = h + token_positions(arch.enc_dim, taus, gy, gx)
    for i in range(arch.enc_depth):
        h = transformer_block(h, params, f"enc{i}.", arch.enc_heads, rnd)
    a = layer_norm(h, params["enc_norm.g"], params["enc_norm.b"])
    z = linear(a, params["e2d.w"], params["e2d.b"], rnd, "e2d")
    z = z + token_positions(arch.dec_dim, taus, gy, gx)
    for i in range(arch.dec_depth):
        z = transformer_block(z, params, f"dec{i}.", arch.dec_heads, rnd)
    P = gy * gx
    zt = layer_norm(z[(J - 1) * P:], params["dec_norm.g"], params["dec_norm.b"])
    o = linear(zt, params["head.w"], params["head.b"], rnd, "head")   # [P, T*256*C]
    return place_target_slot(o, gy, gx, T, C)[:H, :W, :]


def place_target_slot(o, gy, gx, T, C):
    """Frame [16 gy, 16 gx, C] from the head outputs of the target tubelet's
    tokens (§3.4.1: the module outputs the reconstructed frame).  Token
    p = y*gx + x holds T*16*16*C values ordered (t, py, px, c), as its input
    tubelet vector; the target frame is time slot t = T-1, and value
    (py, px, c) goes to pixel (16y + py, 16x + px), channel c."""
    P = gy * gx
    slot = np.asarray(o).reshape(P, T, PATCH, PATCH, C)[:, T - 1]
    return slot.reshape(gy, gx, PATCH, PATCH, C).transpose(0, 2, 1, 3, 4).reshape(gy * PATCH, gx * PATCH, C)


def composite(pred, received, mask, channels):
    """Final frame from the prediction (model units) and the received frame.

    Lost pixels take the clamped, denormalised prediction; received pixels
    are copied unchanged.  Returns (float output, integer output):
    RGB floats in [0, 1] and u8 codes; depth floats in mm and u16 codes.
    Integer codes of lost pixels round half to even.
    """
    lost = np.asarray(mask) != 0
    if channels == 3:
        p = np.clip(pred, 0.0, 1.0)
        recv_f = np.asarray(received, np.float64) / 255.0
        out_f = np.where(lost[..., None], p, recv_f)
        q = np.rint(255.0 * p).astype(np.uint8)
        out_i = np.where(lost[..., None], q, received).astype(np.uint8)
    else:
        p = np.clip(4000.0 * pred[..., 0], 0.0, 65535.0)
        recv_f = np.asarray(received, np.float64)
        out_f = np.where(lost, p, recv_f)
        q = np.rint(p).astype(np.uint16)
        out_i = np.where(lost, q, received).astype(np.uint16)
    return out_f, out_i


def recover(req, blobs, enc_depth=12, dec_depth=4, k=5, tubelet=2, rnd=EXACT,
            modalities=("rgb", "depth")):
    """Recover both modalities of one request (a dict as made by synth).

    blobs: (rgb_blob, depth_blob).  Returns {modality: (pred, out_f, out_i)}.
    """
    out = {}
    for mod in modalities:
        C = 3 if mod == "rgb" else 1
        arch = Arch(channels=C, k=k, tubelet=tubelet, enc_depth=enc_depth, dec_depth=dec_depth)
        params = unpack_weights(blobs[0] if C == 3 else blobs[1], arch)
        refs = req["rgb_refs"] if C == 3 else req["depth_refs"]
        target = req["rgb"] if C == 3 else req["depth"]
        mask = req["mask_rgb"] if C == 3 else req["mask_depth"]
        pred = forward(refs, req["ref_idx"], target, req["t_target"], mask, params, arch, rnd)
        out_f, out_i = composite(pred, target, mask, C)
        out[mod] = (pred, out_f, out_i)
    return out
