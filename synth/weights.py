"""Seeded He-normal weight blobs for the recovery network (FP32, flat).

The paper fixes neither widths nor depths; the model used here is a ViT-S
sized encoder (384 wide, 12 blocks, 6 heads, MLP 1536) and a 192-wide
decoder (4 blocks, 3 heads, MLP 768), patch 16, tubelet T (Sec. 3.4.1 and
App. B.1/B.3 give the ViViT family, k = 5 and T = 2).

Blob layout per modality (every matrix stored [out][in], row-major):
  emb.w [De, T*256*C]  emb.b [De]
  per encoder block: ln1.g ln1.b [De]  qkv.w [3De, De] qkv.b [3De]
                     proj.w [De, De] proj.b [De]  ln2.g ln2.b [De]
                     fc1.w [4De, De] fc1.b [4De]  fc2.w [De, 4De] fc2.b [De]
  enc_norm.g enc_norm.b [De]
  e2d.w [Dd, De] e2d.b [Dd]
  per decoder block: as above with Dd
  dec_norm.g dec_norm.b [Dd]
  head.w [T*256*C, Dd] head.b [T*256*C]

He-normal: every matrix is N(0, 2 / fan_in) drawn in FP64 from one
numpy default_rng(seed) stream (RGB model first, then depth; within a model
in forward order emb, per block qkv/proj/fc1/fc2, e2d, head), then rounded
once to FP32.  Biases are 0, LayerNorm gains 1 and shifts 0.  With
``perturb_seed`` the biases, gains and shifts are instead drawn from a second
stream (bias, shift ~ N(0, 0.1^2); gain ~ 1 + N(0, 0.1^2)) so that tests
exercise every affine term.
"""
import numpy as np

PATCH = 16
ENC = dict(dim=384, depth=12, heads=6, mlp=1536)
DEC = dict(dim=192, depth=4, heads=3, mlp=768)


def model_shapes(channels, tubelet=2, enc_depth=None, dec_depth=None,
                 enc_dim=None, dec_dim=None):
    """Ordered list of (name, shape, kind) with kind in {'w', 'b', 'g', 's'}."""
    C, T = int(channels), int(tubelet)
    De = enc_dim or ENC["dim"]
    Dd = dec_dim or DEC["dim"]
    ne = ENC["depth"] if enc_depth is None else enc_depth
    nd = DEC["depth"] if dec_depth is None else dec_depth
    tub = T * PATCH * PATCH * C
    out = [("emb.w", (De, tub), "w"), ("emb.b", (De,), "b")]

    def block(prefix, D):
        return [
            (prefix + "ln1.g", (D,), "g"), (prefix + "ln1.b", (D,), "s"),
            (prefix + "qkv.w", (3 * D, D), "w"), (prefix + "qkv.b", (3 * D,), "b"),
            (prefix + "proj.w", (D, D), "w"), (prefix + "proj.b", (D,), "b"),
            (prefix + "ln2.g", (D,), "g"), (prefix + "ln2.b", (D,), "s"),
            (prefix + "fc1.w", (4 * D, D), "w"), (prefix + "fc1.b", (4 * D,), "b"),
            (prefix + "fc2.w", (D, 4 * D), "w"), (prefix + "fc2.b", (D,), "b"),
        ]

    for i in range(ne):
        out += block(f"enc{i}.", De)
    out += [("enc_norm.g", (De,), "g"), ("enc_norm.b", (De,), "s")]
    out += [("e2d.w", (Dd, De), "w"), ("e2d.b", (Dd,), "b")]
    for i in range(nd):
        out += block(f"dec{i}.", Dd)
    out += [("dec_norm.g", (Dd,), "g"), ("dec_norm.b", (Dd,), "s")]
    out += [("head.w", (tub, Dd), "w"), ("head.b", (tub,), "b")]
    return out


def weight_count(channels, **kw):
    return int(sum(int(np.prod(s)) for _, s, _ in model_shapes(channels, **kw)))


def _draw_model(rng, prng, channels, **kw):
    parts = []
    for name, shape, kind in model_shapes(channels, **kw):
        if kind == "w":
            fan_in = shape[1]
            a = rng.standard_normal(shape) * np.sqrt(2.0 / fan_in)
        elif prng is None:
            a = np.ones(shape) if kind == "g" else np.zeros(shape)
        elif kind == "g":
            a = 1.0 + 0.1 * prng.standard_normal(shape)
        else:
            a = 0.1 * prng.standard_normal(shape)
        parts.append(a.astype(np.float32).ravel())
    return np.concatenate(parts)


def make_weights(seed=0, tubelet=2, enc_depth=None, dec_depth=None,
                 perturb_seed=None, enc_dim=None, dec_dim=None):
    """Returns (rgb_blob, depth_blob), each a flat float32 array."""
    rng = np.random.default_rng(seed)
    prng = None if perturb_seed is None else np.random.default_rng(perturb_seed)
    kw = dict(tubelet=tubelet, enc_depth=enc_depth, dec_depth=dec_depth,
              enc_dim=enc_dim, dec_dim=dec_dim)
    rgb = _draw_model(rng, prng, 3, **kw)
    depth = _draw_model(rng, prng, 1, **kw)
    return rgb, depth
