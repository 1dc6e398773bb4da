"""An independent FP64 statement of the recovery network built from PyTorch
library routines (conv3d, layer_norm, linear, scaled_dot_product_attention,
gelu).  It pins the oracle's wiring: every layer, residual, positional term
and the output placement must agree.  CPU only; test infrastructure."""
import math

import torch
import torch.nn.functional as F


def _pe(D, tau, gy, gx):
    d = D // 3
    inv = 10000.0 ** (-torch.arange(0, d, 2, dtype=torch.float64) / d)

    def enc(s):                      # s: [n] positions -> [n, d]
        ang = s[:, None] * inv[None, :]
        return torch.stack([torch.sin(ang), torch.cos(ang)], dim=-1).reshape(len(s), d)

    yy, xx = torch.meshgrid(torch.arange(gy, dtype=torch.float64), torch.arange(gx, dtype=torch.float64), indexing="ij")
    rows = []
    for t in tau:
        n = gy * gx
        rows.append(torch.cat([enc(torch.full((n,), float(t), dtype=torch.float64)), enc(yy.reshape(-1)), enc(xx.reshape(-1))], dim=1))
    return torch.cat(rows, 0)


class Params:
    def __init__(self, blob, C, T, De, ne, Dd, nd):
        self.t = blob if isinstance(blob, torch.Tensor) else torch.tensor(blob, dtype=torch.float64)
        self.pos = 0
        L = T * 256 * C
        self.emb_w, self.emb_b = self.take(De, L), self.take(De)
        self.enc = [self.block(De) for _ in range(ne)]
        self.enc_g, self.enc_b = self.take(De), self.take(De)
        self.e2d_w, self.e2d_b = self.take(Dd, De), self.take(Dd)
        self.dec = [self.block(Dd) for _ in range(nd)]
        self.dec_g, self.dec_b = self.take(Dd), self.take(Dd)
        self.head_w, self.head_b = self.take(L, Dd), self.take(L)
        assert self.pos == self.t.numel()

    def take(self, *shape):
        n = math.prod(shape)
        out = self.t[self.pos:self.pos + n].view(*shape)
        self.pos += n
        return out

    def block(self, D):
        names = ["g1", "b1", "wqkv", "bqkv", "wp", "bp", "g2", "b2", "w1", "bb1", "w2", "bb2"]
        shapes = [(D,), (D,), (3 * D, D), (3 * D,), (D, D), (D,), (D,), (D,), (4 * D, D), (4 * D,), (D, 4 * D), (D,)]
        return {n: self.take(*s) for n, s in zip(names, shapes)}


def _block(x, p, heads):
    N, D = x.shape
    a = F.layer_norm(x, (D,), p["g1"], p["b1"], eps=1e-6)
    qkv = F.linear(a, p["wqkv"], p["bqkv"]).view(N, 3, heads, D // heads).permute(1, 2, 0, 3)
    o = F.scaled_dot_product_attention(qkv[0], qkv[1], qkv[2])       # [heads, N, dh]
    x = x + F.linear(o.permute(1, 0, 2).reshape(N, D), p["wp"], p["bp"])
    a = F.layer_norm(x, (D,), p["g2"], p["b2"], eps=1e-6)
    return x + F.linear(F.gelu(F.linear(a, p["w1"], p["bb1"])), p["w2"], p["bb2"])


def predict(refs, ref_idx, target, t_target, mask, blob, C, k=5, T=2,
            De=384, ne=12, heads_e=6, Dd=192, nd=4, heads_d=3, as_tensor=False):
    """Prediction [H, W, C] in model units (a float64 tensor that keeps the
    autograd graph to blob with as_tensor, when blob is a tensor)."""
    P = Params(blob, C, T, De, ne, Dd, nd)
    scale = 255.0 if C == 3 else 4000.0
    tgt = torch.tensor(target, dtype=torch.float64) / scale
    refs_t = torch.tensor(refs, dtype=torch.float64) / scale
    if C == 1:
        tgt, refs_t = tgt[..., None], refs_t[..., None]
    tgt = tgt * (1 - torch.tensor(mask, dtype=torch.float64))[..., None]
    n = len(ref_idx)
    frames = [refs_t[0]] * (k - n) + [refs_t[i] for i in range(n)] + [tgt]
    times = [ref_idx[0]] * (k - n) + list(ref_idx) + [t_target]
    pad = (-len(frames)) % T
    frames = [frames[0]] * pad + frames
    times = [times[0]] * pad + times
    H, W = tgt.shape[:2]
    Hp, Wp = 16 * math.ceil(H / 16), 16 * math.ceil(W / 16)
    vid = torch.stack(frames).permute(3, 0, 1, 2)                        # [C, F, H, W]
    vid = F.pad(vid, (0, Wp - W, 0, Hp - H))
    w = P.emb_w.view(De, T, 16, 16, C).permute(0, 4, 1, 2, 3)
    x = F.conv3d(vid[None], w, P.emb_b, stride=(T, 16, 16))[0]          # [De, J, gy, gx]
    J, gy, gx = x.shape[1:]
    x = x.reshape(De, -1).T
    tau = [t_target - times[j * T] for j in range(J)]
    x = x + _pe(De, tau, gy, gx)
    for b in P.enc:
        x = _block(x, b, heads_e)
    z = F.linear(F.layer_norm(x, (De,), P.enc_g, P.enc_b, eps=1e-6), P.e2d_w, P.e2d_b) + _pe(Dd, tau, gy, gx)
    for b in P.dec:
        z = _block(z, b, heads_d)
    z = F.layer_norm(z, (Dd,), P.dec_g, P.dec_b, eps=1e-6)
    o = F.linear(z, P.head_w, P.head_b).view(J, gy, gx, T, 16, 16, C)[J - 1, :, :, T - 1]
    img = o.permute(0, 2, 1, 3, 4).reshape(gy * 16, gx * 16, C)
    return img[:H, :W] if as_tensor else img[:H, :W].numpy()
