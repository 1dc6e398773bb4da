"""FP64 reference of one pretraining step of the recovery network.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes: the models are first pretrained on frames with
randomly masked pixels, with the RGB objective L_RGB = MSE + alpha * TV used
for both the RGB and the depth model (Sec. 3.4.2, RGB loss equation, and the
"Robustness Across Codecs" paragraph); alpha = 0.01, Adam, learning rate
2e-4 (Sec. 4, implementation details).

Readings where the paper is silent:
  * the loss compares the network's raw prediction of the target frame
    (model units, before the clamp and the composite, which are inference
    steps) with the clean target frame;
  * MSE is the mean over every pixel and channel of a frame, TV the
    anisotropic mean absolute forward difference along x plus along y of the
    prediction (oracle.metrics.total_variation), and the batch loss is the
    mean of the per-frame losses;
  * Adam (Kingma & Ba 2015, Algorithm 1) with beta1 0.9, beta2 0.999,
    epsilon 1e-8 added to the square root of the bias-corrected second
    moment, no weight decay.

Gradients are taken by reverse-mode differentiation (torch autograd, float64)
of ``torch_forward``, which states the forward pass of oracle.model.forward
step by step with torch operations on a flat parameter tensor, so the
gradient comes out in the weight blob's layout.  The tests pin it three
ways: torch_forward against oracle.model.forward, central finite differences
of the NumPy oracle's loss, and autograd through a separate formulation
built from torch library layers.
"""
import math

import numpy as np
import torch

from .metrics import ALPHA_TV, total_variation
from .model import Arch, PATCH, normalise, sequence_frames, token_positions, unpack_weights, zero_fill

ADAM_LR = 2e-4        # Sec. 4
ADAM_BETA1 = 0.9      # not stated in the paper
ADAM_BETA2 = 0.999    # not stated in the paper
ADAM_EPS = 1e-8       # not stated in the paper


def param_views(theta, arch):
    """Named views into a flat float64 parameter tensor, in the blob layout
    of oracle.model.unpack_weights (matrices [out][in])."""
    index = unpack_weights(np.arange(theta.numel(), dtype=np.float64), arch)
    out = {}
    for name, idx in index.items():
        start, n = int(idx.flat[0]), idx.size
        out[name] = theta[start:start + n].view(*idx.shape)
    return out


def _layer_norm(x, g, b, eps=1e-6):
    mu = x.mean(dim=-1, keepdim=True)
    var = ((x - mu) ** 2).mean(dim=-1, keepdim=True)
    return (x - mu) / torch.sqrt(var + eps) * g + b


def _gelu(z):
    return 0.5 * z * (1.0 + torch.erf(z / math.sqrt(2.0)))


def _block(h, p, pre, heads):
    """Pre-LN Transformer block, as oracle.model.transformer_block."""
    N, D = h.shape
    dh = D // heads
    a = _layer_norm(h, p[pre + "ln1.g"], p[pre + "ln1.b"])
    qkv = a @ p[pre + "qkv.w"].T + p[pre + "qkv.b"]
    outs = []
    for i in range(heads):
        q = qkv[:, i * dh:(i + 1) * dh]
        k = qkv[:, D + i * dh:D + (i + 1) * dh]
        v = qkv[:, 2 * D + i * dh:2 * D + (i + 1) * dh]
        s = q @ k.T / math.sqrt(dh)
        e = torch.exp(s - s.max(dim=1, keepdim=True).values)
        outs.append((e / e.sum(dim=1, keepdim=True)) @ v)
    h = h + torch.cat(outs, dim=1) @ p[pre + "proj.w"].T + p[pre + "proj.b"]
    a = _layer_norm(h, p[pre + "ln2.g"], p[pre + "ln2.b"])
    z = _gelu(a @ p[pre + "fc1.w"].T + p[pre + "fc1.b"])
    return h + z @ p[pre + "fc2.w"].T + p[pre + "fc2.b"]


def torch_forward(theta, sample, arch):
    """Raw prediction [H, W, C] of one sample's target frame (model units).

    sample: dict with refs (k clean frames, oldest first), ref_idx, target
    (the clean target frame), t_target and mask ([H, W], 1 = masked: the
    pixel is zero-filled in the network's input)."""
    p = param_views(theta, arch)
    C, T = arch.channels, arch.tubelet
    target = np.asarray(sample["target"])
    H, W = target.shape[:2]
    Hp, Wp = PATCH * -(-H // PATCH), PATCH * -(-W // PATCH)
    gy, gx = Hp // PATCH, Wp // PATCH
    slots, times = sequence_frames(sample["ref_idx"], sample["t_target"], arch.k, T)
    seq = np.zeros((len(slots), Hp, Wp, C))
    n_ref = len(sample["ref_idx"])
    for i, s in enumerate(slots):
        fr = normalise(sample["refs"][s], C) if s < n_ref else zero_fill(normalise(target, C), sample["mask"])
        seq[i, :H, :W, :] = fr
    J = len(slots) // T
    taus = [sample["t_target"] - times[j * T] for j in range(J)]
    # tubelet vectors: token (j, y, x), element ((t*16 + py)*16 + px)*C + c
    U = torch.from_numpy(seq).reshape(J, T, gy, PATCH, gx, PATCH, C).permute(0, 2, 4, 1, 3, 5, 6)
    U = U.reshape(J * gy * gx, T * PATCH * PATCH * C)
    h = U @ p["emb.w"].T + p["emb.b"] + torch.from_numpy(token_positions(arch.enc_dim, taus, gy, gx))
    for i in range(arch.enc_depth):
        h = _block(h, p, f"enc{i}.", arch.enc_heads)
    z = _layer_norm(h, p["enc_norm.g"], p["enc_norm.b"]) @ p["e2d.w"].T + p["e2d.b"]
    z = z + torch.from_numpy(token_positions(arch.dec_dim, taus, gy, gx))
    for i in range(arch.dec_depth):
        z = _block(z, p, f"dec{i}.", arch.dec_heads)
    P = gy * gx
    zt = _layer_norm(z[(J - 1) * P:], p["dec_norm.g"], p["dec_norm.b"])
    o = zt @ p["head.w"].T + p["head.b"]                                # [P, T*256*C]
    slot = o.reshape(P, T, PATCH, PATCH, C)[:, T - 1]
    frame = slot.reshape(gy, gx, PATCH, PATCH, C).permute(0, 2, 1, 3, 4).reshape(gy * PATCH, gx * PATCH, C)
    return frame[:H, :W, :]


def _tv_t(x):
    return (x[:, 1:] - x[:, :-1]).abs().mean() + (x[1:] - x[:-1]).abs().mean()


def pretrain_loss_t(preds, gts):
    """Batch loss: mean over frames of MSE + ALPHA_TV * TV(pred) (torch)."""
    terms = [((pr - g) ** 2).mean() + ALPHA_TV * _tv_t(pr) for pr, g in zip(preds, gts)]
    return sum(terms) / len(terms)


def pretrain_loss(preds, gts):
    """The same batch loss on NumPy arrays (float64)."""
    terms = [float(np.mean((np.asarray(pr) - g) ** 2)) + ALPHA_TV * total_variation(np.asarray(pr))
             for pr, g in zip(preds, gts)]
    return sum(terms) / len(terms)


def ground_truth(sample, channels):
    """Clean target frame in model units, [H, W, C]."""
    return normalise(sample["target"], channels)


def loss_and_grad(blob, samples, arch):
    """Batch loss and its gradient with respect to every parameter (flat,
    blob layout), float64."""
    theta = torch.tensor(np.asarray(blob, np.float64), dtype=torch.float64, requires_grad=True)
    preds = [torch_forward(theta, s, arch) for s in samples]
    gts = [torch.from_numpy(ground_truth(s, arch.channels)) for s in samples]
    loss = pretrain_loss_t(preds, gts)
    loss.backward()
    return float(loss.detach()), theta.grad.numpy().copy(), [p.detach().numpy() for p in preds]


def adam_step(params, grad, m, v, step, lr=ADAM_LR, beta1=ADAM_BETA1, beta2=ADAM_BETA2, eps=ADAM_EPS):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); step counts from 1.
    Returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return params - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def train_step(blob, samples, arch, m=None, v=None, step=1, lr=ADAM_LR):
    """One pretraining step: loss, gradient, and the Adam-updated blob."""
    loss, grad, preds = loss_and_grad(blob, samples, arch)
    params = np.asarray(blob, np.float64)
    m = np.zeros_like(params) if m is None else m
    v = np.zeros_like(params) if v is None else v
    new, m, v = adam_step(params, grad, m, v, step, lr)
    return dict(loss=loss, grad=grad, params=new, m=m, v=v, preds=preds)


__all__ = ["ADAM_LR", "ADAM_BETA1", "ADAM_BETA2", "ADAM_EPS", "Arch", "param_views", "torch_forward",
           "pretrain_loss_t", "pretrain_loss", "ground_truth", "loss_and_grad", "adam_step", "train_step"]
