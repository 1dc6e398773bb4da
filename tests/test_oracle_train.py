"""Pins of the pretraining-step oracle (oracle.train) against things other
than itself: the NumPy forward pass and loss, central finite differences of
that NumPy loss, autograd through an independent network built from torch
library layers (tests/torch_reference.py), and the closed form of Adam's
first steps (Kingma & Ba 2015, Algorithm 1)."""
import math

import numpy as np
import pytest
import torch

import oracle
import oracle.train as ot
import synth
from tests import torch_reference

TINY = dict(enc_depth=2, dec_depth=1)


def _setup(C, H=32, W=48, B=2, seed=3):
    arch = oracle.Arch(channels=C, **TINY)
    blob = synth.make_weights(seed, perturb_seed=seed + 1, **TINY)[0 if C == 3 else 1]
    return arch, blob, synth.make_pretrain_batch(seed, B, H, W, C)


def _numpy_loss(blob, samples, arch, p=None):
    p = oracle.unpack_weights(blob, arch) if p is None else p
    preds = [oracle.forward(s["refs"], s["ref_idx"], s["target"], s["t_target"], s["mask"], p, arch) for s in samples]
    return ot.pretrain_loss(preds, [ot.ground_truth(s, arch.channels) for s in samples]), preds


@pytest.mark.parametrize("C", [3, 1])
def test_torch_forward_and_loss_equal_the_numpy_oracle(C):
    arch, blob, samples = _setup(C)
    loss, grad, preds = ot.loss_and_grad(blob, samples, arch)
    ref_loss, ref_preds = _numpy_loss(blob, samples, arch)
    for a, b in zip(preds, ref_preds):
        assert np.abs(a - b).max() < 1e-11
    assert abs(loss - ref_loss) < 1e-12 * max(1.0, abs(ref_loss))
    assert grad.shape == (len(blob),) and np.isfinite(grad).all()


def _pick(arch, names, rng, per=3):
    index = oracle.unpack_weights(np.arange(synth.weight_count(arch.channels, enc_depth=arch.enc_depth,
                                                               dec_depth=arch.dec_depth), dtype=np.float64), arch)
    out = []
    for n in names:
        flat = index[n].ravel().astype(np.int64)
        out += list(rng.choice(flat, per, replace=False))
    return index, out


@pytest.mark.parametrize("C", [3, 1])
def test_gradient_matches_central_differences_of_the_numpy_loss(C):
    arch, blob, samples = _setup(C, B=2)
    _, grad, _ = ot.loss_and_grad(blob, samples, arch)
    rng = np.random.default_rng(11)
    names = ["emb.w", "emb.b", "enc0.ln1.g", "enc0.qkv.w", "enc0.qkv.b", "enc0.proj.w", "enc1.ln2.b",
             "enc1.fc1.w", "enc1.fc2.w", "enc_norm.g", "e2d.w", "dec0.qkv.w", "dec0.fc2.b", "dec_norm.b"]
    index, picks = _pick(arch, names, rng, per=2)
    # head rows of the target time slot (the second half of the rows at T = 2)
    L = arch.tub_len
    head = index["head.w"].astype(np.int64)
    picks += [int(head[L // 2 + i, j]) for i, j in ((0, 0), (17, 5), (L // 2 - 1, arch.dec_dim - 1))]
    picks += [int(index["head.b"].astype(np.int64)[L // 2 + 7])]
    p = oracle.unpack_weights(blob, arch)
    where = {}
    for n, idx in index.items():
        for j, flat in enumerate(idx.ravel().astype(np.int64)):
            where[int(flat)] = (n, j)
    h = 1e-5
    for i in picks:
        n, j = where[int(i)]
        x0 = p[n].flat[j]
        p[n].flat[j] = x0 + h
        lu = _numpy_loss(None, samples, arch, p)[0]
        p[n].flat[j] = x0 - h
        ld = _numpy_loss(None, samples, arch, p)[0]
        p[n].flat[j] = x0
        fd = (lu - ld) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(abs(fd), 1e-3), (n, j, fd, grad[i])


def test_rows_of_the_other_time_slot_get_no_gradient():
    arch, blob, samples = _setup(3)
    _, grad, _ = ot.loss_and_grad(blob, samples, arch)
    p = ot.param_views(torch.from_numpy(grad), arch)
    L = arch.tub_len
    assert np.all(p["head.w"][:L // 2].numpy() == 0) and np.all(p["head.b"][:L // 2].numpy() == 0)
    assert np.abs(p["head.w"][L // 2:].numpy()).max() > 0
    for n in ("emb.w", "enc0.qkv.w", "enc1.fc2.w", "e2d.w", "dec0.proj.w", "dec_norm.g"):
        assert np.abs(p[n].numpy()).max() > 0, n


@pytest.mark.parametrize("C", [3, 1])
def test_gradient_equals_autograd_through_the_library_layer_network(C):
    arch, blob, samples = _setup(C, H=40, W=40, B=2)
    _, grad, _ = ot.loss_and_grad(blob, samples, arch)
    theta = torch.tensor(np.asarray(blob, np.float64), requires_grad=True)
    preds, gts = [], []
    for s in samples:
        preds.append(torch_reference.predict(s["refs"], s["ref_idx"], s["target"], s["t_target"], s["mask"], theta,
                                             C, ne=arch.enc_depth, nd=arch.dec_depth, as_tensor=True))
        gts.append(torch.from_numpy(ot.ground_truth(s, C)))
    terms = []
    for pr, g in zip(preds, gts):
        tv = (pr[:, 1:] - pr[:, :-1]).abs().mean() + (pr[1:] - pr[:-1]).abs().mean()
        terms.append(((pr - g) ** 2).mean() + 0.01 * tv)
    (sum(terms) / len(terms)).backward()
    ref = theta.grad.numpy()
    scale = np.abs(ref).max()
    assert np.abs(grad - ref).max() <= 1e-10 * scale


def test_loss_terms_on_a_known_prediction():
    """MSE + 0.01 TV on a ramp prediction against a constant frame: MSE and
    TV by hand; the loss is the mean over the batch."""
    H, W, C = 4, 5, 1
    ramp = np.tile(np.arange(W, dtype=np.float64)[None, :, None], (H, 1, C)) * 0.1   # x steps of 0.1, no y steps
    gt = np.full((H, W, C), 0.2)
    mse = np.mean((ramp - 0.2) ** 2)
    assert abs(ot.pretrain_loss([ramp], [gt]) - (mse + 0.01 * 0.1)) < 1e-15
    assert abs(ot.pretrain_loss([ramp, gt], [gt, gt]) - (mse + 0.001) / 2) < 1e-15
    t = torch.from_numpy(ramp).requires_grad_(True)
    ot.pretrain_loss_t([t], [torch.from_numpy(gt)]).backward()
    # d MSE / d p = 2 (p - g) / n; d TV / d p along x: (-1 at x = 0, +1 at x = W-1) / (H (W-1) C)
    expect = 2 * (ramp - 0.2) / ramp.size
    expect[:, 0] -= 0.01 / (H * (W - 1) * C)
    expect[:, -1] += 0.01 / (H * (W - 1) * C)
    assert np.abs(t.grad.numpy() - expect).max() < 1e-15


def test_adam_first_steps_closed_form():
    g = np.array([0.5, -2.0, 0.0, 1e-9])
    p = np.array([1.0, 1.0, 1.0, 1.0])
    z = np.zeros(4)
    lr, eps = 2e-4, 1e-8
    p1, m1, v1 = ot.adam_step(p, g, z, z, 1, lr)
    # step 1: m_hat = g and v_hat = g^2, so the step is lr g / (|g| + eps)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-16)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    # step 2 with gradient g2 by hand
    g2 = np.array([1.0, 1.0, 1.0, 1.0])
    p2, m2, v2 = ot.adam_step(p1, g2, m1, v1, 2, lr)
    m = 0.9 * 0.1 * g + 0.1 * g2
    v = 0.999 * 0.001 * g * g + 0.001 * g2 * g2
    mh, vh = m / (1 - 0.81), v / (1 - 0.999 ** 2)
    assert np.allclose(p2, p1 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-16)
    assert ot.ADAM_LR == 2e-4 and math.isclose(ot.ADAM_BETA1, 0.9) and math.isclose(ot.ADAM_BETA2, 0.999)
