"""The pretraining step on the GPU (include/revo_train.h) against the FP64
oracle (oracle.train): loss, raw prediction, the gradient of every
parameter tensor, and the Adam-updated weights, element by element
(Sec. 3.4.2 L_RGB on randomly masked frames for both models; Sec. 4 Adam,
lr 2e-4)."""
import numpy as np
import pytest
import torch

import oracle
import oracle.train as ot
import synth

pytestmark = pytest.mark.gpu

TINY = dict(enc_depth=2, dec_depth=1)


def _dev(samples, C):
    refs = np.stack([s["refs"] for s in samples])
    target = np.stack([s["target"] for s in samples])
    mask = np.ascontiguousarray(np.stack([s["mask"] for s in samples]))
    if C == 1:
        refs, target = refs.view(np.int16), target.view(np.int16)
    return (torch.from_numpy(np.ascontiguousarray(refs)).cuda(), torch.from_numpy(np.ascontiguousarray(target)).cuda(),
            torch.from_numpy(mask).cuda(), np.stack([s["ref_idx"] for s in samples]),
            np.array([s["t_target"] for s in samples]))


def _tensor_errors(got, ref, arch):
    """max |got - ref| / max |ref| per parameter tensor of the blob."""
    index = oracle.unpack_weights(np.arange(ref.size, dtype=np.float64), arch)
    out = {}
    for name, idx in index.items():
        sl = idx.ravel().astype(np.int64)
        scale = np.abs(ref[sl]).max()
        out[name] = (float(np.abs(got[sl].astype(np.float64) - ref[sl]).max()), float(scale))
    return out


def _check_grads(got, ref, arch, rtol):
    worst = 0.0
    for name, (err, scale) in _tensor_errors(got, ref, arch).items():
        if scale == 0.0:
            assert err == 0.0, name            # e.g. head rows of the other time slot
            continue
        worst = max(worst, err / scale)
        assert err <= rtol * scale, (name, err, scale)
    return worst


def _check_update(new_gpu, new_ref, grad_ref, lr):
    """Adam moves each weight by at most about lr; where the gradient is well
    away from eps the GPU's step matches the oracle's to a small fraction of
    lr (near |g| ~ eps the step lr g / (|g| + eps) is ill-conditioned)."""
    d = np.abs(new_gpu.astype(np.float64) - new_ref)
    assert d.max() <= 1.05 * lr, d.max()
    well = np.abs(grad_ref) > 1e-5
    assert d[well].max() <= 0.02 * lr, d[well].max()


@pytest.mark.parametrize("C", [3, 1])
def test_one_step_matches_the_oracle(C):
    from paper_2604_27441_amd import Trainer
    arch = oracle.Arch(channels=C, **TINY)
    blob = synth.make_weights(5, perturb_seed=6, **TINY)[0 if C == 3 else 1]
    samples = synth.make_pretrain_batch(7, 3, 88, 120, C)     # ragged: 6 x 8 patches, 144 tokens
    ref = ot.train_step(blob, samples, arch)
    with Trainer(blob, C, 3, 88, 120, **TINY) as tr:
        loss = tr.step(*_dev(samples, C))
        grad, pred, new = tr.grads(), tr.pred(), tr.weights()
    print(f"C={C}: loss {loss:.8g} (oracle {ref['loss']:.8g})")
    assert abs(loss - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    for b in range(3):
        assert np.abs(pred[b] - ref["preds"][b]).max() <= 2e-5 * max(1.0, np.abs(ref["preds"][b]).max())
    worst = _check_grads(grad, ref["grad"], arch, rtol=2e-5)
    print(f"C={C}: worst per-tensor gradient error {worst:.3g} of the tensor's max")
    _check_update(new, ref["params"], ref["grad"], ot.ADAM_LR)


def test_full_depth_step_matches_the_oracle():
    from paper_2604_27441_amd import Trainer
    arch = oracle.Arch(channels=3)
    blob = synth.make_weights(8, perturb_seed=9)[0]
    samples = synth.make_pretrain_batch(10, 2, 64, 96, 3)
    ref = ot.train_step(blob, samples, arch)
    with Trainer(blob, 3, 2, 64, 96) as tr:
        loss = tr.step(*_dev(samples, 3))
        grad, new = tr.grads(), tr.weights()
    assert abs(loss - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    worst = _check_grads(grad, ref["grad"], arch, rtol=2e-5)
    print(f"12 + 4 blocks: worst per-tensor gradient error {worst:.3g} of the tensor's max")
    _check_update(new, ref["params"], ref["grad"], ot.ADAM_LR)


def test_three_steps_follow_the_oracle():
    """Moments and bias corrections carry across steps (t = 1, 2, 3), each
    step on a new batch."""
    from paper_2604_27441_amd import Trainer
    arch = oracle.Arch(channels=1, **TINY)
    blob = synth.make_weights(11, perturb_seed=12, **TINY)[1]
    params, m, v = np.asarray(blob, np.float64), None, None
    losses = []
    with Trainer(blob, 1, 2, 48, 64, **TINY) as tr:
        for step in range(1, 4):
            samples = synth.make_pretrain_batch(20 + step, 2, 48, 64, 1)
            ref = ot.train_step(params, samples, arch, m, v, step)
            params, m, v = ref["params"], ref["m"], ref["v"]
            losses.append((tr.step(*_dev(samples, 1)), ref["loss"]))
        new = tr.weights()
    for got, want in losses:
        assert abs(got - want) <= 1e-4 * abs(want), losses
    d = np.abs(new.astype(np.float64) - params)
    assert d.max() <= 3 * 1.05 * ot.ADAM_LR
    assert np.median(d) <= 0.01 * ot.ADAM_LR


def test_shapes_and_arguments_are_checked():
    from paper_2604_27441_amd import Trainer
    from paper_2604_27441_amd._lib import RevoError
    blob = synth.make_weights(5, **TINY)[0]
    with pytest.raises(RevoError):
        Trainer(blob[:-1], 3, 1, 32, 32, **TINY)          # wrong blob size
    with pytest.raises(RevoError):
        Trainer(blob, 2, 1, 32, 32, **TINY)               # channels 3 or 1
    with pytest.raises(RevoError):
        Trainer(blob, 3, 1, 32, 32, k=8, **TINY)          # k + 1 frames beyond the limit


def test_step_at_the_benchmark_frame_size():
    """256 x 192 frames (576 tokens: nine 64-key blocks, five 128-query
    tiles), 12 + 4 blocks, the depth model, batch 2 (bench.py times batch 8
    of the same frames)."""
    from paper_2604_27441_amd import Trainer
    arch = oracle.Arch(channels=1)
    blob = synth.make_weights(0)[1]
    samples = synth.make_pretrain_batch(30, 2, 192, 256, 1)
    ref = ot.train_step(blob, samples, arch)
    with Trainer(blob, 1, 2, 192, 256) as tr:
        loss = tr.step(*_dev(samples, 1))
        grad, new = tr.grads(), tr.weights()
    assert abs(loss - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    worst = _check_grads(grad, ref["grad"], arch, rtol=2e-5)
    print(f"256x192 depth: worst per-tensor gradient error {worst:.3g} of the tensor's max")
    _check_update(new, ref["params"], ref["grad"], ot.ADAM_LR)


@pytest.mark.parametrize("C,k,T", [(3, 2, 1), (1, 4, 3)])
def test_tubelet_variants_match_the_oracle(C, k, T):
    """T = 1 (the head's target slot is the whole head, so its weight and
    bias gradients share one chunk sum like every other layer) and T = 3 with
    k + 1 = 5 frames padded to 6 with the oldest reference."""
    from paper_2604_27441_amd import Trainer
    arch = oracle.Arch(channels=C, k=k, tubelet=T, **TINY)
    blob = synth.make_weights(13, tubelet=T, perturb_seed=14, **TINY)[0 if C == 3 else 1]
    samples = synth.make_pretrain_batch(15, 2, 64, 80, C, k=k)
    ref = ot.train_step(blob, samples, arch)
    with Trainer(blob, C, 2, 64, 80, k=k, tubelet=T, **TINY) as tr:
        loss = tr.step(*_dev(samples, C))
        grad, new = tr.grads(), tr.weights()
    assert abs(loss - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    worst = _check_grads(grad, ref["grad"], arch, rtol=2e-5)
    print(f"C={C} k={k} T={T}: worst per-tensor gradient error {worst:.3g} of the tensor's max")
    _check_update(new, ref["params"], ref["grad"], ot.ADAM_LR)


def test_batch_gradient_is_the_mean_of_its_halves():
    """At batch 16 (9216 token rows, past what the oracle can check in a
    test), the loss is the batch mean, so the step's loss and gradient equal
    the means of the two half batches' losses and gradients, each half run
    on its own trainer from the same weights (FP32 summation order aside)."""
    from paper_2604_27441_amd import Trainer
    blob = synth.make_weights(17)[1]
    samples = synth.make_pretrain_batch(40, 16, 192, 256, 1)
    with Trainer(blob, 1, 16, 192, 256) as tr:
        loss = tr.step(*_dev(samples, 1))
        g = tr.grads().astype(np.float64)
    parts = []
    for half in (samples[:8], samples[8:]):
        with Trainer(blob, 1, 8, 192, 256) as tr:
            parts.append((tr.step(*_dev(half, 1)), tr.grads().astype(np.float64)))
    want_loss = 0.5 * (parts[0][0] + parts[1][0])
    want = 0.5 * (parts[0][1] + parts[1][1])
    assert abs(loss - want_loss) <= 1e-5 * abs(want_loss), (loss, want_loss)
    arch = oracle.Arch(channels=1)
    worst = _check_grads(g.astype(np.float32), want, arch, rtol=1e-4)
    print(f"batch 16 against the mean of its halves: worst per-tensor gradient error {worst:.3g} of the tensor's max")


def test_steps_are_bit_identical_across_trainers():
    """Every sum in the step has a fixed order (row-chunk partials, their sums,
    the LayerNorm column sums, the loss partials), and the weight-gradient
    launches on the second stream are ordered by events against the input-
    gradient chain that reads and rewrites the same buffers; so two trainers
    from the same weights give bit-identical losses, gradients and weights
    over two steps at the benchmark's shape (256 x 192, batch 8, 12 + 4
    blocks). A missing ordering would show up here as differing bits."""
    from paper_2604_27441_amd import Trainer
    blob = synth.make_weights(19)[0]
    batches = [_dev(synth.make_pretrain_batch(50 + i, 8, 192, 256, 3), 3) for i in range(2)]
    runs = []
    for _ in range(2):
        with Trainer(blob, 3, 8, 192, 256) as tr:
            losses = [tr.step(*b) for b in batches]
            runs.append((losses, tr.grads(), tr.weights()))
    assert runs[0][0] == runs[1][0], (runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])
    assert np.array_equal(runs[0][2], runs[1][2])


def test_trainers_stepped_from_two_threads_match_sequential_steps():
    """The RGB and depth trainers stepped at once from two host threads (as
    bench.py times them) give the same bits as when stepped one after the
    other: each trainer owns its streams and buffers."""
    import threading

    from paper_2604_27441_amd import Trainer
    blobs = synth.make_weights(23)
    data = {C: _dev(synth.make_pretrain_batch(60 + C, 4, 192, 256, C), C) for C in (3, 1)}

    def one(C, out):
        with Trainer(blobs[0 if C == 3 else 1], C, 4, 192, 256) as tr:
            out[C] = (tr.step(*data[C]), tr.grads())

    seq, par = {}, {}
    for C in (3, 1):
        one(C, seq)
    threads = [threading.Thread(target=one, args=(C, par)) for C in (3, 1)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    for C in (3, 1):
        assert C in par, "a trainer thread failed"
        assert seq[C][0] == par[C][0], (C, seq[C][0], par[C][0])
        assert np.array_equal(seq[C][1], par[C][1]), C
