"""Seeded packet-loss masks (u8, H x W, 1 = pixel lost).

The paper tracks loss per packet and zero-fills what is missing (Sec. 3.3);
its pretraining uses random pixel masks (Sec. 3.4, robustness across codecs).
Without codecs or loss traces, loss is drawn per slice, where a slice is one
16-pixel macroblock row (a partial last row counts as a slice):

* stripe_mask: every slice lost independently with probability p.
* gilbert_elliott_masks: a two-state (Gilbert) chain over slices with mean
  loss L and mean burst length b: P(B->G) = 1/b, P(G->B) = L / (b (1 - L)).
  The first state is drawn from the stationary distribution, and the chain
  continues across consecutive frames of a stream.
"""
import numpy as np

SLICE_ROWS = 16


def _n_slices(height):
    return (int(height) + SLICE_ROWS - 1) // SLICE_ROWS


def _expand(lost_slices, height, width):
    rows = np.repeat(np.asarray(lost_slices, np.uint8), SLICE_ROWS)[: int(height)]
    return np.ascontiguousarray(np.broadcast_to(rows[:, None], (int(height), int(width))))


def stripe_mask(seed, height, width, p):
    """Each 16-row slice lost i.i.d. with probability p."""
    rng = np.random.default_rng(seed)
    lost = rng.random(_n_slices(height)) < p
    return _expand(lost, height, width)


def ge_params(mean_loss, burst):
    """(p_gb, p_bg) of the Gilbert chain with stationary loss L and mean burst b."""
    L, b = float(mean_loss), float(burst)
    return L / (b * (1.0 - L)), 1.0 / b


def gilbert_elliott_masks(seed, height, width, n_frames, mean_loss, burst):
    """Masks for n_frames consecutive frames from one Gilbert chain."""
    rng = np.random.default_rng(seed)
    p_gb, p_bg = ge_params(mean_loss, burst)
    ns = _n_slices(height)
    state_bad = rng.random() < mean_loss
    out = np.empty((int(n_frames), int(height), int(width)), np.uint8)
    for f in range(int(n_frames)):
        lost = np.empty(ns, bool)
        for s in range(ns):
            lost[s] = state_bad
            u = rng.random()
            state_bad = (u >= p_bg) if state_bad else (u < p_gb)
        out[f] = _expand(lost, height, width)
    return out
