"""FP64 CPU oracle of ReVo's neural loss-recovery forward pass.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import or call anything in this package.  It shares no
code with the HIP path: the only common module is ``synth`` (seeded inputs),
which holds none of the method's arithmetic.

Every function is a plain, slow, direct statement of one step of the method
(Sec. 3.4.1 architecture, App. B.1 design differences, App. B.3 k and T), in
float64 unless a rounding emulation is requested for error budgeting.
``metrics`` holds the frame quality metrics and the per-modality training
losses (Sec. 3.4.2, Sec. 4, Sec. 5.1); ``render`` the RGB-D unprojection and
z-buffered rendering of a new view (Sec. 2, Sec. 5).
"""
from .model import (
    Arch, unpack_weights, normalise, zero_fill, sequence_frames, tubelet_vectors,
    sinusoid, positional_embedding, linear, layer_norm, gelu, attention_head,
    self_attention, transformer_block, forward, place_target_slot, recover, composite, Rounding,
    bf16_round, e4m3_round, FP8Rounding, AbsMaxRecorder, pow2_scale, QK_LOG2,
)
from .metrics import (
    normalise_frame, gaussian_window, gaussian_filter_valid, ssim_map, ssim, total_variation, edge_loss,
    frame_metrics, METRIC_KEYS,
)
from .render import unproject, project, render_view
from . import train

__all__ = [
    "Arch", "unpack_weights", "normalise", "zero_fill", "sequence_frames", "tubelet_vectors",
    "sinusoid", "positional_embedding", "linear", "layer_norm", "gelu", "attention_head",
    "self_attention", "transformer_block", "forward", "place_target_slot", "recover", "composite", "Rounding",
    "bf16_round", "e4m3_round", "FP8Rounding", "AbsMaxRecorder", "pow2_scale", "QK_LOG2",
    "normalise_frame", "gaussian_window", "gaussian_filter_valid", "ssim_map", "ssim", "total_variation",
    "edge_loss", "frame_metrics", "METRIC_KEYS", "unproject", "project", "render_view",
]
