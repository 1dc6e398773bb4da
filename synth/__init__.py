"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module draws inputs only: RGB-D scenes, packet-loss masks and He-normal
weight blobs. It holds none of the recovery method's arithmetic, so both the
FP64 oracle and the HIP path may import it without sharing any computation.
"""
from .scene import scene_frames, perlin2d
from .masks import stripe_mask, gilbert_elliott_masks, ge_params
from .weights import model_shapes, make_weights, weight_count
from .requests import make_request, make_batch, make_calibration_set, make_pretrain_batch

__all__ = [
    "scene_frames", "perlin2d", "stripe_mask", "gilbert_elliott_masks", "ge_params",
    "model_shapes", "make_weights", "weight_count", "make_request", "make_batch", "make_calibration_set",
    "make_pretrain_batch",
]
