"""Seeded synthetic two-view workloads.

This package only manufactures inputs: cameras, a fundamental matrix built
from them (Eq. 1 of the paper), noisy keypoints with a ground-truth map, and
descriptors in the storage formats the matcher accepts.  It contains none of
the matching method's arithmetic (no point-line distances, no angular
intervals), so the CPU oracle and the GPU path can both draw their inputs from
it without sharing any computation.
"""

from .pairs import (  # noqa: F401
    Pair,
    PairBatch,
    batch_pairs,
    cfg0_pair,
    cfg1_pair,
    cfg2_pair,
    cfg3_batch,
    cfg3_pair,
    cfg4_pair,
    fundamental_from_cameras,
    intrinsics,
    make_pair,
    noise_covariance,
    perturbed_F,
    perturbed_pose,
    rot_axis_angle,
    skew,
)
from .mlp_init import mlp_init  # noqa: F401
from .quant import bf16_to_f32, f32_to_bf16, f32_to_fp8_e4m3, fp8_e4m3_to_f32  # noqa: F401
