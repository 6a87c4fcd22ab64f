"""Seeded synthetic inputs: luma/chroma planes and loss masks.

This package holds input generation only.  It contains none of the
concealment arithmetic, so both the HIP product path and the CPU oracle can
read its arrays without sharing any method code.
"""
from .generator import (
    make_luma,
    make_chroma,
    loss_isolated,
    loss_dispersed,
    loss_random,
    loss_slices,
    loss_random_bursts,
    loss_partial_cells,
    workload_plain_512,
    workload_layered_1080p,
    workload_batch,
    workload_stream_4k,
    seed_for,
)

__all__ = [
    "make_luma", "make_chroma", "loss_isolated", "loss_dispersed", "loss_random",
    "loss_slices", "loss_random_bursts", "loss_partial_cells", "workload_plain_512",
    "workload_layered_1080p", "workload_batch", "workload_stream_4k", "seed_for",
]
