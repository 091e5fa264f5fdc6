"""Seeding helpers shared by every generator."""

import numpy as np

#: Global seed of every synthetic stream (the paper's arXiv number).
SEED = 161207875

#: Fourth seed word used for per-stream static parameters (never a frame index).
STATIC = 2**31 - 1


def frame_rng(cfg: int, stream: int, t: int) -> np.random.Generator:
    """Generator for the random content of frame ``t`` of one stream."""
    return np.random.default_rng([SEED, int(cfg), int(stream), int(t)])


def static_rng(cfg: int, stream: int) -> np.random.Generator:
    """Generator for the static parameters of one stream."""
    return np.random.default_rng([SEED, int(cfg), int(stream), STATIC])
