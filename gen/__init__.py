"""Seeded synthetic snapshot streams for streaming method-of-snapshots DMD.

This package only *produces input data*.  It holds none of the method's
arithmetic (no inner products, eigensolves or projections), so it can be
shared by the FP64 oracle tests, the GPU parity tests and the benchmark
without coupling the two implementations.

Every frame is drawn from ``numpy.random.default_rng([SEED, cfg, stream, t])``
so any frame of any stream can be regenerated on its own; per-stream static
parameters (eigenvalues, blob tracks, wave numbers, Fourier amplitudes) come
from ``default_rng([SEED, cfg, stream, STATIC])``.

Workloads (the shapes of the paper's experiments, Sec. 4, with synthetic
content because the paper's video datasets are not available):

* :class:`ModalStream`      -- sum of damped complex modes plus noise (FP64).
* :class:`BlobVideo`        -- smooth background plus moving Gaussian blobs
                               plus pixel noise (FP32 "video").
* :class:`TravelingWaves`   -- 2-D flow of travelling Fourier modes with
                               amplitudes decaying by 10^(-k/2) (FP32).
* :class:`FourierSparse`    -- low-wavenumber Fourier coefficients of an
                               advected field, CSR complex64, with part of
                               the support redrawn every frame.
* :func:`stream_mix`        -- the parameters of a many-stream serving mix.
"""

from .common import SEED, STATIC, frame_rng, static_rng
from .modal import ModalStream
from .video import BlobVideo
from .flow import TravelingWaves
from .fourier import FourierSparse
from .mix import stream_mix, MixStream

__all__ = [
    "SEED", "STATIC", "frame_rng", "static_rng",
    "ModalStream", "BlobVideo", "TravelingWaves", "FourierSparse",
    "stream_mix", "MixStream",
]
