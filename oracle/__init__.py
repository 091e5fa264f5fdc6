"""FP64 CPU oracle for streaming method-of-snapshots DMD.

TEST INFRASTRUCTURE ONLY.  This package is imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``;
the HIP library and its Python binding never import, call or link it, and it
shares no code with them (only the input generators in ``gen/`` serve both).

What it computes, in FP64 (complex128 for complex data), with NumPy/SciPy
LAPACK routines as the only library steps:

* :func:`gram`           -- the inner-product matrix X^* X (Sec. 2.1).
* :func:`exact_dmd`      -- exact DMD by the SVD route: thin SVD of X,
                            A~ = U^* X' V Sigma^-1 (Eq. Atilde),
                            A~ W = W Lambda, Phi = X' V Sigma^-1 W (Eq. Phi),
                            truncated to rank r (Tu et al.'s exact DMD,
                            cited in Sec. 2.2).  This is the standard
                            algorithm the streaming method must reproduce.
* :func:`mos_svd`        -- method-of-snapshots SVD (Sec. 2.1): eig of X^* X,
                            sigma = sqrt(|eig|), U = X V Sigma^-1.
* :class:`StreamingMoS`  -- Algorithms 1 and 2 (streaming SVD and DMD) with
                            the shift-and-new-column Gram update of Sec. 3.1,
                            in FP64; a self-check of the method and the
                            streaming CPU baseline.
* :mod:`oracle.metrics`  -- error metrics (singular-value relative error,
                            matched eigenvalue error, mode angles).
* :mod:`oracle.background` -- mode amplitudes b = (W Lambda)^-1 alpha_1 and
                            the background/foreground split of the newest
                            snapshot (Sec. 3.3, Algorithm 3).
* :mod:`oracle.fourier`  -- the spatial -> Fourier ingest of the sparse path
                            (Sec. 3.5): unitary 2-D DFT and the lowest-|k|
                            support.

Readings of the paper that this oracle fixes (where the paper is silent):
the window holds m+1 snapshots (X = first m, X' = last m); rank truncation
to the r largest singular values (rank r_eff if fewer are resolvable);
conjugate transposes throughout; eigenvalues sorted by descending modulus
(ties: ascending argument); eigenvector columns of unit 2-norm with their
largest-modulus entry real and positive.
"""

from .dmd import (
    as_fp64, gram, mos_svd, exact_dmd, StreamingMoS, DMDResult,
    canonical_columns, sort_eigs, r_effective, default_rcond, pod_modes,
    dmd_from_gram, densify,
)
from . import metrics
from . import background
from . import fourier

__all__ = [
    "as_fp64", "gram", "mos_svd", "exact_dmd", "StreamingMoS", "DMDResult",
    "canonical_columns", "sort_eigs", "r_effective", "default_rcond", "pod_modes",
    "dmd_from_gram", "densify", "metrics", "background", "fourier",
]
