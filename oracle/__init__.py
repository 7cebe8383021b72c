"""FP64 CPU oracle for the SketchNE hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the GPU
library (no kernels, headers, helpers or constant tables); the only inputs
the two sides share are the seeded draws from ``synth``.

It is deliberately plain and slow: NumPy/SciPy in float64, each step written
in the order and notation of the paper (SketchNE, TKDE 2023, arXiv
2110.12782):

* ``netmf``    -- Eq. (1) (the NetMF matrix), Eq. (2), Eq. (11) factors,
                  the truncated logarithm (Section 2, Section 3.2).
* ``freigs``   -- Alg. 5 (fast randomized eigendecomposition) with eigSVD
                  and QR orthonormalisation (Section 3.2).
* ``sketch``   -- Alg. 3 as a dense matrix, Eq. (4) column sampling, the
                  two sketches Y and Z of Alg. 4, and the reduced matrix W /
                  SVD of Alg. 4 (Section 3.1).
* ``pipeline`` -- Alg. 6 lines 1-5 and Alg. 1 (exact NetMF, for context).
* ``propagation`` -- Alg. 6 line 6, spectral propagation by a Chebyshev
                  polynomial of the random-walk Laplacian (coefficients read
                  from ProNE's band-pass filter; see that module).
* ``metrics``  -- relative Frobenius error and principal angles.
* ``mlp``      -- the warm-start MLP (not from the paper: parity unpinned
                  against the paper, pinned by finite differences).
"""
from . import netmf, freigs, sketch, pipeline, metrics, mlp, propagation  # noqa: F401
