"""MI355X (gfx950) implementation of the SketchNE hot path.

The compute lives in ``libsketchne.so`` (hand-written HIP kernels behind the
C ABI declared in ``include/sketchne.h``).  ``binding`` is a thin ctypes layer
that marshals PyTorch device tensors into those calls; it performs no
arithmetic of the method itself.
"""
