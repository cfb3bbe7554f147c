"""MI355X-native hot path of the layer-case FDM transport scheme (arXiv:1911.03225).

The compute lives in ``libfdm.so`` (HIP for gfx950, C ABI declared in
``include/fdm.h``).  ``paper_1911_03225_amd.fdm`` is the thin ctypes binding
with the same entry-point names; importing this package loads nothing.
"""
