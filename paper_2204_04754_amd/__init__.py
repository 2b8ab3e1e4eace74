"""MI355X (gfx950) EM step for 2-D super-resolution multi-reference alignment.

The compute path is the HIP library libsrmra.so (C ABI in include/srmra.h);
`binding` is its thin ctypes mirror and `em` a small driver that owns device
buffers.  Importing this package does not load the library; the first call
that needs it does, and fails loudly if it is not built.
"""
__all__ = ["binding", "em", "synth"]
