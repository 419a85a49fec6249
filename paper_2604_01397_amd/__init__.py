"""MI355X (gfx950) implementation of the EXaCTz correction loop.

The work happens in ``libexactz.so`` (hand-written HIP, C ABI in
``include/exactz.h``); ``exactz`` is a thin ctypes binding that marshals torch
device tensors into it.  Importing the package does not load the library, so
that CPU-only tools (generators, tests) can import it; the first call that
needs the GPU loads it and fails loudly if it is missing.
"""
