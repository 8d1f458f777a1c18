"""Sliced big-head tensor-network contraction on MI355X (gfx950).

The computation lives in the HIP library libtnsim.so behind the C ABI of
include/tn.h; `tn` is its ctypes binding and `runtime` wraps it with torch
device memory and streams.  Importing this package does not load the library;
`tn.library()` does, and fails loudly when it has not been built.
"""
