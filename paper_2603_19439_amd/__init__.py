"""G-REST eigenpair tracking on MI355X (gfx950).

The update runs in the HIP library ``libgrest.so`` behind the C interface in
``include/grest.h``; ``paper_2603_19439_amd.grest`` is its thin ctypes binding.
Importing this package loads nothing; the library is loaded on first use.
"""
__all__ = ["grest", "workloads", "metrics"]
