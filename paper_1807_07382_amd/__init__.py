"""pentbatch for MI355X: batched pentadiagonal solves (one matrix factored once,
many right-hand sides in the interleaved batch-fastest layout) on gfx950.

The solver is the HIP library ``libpentbatch.so`` (C ABI declared in
``include/pentbatch.h``); :mod:`paper_1807_07382_amd.pentbatch` is a thin
ctypes binding over it.  Importing this package loads nothing; the library
is opened on first use and a missing library is an error, never a fallback.
"""
__all__ = ["pentbatch", "inputs"]
