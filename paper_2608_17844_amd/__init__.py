"""MI355X-native multilevel-block-Toeplitz MoM solver for large regular finite arrays.

The solver itself lives in the HIP library ``libmbt.so`` (include/mbt.h);
``mbt`` is its thin ctypes binding and ``workloads`` describes the seeded
synthetic inputs.  Importing the package does not load the library; the first
call into ``mbt`` does, and fails loudly if it has not been built.
"""
__all__ = ["mbt", "workloads"]
