"""MI355X-native hot path of the sketched generalized Krylov subspace method (sGKS).

The solver lives in the HIP library ``_lib/libsgks.so`` (C ABI in include/sgks.h);
``paper_2606_18073_amd.sgks`` is its ctypes binding.
"""
__all__ = ["sgks"]
