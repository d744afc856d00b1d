"""MI355X (gfx950) implementation of SpMV in the group-shared-exponent,
segmented-mantissa format and the stepped mixed-precision CG / GMRES solvers.

The compute lives in ``libgse.so`` (HIP, C ABI declared in ``include/gse.h``);
``paper_2411_04686_amd.gse`` is its ctypes binding.
"""
