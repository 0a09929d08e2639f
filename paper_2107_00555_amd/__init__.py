"""Fused reaction-diffusion array program on MI355X (gfx950).

The GPU work lives in the HIP library ``libdcp.so`` behind the C ABI declared
in ``include/dcp.h``; the modules here only marshal torch tensors into it.
"""
