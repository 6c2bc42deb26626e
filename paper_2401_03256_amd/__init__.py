"""Dynamic Frontier PageRank on MI355X (gfx950).

The compute path is the C-ABI library ``libdfpr.so`` (HIP kernels, declared
in ``include/dfpr.h``); ``paper_2401_03256_amd.dfpr`` is its thin Python
binding and ``paper_2401_03256_amd.synth`` the seeded input generators.
Importing this package loads nothing; the library is opened on first use.
"""
__all__ = ["dfpr", "synth"]
