"""rank-Greville recursive least squares on MI355X (gfx950).

The per-row update of Staub & Steinmann's rank-Greville algorithm runs in
hand-written HIP kernels behind the C ABI declared in ``include/rg.h``
(``librg.so``); ``paper_2106_11594_amd.rg`` is the thin Python binding.
Importing this package does not load the library; ``rg`` does, and fails
loudly when it has not been built.
"""
__all__ = ["rg", "workloads"]
