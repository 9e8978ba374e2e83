"""Reference oracle for the rank-Greville recursive least-squares update.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
runs anything in this directory; only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark do.  The oracle shares no code with the HIP
path: it has its own arithmetic, its own storage and its own build.

Contents
--------
rg_ref.py      Algorithm 1 written out over Python scalars (``fractions.Fraction``
               or ``float``), the exact row-space least-squares solver, SVD
               references, Theorem 1 and the Penrose checks.
rg_ref.c       The same Algorithm 1 as a plain FP64 C loop (the timed CPU
               baseline), with a thread pool over independent streams.
ref_c.py       ctypes loader for the compiled ``rg_ref.c``.
adjoint_ref.py Constant-rank pseudoinverse derivative (FP64, SVD based) and
               central finite differences through the rank-r truncated solve.
"""
