"""FP64 CPU oracle for TASER (arXiv:1609.01797) -- TEST INFRASTRUCTURE ONLY.

This package is the independent, slow, obviously-correct reference that the
HIP path is checked against.  It is written from the paper's equations and
Algorithm 1, in float64 numpy (and plain PyTorch CPU for the unfolded
autograd reference).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path never
does, and this package never imports the product package.

Functions without an external pin say "parity unpinned" in their docstring;
every function here is pinned by a ``-m "not gpu"`` test (closed forms,
invariants, brute force, Table I's operation count, exact symmetries).
"""
from .taser import (BPSK, QPSK, COHERENT, JED, VEC_DEGENERATE, VEC_NONFINITE,  # noqa: F401
                    VEC_ZERO_NORM, VEC_VNN_NONPOS, problem_size,
                    real_decomposition_coherent, real_decomposition_jed,
                    build_T_coherent, build_T_jed, precondition, spectral_norm,
                    step_size, objective, taser_iterate, slice_decisions, backmap,
                    run_taser, detect_coherent, detect_jed)
