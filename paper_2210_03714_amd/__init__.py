"""pfm: parallel fractional matrix functions on MI355X (gfx950).

GPU implementation of the shifted-solve rational method of Blanes,
"Parallel computation of functions of matrices and their action on vectors"
(arXiv:2210.03714): f(A) and f(A)V for exp and phi1 as a fixed linear
combination of m independent shifted solves (I - c_k B)^{-1} B, with
scaling-and-squaring (full matrix) or an N-step recurrence (action).

The compute path lives in the C-ABI library ``libpfm.so`` (HIP kernels for
gfx950); ``paper_2210_03714_amd.pfm`` is its thin ctypes binding.  Importing
this package does not load the library; ``workloads`` is the seeded input
generator shared with the tests.
"""

__all__ = ["pfm", "workloads"]
