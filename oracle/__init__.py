"""Plain FP64 CPU oracle for stochastic Lanczos quadrature (SLaQ, arXiv 2003.01282).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package;
only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the HIP library: it has its own probe generator (SplitMix64
written from its published definition), its own Laplacian, its own Lanczos
recurrence and uses LAPACK (through numpy) for the small tridiagonal
eigenproblems.

Modules
-------
slq      the method itself: graph quantities, probes, Lanczos, Gauss rule,
         heat / wave trace and von Neumann graph entropy.
exact    test-only ground truth: dense Laplacian, full spectrum, brute-force
         Hutchinson on the same probes.
radau    Gauss-Radau companion rule, the upper end of the per-probe bracket.
mlp      FP64 forward/backward of the closure network (reference for the
         gradient checks of the BF16 kernels).

Every function names the passage of the paper it follows.  Readings of places
where the paper is silent or garbled are listed in each function's docstring.
"""
from . import slq, exact, radau  # noqa: F401
