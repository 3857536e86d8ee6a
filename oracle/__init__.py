"""FP64 CPU oracle for trace-regularized FCTN tensor completion solved by PAM.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import
this package.  The GPU library never calls it, links it or falls back to it,
and this package imports nothing from the GPU library.

Every function here is a plain, slow restatement of the paper (arXiv
2510.22506, "Accelerated Tensor Completion via Trace-Regularized
Fully-Connected Tensor Network") in float64, with NumPy/LAPACK primitives as
single steps:

* ``tensor``     Definitions 1-3 (generalized transpose, unfolding,
                 contraction), the FCTN element formula (Section 1) and
                 Property 1 (sub-network M_k).
* ``laplacian``  the periodically modified negative Laplacian L_k (Section 3.1)
                 and its Fourier diagonalization (eq. 7).
* ``sylvester``  the factor subproblem: Sylvester equation (eq. 5), its
                 Kronecker form (eq. 6) and the fast solution (Theorem 1,
                 eq. 8), plus the generalized fold (eq. 9).
* ``pam``        Algorithm 1 (PAM-FCTNLR) and Algorithm 2 (PAM-AFCTNLR with
                 intermediate-tensor reuse), the X update (eq. 10), the
                 stopping rule and the objective f (Section 3.5), with flop
                 counters for the complexity tables (Tables 1-2).
* ``metrics``    PSNR as defined in Section 4.

Pinning: every function is checked in ``tests/test_oracle_*.py`` against
something other than itself (brute-force index sums, closed forms, exact
block-decrease identities, the Eckart-Young bound, Table 1-2 counts).
Parity unpinned: the paper's PSNR/SSIM/runtime on its real datasets (absent),
and the exact schedules drawn in the missing figures: the permutation of
Figure 6 and the group chain for N >= 5 are readings constrained only by the
Table 1 and Table 2 counts, which they reproduce.
"""

from . import tensor, laplacian, sylvester, pam, metrics  # noqa: F401
