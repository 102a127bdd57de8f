"""Dense CPU oracle for the fast multitask-GP hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
executes this package; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP path: it
generates the design points by their defining digit loops, assembles the
dense N x N Gram matrix, and factors it with LAPACK (float64) or with the
companion C twin in extended precision (``hp_dense.c``).

Modules
-------
points   rank-1 lattices (Def. "Shifted rank-1 lattice") and base-2 digital
         sequences (Def. "Base-2 digitally-shifted digital sequences").
kernels  SI Bernoulli kernels (Eq. SI_kernel_1d_ex), adaptive-smoothness DSI
         kernels (Eq. DSI_kernel_1d_ex), the product form (Eq. prod_kernel)
         and the multitask product (Eq. mtprod).
dense    Gram matrix, MLE loss, optimal means, gradient, posterior mean
         (Eqs. MTGP_post_mean_cov, MTGP_MLE_GCV_loss, MTGP_optimal_tau).
hp       ctypes front-end of the extended-precision twin.
spectral equal-size MLE loss through the per-frequency blocks of Theorem
         "Fast MTGP computations" (numpy Walsh / DFT, O(T^3 n + T^2 n log n));
         pinned to ``dense``, it carries loss parity beyond dense sizes.

Parity status per function is listed in the module docstrings; every
function here is pinned by a ``-m "not gpu"`` test except where its
docstring says "parity unpinned".
"""
from . import points, kernels, dense  # noqa: F401
