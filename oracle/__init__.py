"""Plain FP64 CPU oracle for the two-level additive Schwarz preconditioner of
Al Daas, Jolivet, Nataf and Tournier, "A robust two-level Schwarz
preconditioner for sparse matrices" (arXiv 2401.03915).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute anything under ``oracle/``: only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it. It shares no code with the GPU
library (no kernels, helpers, tables or pre/post-processing); the two only
read the same seeded inputs from ``workloads``.

It computes the paper's definitions literally, in float64, with NumPy/SciPy:

* ``schwarz``  - overlap layers (Section 2.1), local matrices and one-level
  Schwarz (Section 2.3), the harmonic operator (eq. HOp), the two local
  generalized eigenproblems (eq. uppergevp, eq. gevpsvd), the nonsymmetric
  variant (Section 6), the coarse space (eq. coarse_space_2), the Galerkin
  coarse operator and the two-level apply (Remark in Section 4.3);
* ``krylov``   - PCG and right-preconditioned flexible GMRES;
* ``pool``     - the same setup, apply and solve with the per-subdomain work
  spread over worker processes (for the benchmark-size configurations);
* ``gnn``      - forward, loss and backward of the warm-start network of
  the local eigensolver (not in the paper; see its docstring);
* ``theory``   - brute-force objects for tiny inputs: the SPSD splitting
  (Lemma spsd_splitting), colors k_c, lambda_* (eq. lambda_star), the
  condition-number bounds (Theorems upper_bound_1 and upper_bound_2) and the
  dense spectrum of M^{-1} A.

Parity status of each function is stated in its docstring; functions whose
result nothing independent fixes say "parity unpinned".
"""

from . import gnn, krylov, pool, schwarz, theory  # noqa: F401
from .schwarz import Handle, apply, setup, solve  # noqa: F401
