"""FP64 CPU oracle for the in-solve algebraic coarsening linear solve.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import anything from this package.  The
product path (the HIP library and its Python binding) never calls it and
shares no code with it.

What it computes, after "AGIPC: Adaptive In-Solve Algebraic Coarsening for
GPU IPC" (Wang, Luo, Li, Komura, Huang; SIGGRAPH 2026):

* ``aggregate``  - the fine-to-coarse map (Sec. 4.1 "Adaptive Coarsening via
  Edge Collapse"; supplement Sec. 1, Alg. 1-2 and the worked examples of
  Sec. 1.2-1.3): connected components of the collapsible-edge graph,
  labelled in increasing order of their smallest fine vertex id.
* ``galerkin``   - the coarse system H_c = U H U^T, g_c = U g with U = P^T
  (Sec. 4.1 "Algebraic Coarsening and System Assembly"; supplement Sec. 2).
* ``solve``      - the coarse solve d_c = H_c^{-1} g_c (Alg. overview, solve
  step; Sec. 5.1 "Preconditioners": 3x3 block-Jacobi PCG) and the
  prolongation d_f = U^T d_c (Sec. 4.3).
* ``adjoint``    - derivatives of L(x) with x = P H_c^{-1} P^T g with respect
  to g and to every element block.
* ``method``     - the four steps chained in the order of Alg. overview.

Everything is float64.  Sign convention: the oracle returns
x = P H_c^{-1} P^T g; the Newton direction is d = -x.
"""
from . import aggregate, galerkin, solve, adjoint, method  # noqa: F401
