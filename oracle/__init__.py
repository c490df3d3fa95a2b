"""Plain FP64 CPU oracle for subquadratic Kronecker regression.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
executes anything here; only the test suite, the smoke check and the benchmark's
CPU-baseline leg may.  The oracle shares no code with the HIP path: every step is
restated from the paper (Fahrbach, Fu, Ghadiri, "Subquadratic Kronecker
Regression with Applications to Tensor Decomposition", NeurIPS 2022) in plain
NumPy float64, in the paper's order and notation, with no blocking, fusion or
reordering beyond what each definition states.

Modules
  philox      Philox4x64-10 counter-based generator (Salmon et al., SC'11).
  kron        mode-n products, explicit Kronecker products, KronMatMul
              (Lemma kron_mat_mul), vec/unfolding conventions.
  leverage    statistical and ridge leverage scores (Section 3), the integer
              quantisation of the sampling distribution and its CDF.
  sampling    RowSampling (Definition def:sample_rows_alg) on the product
              distribution of Lemma kronecker_cross_leverage_scores.
  regression  Algorithm 2 (FastKroneckerRegression): the sketched problem, its
              direct minimiser, the preconditioned Richardson replay, the exact
              optimum (KronMatMul baseline) and the loss.
  response    implicit responses b = K X_true + sigma E (Philox Box-Muller
              noise indexed by row), for workloads whose dense b is too large.
  tucker      Algorithm 3 (FastFactorMatrixUpdate), the Woodbury form of its
              preconditioner, exact factor-row solutions and exact Tucker ALS
              (Algorithm 1).

Parity status of every function is stated in its docstring ("pinned by ..."
names the test that ties it to something other than itself).
"""

from . import philox, kron, leverage, sampling, regression, tucker, response  # noqa: F401
