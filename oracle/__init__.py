"""Plain, slow CPU oracle of the PM-LSH query path (FP64, NumPy).

TEST INFRASTRUCTURE ONLY. Nothing in the GPU library or its Python binding
imports this package; only the test suite, the package smoke check and the
CPU-baseline leg of the benchmark may call it. It shares no code with the
HIP/C++ implementation: the only common input is the seeded workload module
``synth``, which draws random numbers and computes nothing of the method.

Modules
  chi2     chi-square CDF/survival/quantile and the parameter setting of
           Lemma 3 and Eq. 10 (t, alpha2, beta, budgets)
  rmin     the r_min rule of Section 5.2 (distance-distribution quantile)
  ann      (c,k)-ANN, Algorithm 2, one query at a time
  bc       (r,c)-BC, Algorithm 1, one query at a time
  acp      (c,k)-ACP by radius filtering (Section 6.3), canonical form
  brute    exact kNN and exact k closest pairs, straight from Defs. 1-4
  metrics  overall ratio and recall, Eqs. 12-14

Every function cites the passage it follows. Readings of passages where the
paper is silent or ambiguous are stated where they are applied.
"""

from . import chi2, rmin, ann, acp, brute, metrics  # noqa: F401
