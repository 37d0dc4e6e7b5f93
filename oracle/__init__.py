"""Oracle for the MLMC estimator of x = exp(beta*A) u (arXiv:1904.12754).

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import, call or execute anything in this package; the product path
(the C-ABI library and its Python binding) never does, and shares no code with it.

Contents:
  mlmc_oracle.c  plain FP64 C: Philox4x32-10, the logarithm used for the exponential
                 holding times, the decomposition A = D - T, alias tables, one sample
                 of Algorithm 2, per-row level sums.
  mlmc.py        ctypes binding, the MLMC combine (section 2.2, the telescoping
                 estimator) and Algorithm 1's driver.
  reference.py   deterministic FP64 references used to pin the oracle: dense exp(tA)
                 (library routine), dense Strang-split level products (section 2.1),
                 closed forms for Laplacians.
"""
