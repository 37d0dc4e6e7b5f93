"""MI355X-native multilevel Monte Carlo for x = exp(beta A) u (arXiv:1904.12754).

The compute path is the C-ABI library libmlmc_expv.so (HIP kernels for gfx950, declared
in include/mlmc_expv.h); `api.Plan` is its Python binding. Importing this package does
not load the library; `api` does, and raises if it is missing.
"""
__all__ = ["api", "inputs", "build"]
