"""Seeded synthetic inputs for the Nystrom PCG workloads.

This module only draws random numbers and lays them out (shapes, dtypes,
scalings of the data itself).  It performs none of the method's arithmetic:
no kernel evaluation, no matrix-vector product, no sketch, no solve.  Right-hand
sides that are defined through the operator (``b = K w + 0.01 eps`` or
``b = X^T y``) are returned as their random ingredients; whoever consumes them
(the CPU oracle in tests, the device operator in the benchmark) assembles ``b``.

Both the CPU oracle and the HIP path take their inputs from here, so the two
solve the identical system.  The recipes stand in for the paper's datasets
(Section 6: regularisation path on Guillermo-shaped data, random-features
ridge regression with l = 800, kernel ridge regression at n ~ 1e5 with
l = 1000); no dataset item is reproduced.
"""
from .synth import (  # noqa: F401
    gaussian_test_matrix,
    column_sample,
    krr_small,
    ridge_dense,
    krr_mixture,
    batched_cv,
    differentiation,
    spectrum_psd,
    lowrank_psd,
    logistic_weights,
)
