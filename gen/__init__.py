"""Seeded synthetic survival data shared by the tests, the smoke check and
the benchmark.  Holds no arithmetic of the method itself (no risk sets, no
likelihood, no weights): it only draws covariates, coefficients and times.
"""
from .survival import (  # noqa: F401
    indicator_design, cox_data, fg_data, uniform_tuple_data, force_ties,
    dense_column, linear_predictor, csc_from_dense, cv_folds,
)
