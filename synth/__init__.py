"""Seeded synthetic inputs shared by the oracle, the tests and the bench.

This module draws random numbers and lays out locations; it holds none of the
likelihood method's arithmetic (no covariance, no factorisation, no ordering).
Both the CPU oracle and the GPU path take their inputs from here, so the two
sides see identical bytes.

Synthetic design (paper, Section VII "Definitions of Synthetic and Real
Datasets"): location (r, l) of an m x m grid is (r - 0.5 + X_rl, l - 0.5 + Y_rl)
with X, Y ~ U(-0.4, 0.4).  The paper prints a factor n^{1/2} in front, which
would put the points in [0, sqrt(n)]^2; the reading used here divides by m
instead, so the points lie in the unit square and no two are closer than 0.2/m.
"""
from .fields import (jittered_grid, jittered_subset, standard_normal,
                     batched_field_specs, FieldSpec)

__all__ = ["jittered_grid", "jittered_subset", "standard_normal",
           "batched_field_specs", "FieldSpec"]
