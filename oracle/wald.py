"""CPU FP64 oracle of the Wald test of the SNP effect (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module.  The problem statement (supplementary notes, section 1) asks for
the estimates together with their p-values; for the SNP effect b with
standard error SE the statistic is z = b / SE, and its two-sided p-value
under the null b = 0 is the probability that a standard normal exceeds |z| in
absolute value, P(|N(0,1)| >= |z|) = erfc(|z| / sqrt 2), which is also the
upper tail of a chi-square with one degree of freedom at z^2.
Parity status: pinned by tests/test_oracle_wald.py (textbook quantiles of the
normal distribution, the normal and chi-square tails of scipy, numerical
integration of the normal density, the asymptotic tail series)."""
from __future__ import annotations

import math

import numpy as np

_erfc = np.vectorize(math.erfc, otypes=[np.float64])


def wald(b, se):
    """(z, p): the Wald statistic and its two-sided p-value, elementwise; NaN where b or SE is NaN."""
    b = np.asarray(b, dtype=np.float64)
    se = np.asarray(se, dtype=np.float64)
    z = b / se
    p = np.where(np.isnan(z), np.nan, _erfc(np.where(np.isnan(z), 0.0, np.abs(z)) / math.sqrt(2.0)))
    return z, p
