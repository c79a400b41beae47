"""Sample statistics of the salt mass fraction over parameter samples.

TEST INFRASTRUCTURE ONLY (oracle).  Section 3 of the paper:
  mean      c_bar(x) = sum_i w_i c(x, theta_i)                 (eq. pdestat)
  variance  Var(x)   = sum_i w_i (c_bar(x) - c(x, theta_i))^2  (eq. numer_var)
  exceedance P(c > c*) = #{i : c_i > c*} / N, strict '>'      (Section 3.2)
With quasi-Monte Carlo points every weight is 1/N.  The exceedance estimate is
written with the same weights, sum_i w_i [c_i > c*], which is the paper's count
divided by N when w_i = 1/N.
"""
from __future__ import annotations

import numpy as np


def moments(fields, weights=None, threshold=0.5):
    """fields: [S, ...] samples of c on a common vertex set.  Returns (mean, var, exceed)."""
    f = np.asarray(fields, dtype=float)
    S = f.shape[0]
    w = np.full(S, 1.0 / S) if weights is None else np.asarray(weights, dtype=float)
    mean = np.zeros(f.shape[1:])
    for i in range(S):
        mean += w[i] * f[i]
    var = np.zeros(f.shape[1:])
    for i in range(S):
        var += w[i] * (mean - f[i]) ** 2
    exceed = np.zeros(f.shape[1:])
    for i in range(S):
        exceed += w[i] * (f[i] > threshold)
    return mean, var, exceed


def inject(field, n_common):
    """Restrict a vertex field [nz, ny, nx] to the nested coarse vertex set with
    (nx_c, ny_c, nz_c) = n_common by picking every r-th vertex."""
    nz, ny, nx = field.shape
    ncx, ncy, ncz = n_common
    rx, ry, rz = (nx - 1) // (ncx - 1), (ny - 1) // (ncy - 1), (nz - 1) // (ncz - 1)
    assert (ncx - 1) * rx == nx - 1 and (ncy - 1) * ry == ny - 1 and (ncz - 1) * rz == nz - 1
    return field[::rz, ::ry, ::rx]
