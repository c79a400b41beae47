"""Quasi-Monte Carlo against polynomial chaos statistics of one problem, and multilevel
Monte Carlo statistics on nested grids.

The box experiment with three random variables (Section 5, eq. poro-paral3RVS) runs
the same porosity model twice: as 200 Halton qMC samples, whose mean, variance and
exceedance probability are the equally weighted sample statistics (Section 3), and at
the 125 tensor Gauss-Legendre nodes of a degree-4 Legendre surrogate, whose mean and
variance follow from its coefficients and whose exceedance probability from sampling
the surrogate (Section 3.1).  The paper compares the two through the isosurfaces
mean = 0.5 and variance = 0.05 after 1500 steps; this module puts numbers on that
comparison: field differences and the share of vertices on which the two methods put
a vertex on different sides of those levels.

Every statistic here is computed by the library (edf_moments, edf_gpc_project,
edf_gpc_exceed); this module only chooses the weights and compares the results.
"""
from __future__ import annotations

import numpy as np


def _rel_l2(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / nb if nb > 0 else float(np.linalg.norm(a - b))


def qmc_vs_gpc(pb, qmc_group: int, gpc_group: int, gl_weights, common, degree: int = 4,
               truncation: int = 0, threshold: float = 0.5, var_level: float = 0.05,
               n_points: int = 100_000, seed: int = 0) -> dict:
    """Statistics of `qmc_group` (equally weighted samples) and of the surrogate projected
    from `gpc_group` (its samples are the quadrature nodes with weights `gl_weights`),
    both on the nested common grid `common` = (cx, cy, cz).

    Returns the fields (qmc_mean, qmc_var, qmc_exceed, gpc_mean, gpc_var, gpc_exceed,
    each [cz, cy, cx]) and a `compare` dict: relative L2 and largest differences of the
    means, variances and exceedance probabilities, and the fraction of vertices whose
    side of mean = threshold and of variance = var_level differs between the methods."""
    first, n_q = int(pb.offsets[qmc_group]), pb.groups[qmc_group][4]
    w = np.zeros(pb.S)
    w[first:first + n_q] = 1.0 / n_q
    qm, qv, qe = pb.moments(common, threshold=threshold, weights=w)
    g = pb.gpc_project(gpc_group, common, degree, gl_weights, truncation=truncation,
                       coefficients=False)
    pts = np.random.default_rng(seed).uniform(-1.0, 1.0, (n_points, pb.n_xi))
    ge, _ = pb.gpc_exceed(pts, threshold, common)
    gm, gv = g["mean"], g["var"]
    cmp = {
        "mean_rel_l2": _rel_l2(qm, gm), "mean_max_abs": float(np.abs(qm - gm).max()),
        "var_rel_l2": _rel_l2(qv, gv), "var_max_abs": float(np.abs(qv - gv).max()),
        "exceed_max_abs": float(np.abs(qe - ge).max()),
        "exceed_mean_abs": float(np.abs(qe - ge).mean()),
        "mean_level_side_differs": float(np.mean((qm > threshold) != (gm > threshold))),
        "var_level_side_differs": float(np.mean((qv > var_level) != (gv > var_level))),
        "mean_level_vertices": [int(np.sum(qm > threshold)), int(np.sum(gm > threshold))],
        "var_level_vertices": [int(np.sum(qv > var_level)), int(np.sum(gv > var_level))],
        "max_var": [float(qv.max()), float(gv.max())],
        "n_coef": g["n_coef"], "surrogate_points": n_points,
    }
    return {"qmc_mean": qm, "qmc_var": qv, "qmc_exceed": qe, "gpc_mean": gm, "gpc_var": gv,
            "gpc_exceed": ge, "compare": cmp}


def mlmc_weights(n_per_level) -> np.ndarray:
    """Sample weights of the multilevel estimator on nested grids (level 0 coarsest).

    Layout of the problem: group l holds the n_l samples of level l followed by the
    coarse partners (the same parameters) of the n_{l+1} samples of level l + 1.  The
    estimator E[c_L] = E[c_0] + sum_l E[c_l - c_{l-1}] with sample means per level gives
    weight +1/n_l to the level-l samples and -1/n_{l+1} to the partners; the weights sum
    to 1.  Applied to c and c^2 alike, the weighted mean and the weighted spread
    sum w (c - mean)^2 = sum w c^2 - mean^2 are the multilevel estimates of the mean and
    the variance (the latter may come out slightly negative where the variance is small);
    the weighted indicator sum is the multilevel estimate of the exceedance probability."""
    n = [int(k) for k in n_per_level]
    w = []
    for l, k in enumerate(n):
        w += [1.0 / k] * k
        if l + 1 < len(n):
            w += [-1.0 / n[l + 1]] * n[l + 1]
    return np.array(w)


def mlmc_moments(pb, n_per_level, common, threshold: float = 0.5):
    """Multilevel mean, variance and exceedance probability [cz, cy, cx] on the common
    grid (edf_moments with the weights of mlmc_weights).  Every sample must have taken its
    last step: a failed one would break its level pair."""
    w = mlmc_weights(n_per_level)
    if w.size != pb.S:
        raise ValueError(f"{w.size} weights for {pb.S} samples")
    return pb.moments(common, threshold=threshold, weights=w)
