"""Host logic of the multilevel estimator weights (paper_1906_01632_amd.uq); CPU only.
The oracle's weighted moments serve as the reference arithmetic."""
import numpy as np
import pytest

from oracle import stats
from paper_1906_01632_amd.uq import mlmc_weights


def _layout(levels, rng, shape=(3, 4)):
    """Fields in the multilevel layout: per level the level's samples, then the coarse
    partners of the next level's samples."""
    fine = [rng.random((n,) + shape) for n in levels]
    coarse = [rng.random((n,) + shape) for n in levels]  # coarse[l]: level l-1 partners of level l
    out = []
    for l, n in enumerate(levels):
        out.append(fine[l])
        if l + 1 < len(levels):
            out.append(coarse[l + 1])
    return np.concatenate(out), fine, coarse


@pytest.mark.parametrize("levels", [(7,), (8, 3), (256, 64, 16), (5, 4, 3, 2)])
def test_weights_sum_to_one_and_follow_the_layout(levels):
    w = mlmc_weights(levels)
    assert w.size == sum(levels) + sum(levels[1:])
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.all(w[:levels[0]] == 1.0 / levels[0])


@pytest.mark.parametrize("levels", [(6, 3), (10, 5, 2)])
def test_multilevel_mean_and_variance_written_out(levels):
    """The weighted mean equals mean(level 0) + sum_l mean(c_l - c_{l-1}) over the pairs,
    the weighted spread equals the same telescoping sum for c^2 minus the mean squared,
    and a single level is the plain sample mean and variance."""
    rng = np.random.default_rng(4)
    f, fine, coarse = _layout(levels, rng)
    m, v, e = stats.moments(f, mlmc_weights(levels), threshold=0.5)
    m1 = fine[0].mean(axis=0) + sum((fine[l] - coarse[l]).mean(axis=0) for l in range(1, len(levels)))
    m2 = (fine[0] ** 2).mean(axis=0) + sum((fine[l] ** 2 - coarse[l] ** 2).mean(axis=0)
                                             for l in range(1, len(levels)))
    ex = (fine[0] > 0.5).mean(axis=0) + sum(((fine[l] > 0.5).astype(float) - (coarse[l] > 0.5)).mean(axis=0)
                                            for l in range(1, len(levels)))
    assert np.abs(m - m1).max() < 1e-14
    assert np.abs(v - (m2 - m1 ** 2)).max() < 1e-14
    assert np.abs(e - ex).max() < 1e-14
    one = fine[0]
    m0, v0, _ = stats.moments(one, mlmc_weights((len(one),)))
    assert np.abs(m0 - one.mean(axis=0)).max() < 1e-15 and np.abs(v0 - one.var(axis=0)).max() < 1e-15


def test_identical_pairs_telescope_to_the_coarsest_level():
    """If every sample equals its coarse partner the corrections vanish; if level l is the
    constant l, the estimate is the finest level's value."""
    levels = (9, 4, 2)
    rng = np.random.default_rng(1)
    f, fine, coarse = _layout(levels, rng)
    # copy the partners into the fine samples: corrections vanish
    start = [0]
    for l, n in enumerate(levels):
        start.append(start[-1] + n + (levels[l + 1] if l + 1 < len(levels) else 0))
    g = f.copy()
    for l in range(1, len(levels)):
        partners = g[start[l - 1] + levels[l - 1]: start[l - 1] + levels[l - 1] + levels[l]]
        g[start[l]: start[l] + levels[l]] = partners
    m, _, _ = stats.moments(g, mlmc_weights(levels))
    assert np.abs(m - g[:levels[0]].mean(axis=0)).max() < 1e-14
    h = np.zeros_like(f)
    for l, n in enumerate(levels):
        h[start[l]: start[l] + n] = l
        if l + 1 < len(levels):
            h[start[l] + n: start[l + 1]] = l
    m, v, _ = stats.moments(h, mlmc_weights(levels))
    assert np.abs(m - (len(levels) - 1)).max() < 1e-14
