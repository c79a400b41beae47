"""The seeded input generators: Halton points, tensor Gauss-Legendre nodes and the box
experiment's workloads, pinned by closed forms and the paper's counts.  CPU only."""
import json
import math
import os
from fractions import Fraction

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _radical_inverse_exact(i, b):
    x, f = Fraction(0), Fraction(1, b)
    while i:
        i, d = divmod(i, b)
        x += d * f
        f /= b
    return x


def test_radical_inverse_closed_forms():
    """Van der Corput values in bases 2, 3 and 5 written out by hand, and agreement with
    exact rational digit reversal for the first thousand indices."""
    assert [synth.radical_inverse(i, 2) for i in range(1, 9)] == \
        [0.5, 0.25, 0.75, 0.125, 0.625, 0.375, 0.875, 0.0625]
    want3 = [Fraction(1, 3), Fraction(2, 3), Fraction(1, 9), Fraction(4, 9), Fraction(7, 9),
             Fraction(2, 9), Fraction(5, 9), Fraction(8, 9), Fraction(1, 27)]
    assert np.allclose([synth.radical_inverse(i, 3) for i in range(1, 10)],
                       [float(x) for x in want3], rtol=0, atol=1e-15)
    assert abs(synth.radical_inverse(7, 5) - float(Fraction(2, 5) + Fraction(1, 25))) < 1e-15  # 7 = 12_5
    for b in (2, 3, 5):
        for i in range(1000):
            assert abs(synth.radical_inverse(i, b) - float(_radical_inverse_exact(i, b))) < 1e-15


def test_halton_stratification():
    """Indices 1 .. b^k - 1 of a base-b coordinate hit every cell j / b^k (j >= 1) once, so
    the first 2^k - 1 points are equidistributed in the base-2 coordinate and the first
    3^k - 1 in the base-3 one; the mapping to [-1, 1] is 2u - 1."""
    p = synth.halton_points(3 ** 5 - 1, 3)
    u3 = np.sort((p[:, 1] + 1) / 2)
    assert np.allclose(u3, np.arange(1, 3 ** 5) / 3 ** 5, atol=1e-14)
    p = synth.halton_points(2 ** 8 - 1, 3)
    u2 = np.sort((p[:, 0] + 1) / 2)
    assert np.allclose(u2, np.arange(1, 2 ** 8) / 2 ** 8, atol=1e-14)
    assert np.all(np.abs(p) < 1)
    # skip = 0 starts at the corner
    assert np.array_equal(synth.halton_points(1, 3, skip=0), [[-1.0, -1.0, -1.0]])


def test_tensor_gauss_legendre_exactness():
    """5^3 nodes integrate every monomial of degree <= 9 per variable exactly against the
    uniform probability measure on [-1, 1]^3: E[x^a y^b z^c] = prod 1/(k+1) for even k, 0
    for odd k."""
    nodes, w = synth.gauss_legendre_tensor(5, 3)
    assert nodes.shape == (125, 3) and abs(w.sum() - 1) < 1e-14 and np.all(w > 0)
    mom = lambda k: 0.0 if k % 2 else 1.0 / (k + 1)
    for a, b, c in [(0, 0, 0), (2, 0, 0), (8, 2, 0), (9, 4, 6), (4, 4, 4), (1, 2, 3), (6, 8, 2)]:
        got = np.sum(w * nodes[:, 0] ** a * nodes[:, 1] ** b * nodes[:, 2] ** c)
        assert abs(got - mom(a) * mom(b) * mom(c)) < 1e-14
    # the tenth power is not exact for a 5-point rule
    assert abs(np.sum(w * nodes[:, 0] ** 10) - 1 / 11) > 1e-4


def test_box_experiment_workloads_follow_the_paper():
    """Section 5, box with three random variables: 200 Halton qMC samples, 125 tensor
    Gauss-Legendre nodes (degree-4 surrogate), steps of 0.005 years, 1500 of them."""
    g = json.load(open(os.path.join(GOLDEN, "paper_counts.json")))
    for name in synth.E1_GRIDS:
        wl = synth.workload(name)
        q, n = wl.groups
        assert q.samples == g["box_qmc_samples"] and n.samples == g["box_gpc_nodes"]
        assert (q.nx, q.ny, q.nz) == (n.nx, n.ny, n.nz)
        assert wl.field_model == synth.FIELD_PAPER3
        assert wl.xi.shape == (g["box_qmc_samples"] + g["box_gpc_nodes"], g["box_random_variables"])
        assert math.isclose(wl.dt, g["box_dt_years"] * synth.YEAR_S)
        assert wl.steps == g["box_steps"]
        assert np.array_equal(wl.xi[:200], synth.halton_points(200, 3))
        nodes, w = synth.gauss_legendre_tensor(5, 3)
        assert np.array_equal(wl.xi[200:], nodes) and np.array_equal(wl.weights, w)
        assert round(len(nodes) ** (1 / 3)) == g["box_gpc_degree"] + 1
