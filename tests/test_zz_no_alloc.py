"""edf_moments_noalloc (no device allocation, a fixed scratch array per GPU) against
edf_moments through the C-ABI: bitwise the same statistics, on two calls in a row, the
second with a smaller common grid; samples taken in several chunks; a failed sample
left out by both; a grid beyond the scratch rejected.  GPU."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

DT = synth.MONTH_S


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _problem(phys, groups, **opts):
    from paper_1906_01632_amd import Problem
    o = dict(newton_rtol=1e-10, lin_rtol=1e-8, lin_max_it=400, newton_max_it=30, check_every=4)
    o.update(opts)
    return Problem(phys, groups, o)


def _same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_noalloc_moments_equal_moments_two_calls_smaller_second():
    phys = synth.physics(2)
    xi = np.random.default_rng(2).uniform(-0.8, 0.8, (5, 4))
    xi[1] = 0.9  # fails a 4-month step without halving: left out of both
    pb = _problem(phys, [(17, 17, 5, 3, 3), (33, 33, 9, 4, 2)], dt_max_halvings=0)
    pb.set_parameters(xi)
    st = pb.step(4 * DT)
    failed = [s for s in range(5) if st[s]["status"] != 0]
    assert 1 in failed and len(failed) < 5, failed
    w = np.random.default_rng(3).uniform(0.5, 1.5, 5)
    for common, weights in (((9, 9, 3), w), ((5, 5, 2), None)):
        ref = pb.moments(common, threshold=0.3, weights=weights)
        got = pb.moments(common, threshold=0.3, weights=weights, noalloc=True)
        _same(got, ref)
        assert np.abs(ref[0]).max() > 0
    pb.destroy()


def test_noalloc_moments_in_chunks():
    """256 samples on 33x33x9 with the full grid as the common grid: the scratch holds
    about 200 sample fields, so the sums run over two chunks; then a smaller grid."""
    phys = synth.physics(2)
    pb = _problem(phys, [(33, 33, 9, 4, 256)], newton_rtol=1e-8, lin_rtol=1e-6, forcing=1)
    pb.set_parameters(synth.lattice_points(256, 4, seed=1))
    pb.step(DT)
    for common in ((33, 33, 9), (17, 17, 5)):
        _same(pb.moments(common, noalloc=True), pb.moments(common))
    pb.destroy()


def test_noalloc_moments_reject_a_grid_beyond_the_scratch():
    from paper_1906_01632_amd import EDFError
    phys = synth.physics(0)
    pb = _problem(phys, [(129, 129, 33, 6, 1)])
    pb.set_parameters(np.zeros((1, 0)))
    with pytest.raises(EDFError, match="EDF_ERR_ARG"):
        pb.moments((129, 129, 33), noalloc=True)
    m, v, e = pb.moments((65, 65, 17), noalloc=True)  # 4 x 71,825 doubles fit
    _same((m, v, e), pb.moments((65, 65, 17)))
    pb.destroy()
