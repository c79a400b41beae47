"""The discrete adjoint of the library against the oracle's tangent-linear gradient
and against finite differences of the library's own forward map.  GPU."""
import numpy as np
import pytest

import synth
from oracle import elder, gradient

pytestmark = pytest.mark.gpu

DT = synth.MONTH_S
BOX_UPPER = (200.0, 400.0, 200.0, 400.0, 0.0, 60.0)
TIGHT = dict(newton_rtol=1e-13, newton_atol=0.0, lin_rtol=1e-12, lin_max_it=800,
             newton_max_it=40, check_every=8)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _problem(phys, groups, **opts):
    from paper_1906_01632_amd import Problem
    o = dict(TIGHT)
    o.update(opts)
    return Problem(phys, groups, o)


@pytest.mark.parametrize("model,precision", [(2, 0), (3, 0), (2, 1), (2, 2)])
def test_adjoint_gradient_matches_oracle_tangent_linear(model, precision):
    nx, ny, nz = 17, 17, 5
    phys = synth.physics(model)
    xi = np.random.default_rng(21).uniform(-0.6, 0.6, (2, synth.N_XI[model]))
    pb = _problem(phys, [(nx, ny, nz, 3, 2)], precision=precision)
    pb.set_parameters(xi)
    J, g = pb.adjoint(BOX_UPPER, DT, 3)
    box = elder.Box(nx, ny, nz, phys)
    for s in range(2):
        Jr, gr, states = gradient.tangent_linear_gradient(
            box, xi[s], synth.initial_state(nx, ny, nz, phys), [DT] * 3, BOX_UPPER)
        print(f"sample {s}: J {J[s]:.9e} vs {Jr:.9e}; dJ {g[s]} vs {gr}", flush=True)
        assert abs(J[s] - Jr) <= 1e-9 * abs(Jr)
        assert np.abs(g[s] - gr).max() <= 1e-6 * np.abs(gr).max()
        # the problem is left at the final state
        assert np.abs(pb.get_state(s)[..., 1] - states[-1][..., 1]).max() < 1e-9
    pb.destroy()


def test_adjoint_gradient_matches_finite_differences_of_the_library():
    """Central differences (h = 1e-6) of the library's own forward map."""
    nx, ny, nz = 17, 17, 5
    phys = synth.physics(2)
    xi0 = np.array([0.2, -0.4, 0.5, 0.1])
    box = (200.0, 400.0, 200.0, 400.0, 0.0, 60.0)
    pb = _problem(phys, [(nx, ny, nz, 3, 1)])
    pb.set_parameters(xi0[None])
    J, g = pb.adjoint(box, DT, 2)
    pb.destroy()
    h = 1e-6
    pts = [xi0 + h * np.eye(4)[m] for m in range(4)] + [xi0 - h * np.eye(4)[m] for m in range(4)]
    fd_pb = _problem(phys, [(nx, ny, nz, 3, 8)])
    fd_pb.set_parameters(np.array(pts))
    fd_pb.solve(DT, 2)
    ph = phys
    ebox = elder.Box(nx, ny, nz, ph)
    vals = [gradient.qoi(ebox, elder.coefficients(ebox, pts[i]), fd_pb.get_state(i), box)
            for i in range(8)]
    fd = np.array([(vals[m] - vals[4 + m]) / (2 * h) for m in range(4)])
    print("adjoint", g[0], "fd", fd, flush=True)
    assert np.abs(g[0] - fd).max() <= 1e-5 * np.abs(fd).max()
    fd_pb.destroy()


def test_adjoint_through_split_steps():
    """A 4-month step that one sample has to take as sub-steps: the adjoint recomputes
    them from the checkpoint and still matches the oracle replaying the same steps."""
    nx, ny, nz = 17, 17, 5
    phys = synth.physics(2)
    xi = np.array([[0.0, 0.0, 0.0, 0.0], [0.9, 0.9, 0.9, 0.9]])
    pb = _problem(phys, [(nx, ny, nz, 3, 2)], dt_max_halvings=4)
    pb.set_parameters(xi)
    # first step alone to learn the sub-step counts the adjoint run will use
    probe = _problem(phys, [(nx, ny, nz, 3, 2)], dt_max_halvings=4)
    probe.set_parameters(xi)
    sub = [s["substeps"] for s in probe.step(4 * DT)]
    probe.destroy()
    assert sub[0] == 1 and sub[1] >= 2
    J, g = pb.adjoint(BOX_UPPER, 4 * DT, 1)
    box = elder.Box(nx, ny, nz, phys)
    for s in range(2):
        Jr, gr, _ = gradient.tangent_linear_gradient(
            box, xi[s], synth.initial_state(nx, ny, nz, phys), [4 * DT / sub[s]] * sub[s],
            BOX_UPPER)
        print(f"sample {s} substeps {sub[s]}: dJ {g[s]} vs {gr}", flush=True)
        assert abs(J[s] - Jr) <= 1e-9 * abs(Jr)
        assert np.abs(g[s] - gr).max() <= 1e-6 * np.abs(gr).max()
    pb.destroy()


def test_autograd_wrapper_gives_the_adjoint_gradient():
    """ElderQoI (torch.autograd): J and xi.grad equal the library's edf_adjoint output,
    the backward pass applies the incoming gradient per sample, and the problem's
    states are the starting states again after the call."""
    import torch
    from paper_1906_01632_amd import salt_mass
    nx, ny, nz = 17, 17, 5
    phys = synth.physics(2)
    xi0 = np.random.default_rng(4).uniform(-0.5, 0.5, (2, 4))
    pb = _problem(phys, [(nx, ny, nz, 3, 2)])
    pb.set_parameters(xi0)
    u0 = [pb.get_state(s) for s in range(2)]
    xi = torch.tensor(xi0, dtype=torch.float64, requires_grad=True)
    J = salt_mass(xi, pb, BOX_UPPER, DT, 2)
    w = torch.tensor([1.0, -2.5], dtype=torch.float64)
    (w * J).sum().backward()
    for s in range(2):
        assert np.array_equal(pb.get_state(s), u0[s])
    ref = _problem(phys, [(nx, ny, nz, 3, 2)])
    ref.set_parameters(xi0)
    Jr, gr = ref.adjoint(BOX_UPPER, DT, 2)
    ref.destroy()
    pb.destroy()
    np.testing.assert_array_equal(J.detach().numpy(), Jr)
    np.testing.assert_array_equal(xi.grad.numpy(), w.numpy()[:, None] * gr)


def test_adjoint_of_the_65_cubed_lattice_batch_converges():
    """64 lattice samples on 65x65x17 over 10 one-month steps with the solver options of
    the benchmark and the V-cycle bottom fused from the 9x9x3 level: the transposed
    systems' BiCGStab converges for every sample (with the residual of the zero-start
    sweep taken from the blocks towards the later colours on the transposed 17x17x5
    level, one sample's adjoint system had stalled) and the gradients are finite."""
    from paper_1906_01632_amd import PREC_F64, Problem
    wl = synth.workload("adjoint65")
    phys = synth.physics(wl.field_model)
    g = wl.groups[0]
    pb = Problem(phys, [(g.nx, g.ny, g.nz, g.levels, g.samples)],
                 dict(newton_rtol=wl.newton_rtol, lin_rtol=1e-6, lin_max_it=400,
                      newton_max_it=20, precision=PREC_F64, check_every=1, forcing=1))
    pb.set_parameters(wl.xi)
    pb.set_tuning(0, 3)
    J, dJ = pb.adjoint((200.0, 400.0, 200.0, 400.0, 100.0, 150.0), wl.dt, 10)
    print(f"J mean {np.mean(J):.6f}; dJ/dxi mean {np.mean(dJ, axis=0)}", flush=True)
    assert np.all(np.isfinite(J)) and np.all(np.isfinite(dJ))
    pb.destroy()
