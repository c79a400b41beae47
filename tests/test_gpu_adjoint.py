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


@pytest.mark.parametrize("model,precision,mf", [(2, 0, 0), (3, 0, 0), (2, 1, 0), (2, 2, 0),
                                               (1, 0, 1), (2, 1, 1)])
def test_adjoint_gradient_matches_oracle_tangent_linear(model, precision, mf):
    """Models 1-3, FP64/FP32/FP16-finest V-cycles, assembled or matrix-free forward
    products (the transposed products are always assembled)."""
    nx, ny, nz = 17, 17, 5
    phys = synth.physics(model)
    xi = np.random.default_rng(21).uniform(-0.6, 0.6, (2, synth.N_XI[model]))
    pb = _problem(phys, [(nx, ny, nz, 3, 2)], precision=precision, matrix_free=mf)
    pb.set_parameters(xi)
    J, g = pb.gradient(BOX_UPPER, DT, 3, checkpoint_every=2)
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
    J, g = pb.gradient(box, DT, 2)
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
    J, g = pb.gradient(BOX_UPPER, 4 * DT, 1)
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
    Jr, gr = ref.gradient(BOX_UPPER, DT, 2)
    ref.destroy()
    pb.destroy()
    np.testing.assert_array_equal(J.detach().numpy(), Jr)
    np.testing.assert_array_equal(xi.grad.numpy(), w.numpy()[:, None] * gr)


BOX_LOWER = (200.0, 400.0, 200.0, 400.0, 100.0, 150.0)  # the bottom 50 m under the centre


def _fd_gradient(phys, shape, levels, xi0, box, n_steps, h=1e-6):
    """Central differences of the library's own forward map, all 2 n_xi points in one
    batch with tight tolerances.  A component whose two runs took different sub-steps in
    some step (a different discrete trajectory, so J jumps) is returned as NaN: finite
    differences do not apply across that jump."""
    nx, ny, nz = shape
    m = xi0.size
    pts = [xi0 + h * np.eye(m)[q] for q in range(m)] + [xi0 - h * np.eye(m)[q] for q in range(m)]
    pb = _problem(phys, [(nx, ny, nz, levels, 2 * m)])
    pb.set_parameters(np.array(pts))
    subs = np.array([[t["substeps"] for t in pb.step(DT)] for _ in range(n_steps)])
    ebox = elder.Box(nx, ny, nz, phys)
    vals = [gradient.qoi(ebox, elder.coefficients(ebox, pts[i]), pb.get_state(i), box)
            for i in range(2 * m)]
    pb.destroy()
    fd = np.array([(vals[q] - vals[m + q]) / (2 * h) for q in range(m)])
    for q in range(m):
        if not np.array_equal(subs[:, q], subs[:, m + q]):
            print(f"FD component {q}: sub-steps {subs[:, q]} vs {subs[:, m + q]}, skipped",
                  flush=True)
            fd[q] = np.nan
    return fd


def test_checkpoint_spacing_does_not_change_the_gradient():
    """The trajectory recomputed segment by segment from checkpoints every 1, 2 or 5 steps
    (and every step kept) gives the same J and dJ/dxi bitwise: the forward kernels are
    deterministic and the recorded sub-step counts are replayed."""
    nx, ny, nz = 17, 17, 5
    phys = synth.physics(2)
    xi = np.random.default_rng(5).uniform(-0.8, 0.8, (3, 4))
    out = []
    for k in (1, 2, 5):
        pb = _problem(phys, [(nx, ny, nz, 3, 3)])
        pb.set_parameters(xi)
        out.append(pb.gradient(BOX_LOWER, DT, 5, checkpoint_every=k))
        pb.destroy()
    for J, g in out[1:]:
        np.testing.assert_array_equal(J, out[0][0])
        np.testing.assert_array_equal(g, out[0][1])


def test_adjoint_needs_a_recorded_trajectory():
    from paper_1906_01632_amd import EDFError
    nx, ny, nz = 17, 17, 5
    pb = _problem(synth.physics(2), [(nx, ny, nz, 3, 1)])
    pb.set_parameters(np.zeros((1, 4)))
    with pytest.raises(EDFError, match="EDF_ERR_STATE"):
        pb.adjoint(BOX_LOWER)
    pb.solve(DT, 2, checkpoint_every=1, stats=False)
    pb.adjoint(BOX_LOWER)
    pb.step(DT)  # a step after the recorded trajectory drops it
    with pytest.raises(EDFError, match="EDF_ERR_STATE"):
        pb.adjoint(BOX_LOWER)
    pb.destroy()


def test_adjoint_lower_box_33_matches_oracle_tangent_linear():
    """The lower-central box of the gradient workload on 33x33x9, two samples, 4 steps:
    J and dJ/dxi against the oracle's tangent-linear gradient (a different mode from the
    library's adjoint)."""
    nx, ny, nz = 33, 33, 9
    phys = synth.physics(2)
    xi = synth.lattice_points(512, 4, seed=0)[[0, 8]]
    pb = _problem(phys, [(nx, ny, nz, 4, 2)])
    pb.set_parameters(xi)
    J, g = pb.gradient(BOX_LOWER, DT, 4, checkpoint_every=3)
    box = elder.Box(nx, ny, nz, phys)
    for s in range(2):
        Jr, gr, _ = gradient.tangent_linear_gradient(
            box, xi[s], synth.initial_state(nx, ny, nz, phys), [DT] * 4, BOX_LOWER)
        print(f"sample {s}: J {J[s]:.9e} vs {Jr:.9e}; dJ {g[s]} vs {gr}", flush=True)
        assert abs(J[s] - Jr) <= 1e-9 * abs(Jr)
        assert np.abs(g[s] - gr).max() <= 1e-6 * np.abs(gr).max()
    pb.destroy()


def test_adjoint_of_the_65_cubed_lattice_batch_matches_finite_differences():
    """The gradient workload's shape: 64 lattice samples on 65x65x17, 10 one-month steps
    with a checkpoint every 10, the salt mass in the lower-central box, the benchmark's
    solver options and the V-cycle bottom fused from the 9x9x3 level.  Every transposed
    system converges (one sample's, 57, had stalled when the zero-start residual was used
    on the transposed 17x17x5 level), the gradients are finite, and for samples 0 and 57
    they agree with a tightly converged adjoint of the same two samples, which in turn
    agrees with central differences (h = 1e-6) of the library's forward map to 1e-5 (a
    component whose +h and -h runs took different sub-steps is reported and skipped)."""
    from paper_1906_01632_amd import PREC_F64, Problem
    wl = synth.workload("adjoint65")
    phys = synth.physics(wl.field_model)
    g = wl.groups[0]
    pb = Problem(phys, [(g.nx, g.ny, g.nz, g.levels, g.samples)],
                 dict(newton_rtol=wl.newton_rtol, lin_rtol=1e-6, lin_max_it=400,
                      newton_max_it=20, precision=PREC_F64, check_every=1, forcing=1))
    pb.set_parameters(wl.xi)
    pb.set_tuning(0, 3)
    st = pb.solve(wl.dt, 10, checkpoint_every=10)
    J, dJ = pb.adjoint(BOX_LOWER)
    print(f"J mean {np.mean(J):.6f}; dJ/dxi mean {np.mean(dJ, axis=0)}", flush=True)
    assert np.all(np.isfinite(J)) and np.all(np.isfinite(dJ))
    pb.destroy()
    pick = [0, 57]
    tight = _problem(phys, [(g.nx, g.ny, g.nz, g.levels, 2)])
    tight.set_parameters(wl.xi[pick])
    st2 = tight.solve(wl.dt, 10, checkpoint_every=10)
    Jt, gt = tight.adjoint(BOX_LOWER)
    tight.destroy()
    checked = 0
    for q, s in enumerate(pick):
        fd = _fd_gradient(phys, (g.nx, g.ny, g.nz), g.levels, wl.xi[s], BOX_LOWER, 10)
        print(f"sample {s}: batch {dJ[s]} tight {gt[q]} fd {fd}", flush=True)
        ok = np.isfinite(fd)
        checked += int(ok.sum())
        assert np.abs(gt[q] - fd)[ok].max() <= 1e-5 * np.abs(gt[q]).max()
        if st[s]["substeps_total"] == st2[q]["substeps_total"]:  # same sub-steps taken
            assert abs(J[s] - Jt[q]) <= 1e-8 * abs(Jt[q])
            assert np.abs(dJ[s] - gt[q]).max() <= 1e-4 * np.abs(gt[q]).max()
    assert checked >= 6  # of the 8 components of the two samples


def test_merged_groups_give_the_serial_gradient():
    """With merged V-cycles (concurrent_groups = 2) the forward steps of two nested groups
    share launches and the adjoint's transposed solves run group by group: J and dJ/dxi
    are bitwise those of the serial mode."""
    phys = synth.physics(2)
    groups = [(9, 9, 3, 2, 2), (17, 17, 5, 3, 2)]
    xi = np.random.default_rng(7).uniform(-0.6, 0.6, (4, 4))
    out = {}
    for conc in (0, 2):
        pb = _problem(phys, groups, concurrent_groups=conc, check_every=1)
        pb.set_parameters(xi)
        out[conc] = pb.gradient(BOX_UPPER, DT, 3, checkpoint_every=2)
        pb.destroy()
    assert np.array_equal(out[2][0], out[0][0])
    assert np.array_equal(out[2][1], out[0][1])
