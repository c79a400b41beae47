"""Parity of the HIP path (through the C-ABI) with the oracle, element by element.

All tests here need an MI355X and the built libedf.so.  Inputs are seeded and
synthetic; the oracle runs on the host CPU.  Tolerances: FP64 results within
1e-10 relative L2 per field (the bar for the FP64 path), residual and Jacobian
entries within 1e-11 of the largest entry of their row (rounding of ~30 terms).
"""
import numpy as np
import pytest

import synth
from oracle import elder, newton, stats

pytestmark = pytest.mark.gpu

DT = synth.MONTH_S
TIGHT = dict(newton_rtol=1e-13, newton_atol=0.0, lin_rtol=1e-12, lin_max_it=600,
             newton_max_it=40, check_every=8)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_01632_amd import load_library
    load_library()


def _problem(phys, groups, **opts):
    from paper_1906_01632_amd import Problem
    o = dict(TIGHT)
    o.update(opts)
    return Problem(phys, groups, o)


def _xi(model, S, seed=3):
    n = synth.N_XI[model]
    return np.random.default_rng(seed).uniform(-1, 1, (S, n))


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


SHAPES = [((9, 9, 3), 2), ((17, 13, 5), 3), ((33, 33, 9), 4), ((41, 25, 9), 3)]


@pytest.mark.parametrize("shape,levels", SHAPES)
@pytest.mark.parametrize("model", [0, 1, 2, 3])
def test_defect_matches_oracle(shape, levels, model):
    nx, ny, nz = shape
    phys = synth.physics(model)
    xi = _xi(model, 2)
    pb = _problem(phys, [(nx, ny, nz, levels, 2)])
    pb.set_parameters(xi)
    box = elder.Box(nx, ny, nz, phys)
    for s in range(2):
        u = synth.random_state(nx, ny, nz, phys, seed=10 + s)
        uo = synth.random_state(nx, ny, nz, phys, seed=20 + s)
        got = pb.residual(s, u, uo, DT)
        coef = elder.coefficients(box, xi[s])
        ref = elder.residual(box, coef, u, uo, DT) * elder.row_scale(box, DT)
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-11 * scale, (s, np.abs(got - ref).max(), scale)
    pb.destroy()


@pytest.mark.parametrize("model", [0, 2, 3])
def test_stratified_hydrostatic_defect(model):
    """A non-uniform stratification c(z) with its discrete hydrostatic pressure (trapezoid
    rule down each column): the library's liquid rows vanish (no Darcy flux through any
    face, whatever K), and its whole defect equals the oracle's."""
    nx, ny, nz = 17, 13, 5
    phys = synth.physics(model)
    xi = _xi(model, 1)
    pb = _problem(phys, [(nx, ny, nz, 3, 1)])
    pb.set_parameters(xi)
    box = elder.Box(nx, ny, nz, phys)
    cz = np.array([0.0, 0.45, 0.2, 0.8, 0.6])
    rho = phys["rho0"] + (phys["rho1"] - phys["rho0"]) * cz
    p = np.concatenate([[0.0], np.cumsum(phys["g"] * box.h[2] * 0.5 * (rho[1:] + rho[:-1]))])
    u = np.zeros((nz, ny, nx, 2))
    u[..., 0] = p[:, None, None]
    u[..., 1] = cz[:, None, None]
    got = pb.residual(0, u, u, DT)
    ref = elder.residual(box, elder.coefficients(box, xi[0]), u, u, DT) * elder.row_scale(box, DT)
    assert np.abs(got[..., 0]).max() < 1e-12
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
    pb.destroy()


def _oracle_stencil(box, coef, u):
    """Oracle Jacobian scaled like the library's, as [27][2][2][nz][ny][nx]."""
    J = elder.jacobian(box, coef, u, DT)
    rs = elder.row_scale(box, DT).reshape(-1)
    cs = np.tile(elder.col_scale(box), box.N)
    Js = (J.multiply(rs[:, None]).multiply(cs[None, :])).tocoo()
    out = np.zeros((27, 2, 2, box.nz, box.ny, box.nx))
    v, w = Js.row // 2, Js.col // 2
    eq, var = Js.row % 2, Js.col % 2
    nx, ny = box.nx, box.ny
    iv, jv, kv = v % nx, (v // nx) % ny, v // (nx * ny)
    iw, jw, kw = w % nx, (w // nx) % ny, w // (nx * ny)
    o = (iw - iv + 1) + 3 * (jw - jv + 1) + 9 * (kw - kv + 1)
    np.add.at(out, (o, eq, var, kv, jv, iv), Js.data)
    return out


@pytest.mark.parametrize("shape,levels", SHAPES[:3])
@pytest.mark.parametrize("model", [0, 1, 2])
def test_jacobian_matches_oracle_on_every_level(shape, levels, model):
    nx, ny, nz = shape
    phys = synth.physics(model)
    xi = _xi(model, 1)
    pb = _problem(phys, [(nx, ny, nz, levels, 1)])
    pb.set_parameters(xi)
    u = synth.random_state(nx, ny, nz, phys, seed=5)
    for level in range(levels):
        got = pb.get_jacobian(0, u, DT, level)
        r = 2 ** level
        box = elder.Box((nx - 1) // r + 1, (ny - 1) // r + 1, (nz - 1) // r + 1, phys)
        ul = u[::r, ::r, ::r]
        ref = _oracle_stencil(box, elder.coefficients(box, xi[0]), ul)
        rowmax = np.abs(ref).max(axis=(0, 2), keepdims=True)
        err = np.abs(got - ref) / np.maximum(rowmax, 1e-300)
        assert err.max() < 1e-11, (level, err.max())
    pb.destroy()


@pytest.mark.parametrize("shape,levels,model", [((9, 9, 3), 2, 0), ((17, 17, 5), 3, 2),
                                                ((33, 33, 9), 4, 0), ((41, 25, 9), 3, 3),
                                                ((33, 33, 9), 4, 1), ((17, 17, 5), 3, 1)])
def test_one_step_from_initial_state(shape, levels, model):
    nx, ny, nz = shape
    phys = synth.physics(model)
    xi = _xi(model, 1, seed=9)
    pb = _problem(phys, [(nx, ny, nz, levels, 1)])
    pb.set_parameters(xi)
    st = pb.step(DT)
    assert st[0]["status"] == 0, st
    box = elder.Box(nx, ny, nz, phys)
    ref = newton.newton_solve(box, elder.coefficients(box, xi[0]),
                              synth.initial_state(nx, ny, nz, phys), DT)
    got = pb.get_state(0)
    for f in range(2):
        assert _rel(got[..., f], ref[..., f]) < 1e-10, (f, _rel(got[..., f], ref[..., f]))
    pb.destroy()


def test_step_from_shared_later_state():
    """Per-step parity from a developed state (after 3 oracle steps)."""
    nx, ny, nz = 17, 17, 5
    phys = synth.physics(2)
    xi = _xi(2, 1, seed=4)
    box = elder.Box(nx, ny, nz, phys)
    coef = elder.coefficients(box, xi[0])
    u = synth.initial_state(nx, ny, nz, phys)
    for _ in range(3):
        u = newton.newton_solve(box, coef, u, DT)
    ref = newton.newton_solve(box, coef, u, DT)
    pb = _problem(phys, [(nx, ny, nz, 3, 1)])
    pb.set_parameters(xi)
    pb.set_state(0, u)
    pb.step(DT)
    got = pb.get_state(0)
    for f in range(2):
        assert _rel(got[..., f], ref[..., f]) < 1e-10
    # the increment itself agrees, not only the state
    dc_ref, dc_got = ref[..., 1] - u[..., 1], got[..., 1] - u[..., 1]
    assert _rel(dc_got, dc_ref) < 1e-8
    pb.destroy()


def test_trajectory_33_twenty_steps():
    """The plain-method workload in full: 20 one-month steps of the 33x33x9 deterministic
    box, the oracle stepping beside it; every step's state within 1e-10 relative L2 per
    field (the error of each step is printed)."""
    nx, ny, nz = 33, 33, 9
    phys = synth.physics(0)
    pb = _problem(phys, [(nx, ny, nz, 4, 1)])
    pb.set_parameters(np.zeros((1, 0)))
    box = elder.Box(nx, ny, nz, phys)
    coef = elder.coefficients(box, [])
    u = synth.initial_state(nx, ny, nz, phys)
    for n in range(20):
        u = newton.newton_solve(box, coef, u, DT)
        pb.step(DT)
        got = pb.get_state(0)
        errs = [_rel(got[..., f], u[..., f]) for f in range(2)]
        print(f"step {n + 1}: rel L2 p {errs[0]:.2e} c {errs[1]:.2e}", flush=True)
        assert max(errs) < 1e-10
    pb.destroy()


def test_batched_sample_equals_single_sample():
    """A sample advanced inside a batch is bitwise the sample advanced alone."""
    nx, ny, nz = 17, 17, 5
    phys = synth.physics(2)
    xi = _xi(2, 3, seed=8)
    opts = dict(newton_rtol=1e-10, lin_rtol=1e-8)
    pb = _problem(phys, [(nx, ny, nz, 3, 3)], **opts)
    pb.set_parameters(xi)
    pb.step(DT)
    pb.step(DT)
    batch = [pb.get_state(s) for s in range(3)]
    pb.destroy()
    for s in range(3):
        one = _problem(phys, [(nx, ny, nz, 3, 1)], **opts)
        one.set_parameters(xi[s:s + 1])
        one.step(DT)
        one.step(DT)
        np.testing.assert_array_equal(one.get_state(0), batch[s])
        one.destroy()


def test_runs_are_deterministic():
    nx, ny, nz = 33, 17, 9
    phys = synth.physics(2)
    xi = _xi(2, 2, seed=1)
    out = []
    for _ in range(2):
        pb = _problem(phys, [(nx, ny, nz, 3, 2)], newton_rtol=1e-10, lin_rtol=1e-8)
        pb.set_parameters(xi)
        pb.solve(DT, 2)
        out.append([pb.get_state(s) for s in range(2)])
        pb.destroy()
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)


def test_mixed_resolution_groups_and_moments():
    """Two resolution groups in one problem; pooled moments on the common grid equal
    the oracle's statistics of the same injected fields, and each group's own moments at
    its own resolution those of its fields."""
    phys = synth.physics(2)
    xi = synth.lattice_points(16, 4, seed=2)[:6]
    pb = _problem(phys, [(9, 9, 3, 2, 4), (17, 17, 5, 3, 2)], newton_rtol=1e-10, lin_rtol=1e-8)
    pb.set_parameters(xi)
    st = pb.solve(DT, 2)
    assert all(s["status"] == 0 for s in st)
    mean, var, exc = pb.moments((9, 9, 3), threshold=0.5)
    fields = [pb.get_state(s)[..., 1] for s in range(4)]
    fields += [stats.inject(pb.get_state(s)[..., 1], (9, 9, 3)) for s in range(4, 6)]
    m, v, e = stats.moments(np.array(fields), threshold=0.5)
    assert np.abs(mean - m).max() < 1e-14
    assert np.abs(var - v).max() < 1e-14
    assert np.abs(exc - e).max() < 1e-14
    w = np.arange(1, 7, dtype=float)
    mean_w, var_w, _ = pb.moments((9, 9, 3), weights=w)
    m, v, _ = stats.moments(np.array(fields), weights=w / w.sum())
    assert np.abs(mean_w - m).max() < 1e-14 and np.abs(var_w - v).max() < 1e-14
    # each group's statistics at its own resolution (edf_group_moments)
    for gi, members, shape in ((0, range(4), (9, 9, 3)), (1, range(4, 6), (17, 17, 5))):
        own = np.array([pb.get_state(s)[..., 1] for s in members])
        for wg in (None, np.arange(1, len(own) + 1, dtype=float)):
            mean_g, var_g, exc_g = pb.group_moments(gi, threshold=0.5, weights=wg)
            assert mean_g.shape == shape[::-1]
            m, v, e = stats.moments(own, weights=None if wg is None else wg / wg.sum(),
                                    threshold=0.5)
            assert np.abs(mean_g - m).max() < 1e-14
            assert np.abs(var_g - v).max() < 1e-14
            assert np.abs(exc_g - e).max() < 1e-14
    # each group stepped exactly like the oracle
    for s, (nx, ny, nz) in [(0, (9, 9, 3)), (5, (17, 17, 5))]:
        box = elder.Box(nx, ny, nz, phys)
        coef = elder.coefficients(box, xi[s])
        u = synth.initial_state(nx, ny, nz, phys)
        for _ in range(2):
            u = newton.newton_solve(box, coef, u, DT)
        got = pb.get_state(s)
        assert _rel(got[..., 1], u[..., 1]) < 1e-8
    pb.destroy()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_vcycle_is_a_contraction(precision):
    """One V-cycle reduces the residual of the Newton matrix by a solid factor."""
    nx, ny, nz = 33, 33, 9
    phys = synth.physics(2)
    pb = _problem(phys, [(nx, ny, nz, 4, 2)], precision=precision)
    pb.set_parameters(_xi(2, 2))
    b = np.random.default_rng(0).standard_normal((2, nz, ny, nx, 2))
    b[..., 1][:, -1] = 0.0
    y = pb.apply_vcycle(0, DT, b)
    Ay = pb.apply_jacobian(0, y)
    for s in range(2):
        red = np.linalg.norm(b[s] - Ay[s]) / np.linalg.norm(b[s])
        print(f"sample {s} precision {precision}: |b - A M^-1 b|/|b| = {red:.3f}", flush=True)
        assert red < 0.5
    pb.destroy()


@pytest.mark.parametrize("precision,smoother", [(0, 0), (1, 0), (2, 0), (0, 1), (1, 1), (2, 1)])
def test_vcycle_same_for_every_fused_bottom(precision, smoother):
    """The V-cycle gives the same result whichever levels run in the fused bottom launch,
    and set_tuning rejects levels that do not fit the fused launch.  Levels swept by
    separate launches take the zero-start forms (first sweep from x = 0 reading only the
    colours already swept, residual from the blocks towards the later colours); the fused
    bottom takes the general forms (full stencil, r = b - A x): the two agree to rounding.
    The fused bottom sweeps its levels with the same smoother, points (0) or vertical
    lines (1), as the levels swept by their own launches."""
    nx, ny, nz = 33, 33, 9
    phys = synth.physics(2)
    # the same smoother on every level, so that moving a level into the fused bottom changes
    # only the forms of its sweeps, not the smoother
    pb = _problem(phys, [(nx, ny, nz, 4, 3)], precision=precision, smoother=smoother)
    pb.set_parameters(_xi(2, 3, seed=11))
    b = np.random.default_rng(5).standard_normal((3, nz, ny, nx, 2))
    b[..., 1][:, -1] = 0.0
    ys = {}
    for l0 in (1, 2, 3):  # 17x17x5, 9x9x3 and the 5x5x2 coarse solve alone
        pb.set_tuning(0, l0)
        assert pb.tuning(0)[0] == l0
        ys[l0] = pb.apply_vcycle(0, DT, b)
    tol = 1e-13 if precision == 0 else 1e-6
    for l0 in (2, 3):
        assert _rel(ys[l0], ys[1]) < tol, (l0, _rel(ys[l0], ys[1]))
    for bad in (0, 4, -1):  # 33x33x9 exceeds the fused launch; 4 is no level
        with pytest.raises(RuntimeError):
            pb.set_tuning(0, bad)
    pb.destroy()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_line_smoothed_vcycle_is_a_contraction(precision):
    """The vertical-line smoother (columns solved exactly, 4 column colours) on the levels
    swept by their own launches: one V-cycle reduces the residual at least as well as
    the point smoother's, and it stays a contraction whichever levels are fused."""
    nx, ny, nz = 33, 33, 9
    phys = synth.physics(2)
    b = np.random.default_rng(0).standard_normal((2, nz, ny, nx, 2))
    b[..., 1][:, -1] = 0.0
    red = {}
    for smoother in (0, 1):
        pb = _problem(phys, [(nx, ny, nz, 4, 2)], precision=precision, smoother=smoother)
        pb.set_parameters(_xi(2, 2))
        for l0 in (2, 3):
            pb.set_tuning(0, l0)
            y = pb.apply_vcycle(0, DT, b)
            Ay = pb.apply_jacobian(0, y)
            red[(smoother, l0)] = [np.linalg.norm(b[s] - Ay[s]) / np.linalg.norm(b[s])
                                   for s in range(2)]
        pb.destroy()
    print(f"precision {precision}: |b - A M^-1 b|/|b| {red}", flush=True)
    for l0 in (2, 3):
        assert max(red[(1, l0)]) < 0.5
        assert max(red[(1, l0)]) <= 1.05 * max(red[(0, l0)])


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6), (2, 1e-6)])
def test_line_smoother_step_matches_oracle(precision, tol):
    """One step with the line-smoothed V-cycle (levels 0-2 of a 4-level 33x33x9
    hierarchy swept by separate launches; with precision 2 the finest level's lines are
    swept over its FP16 scaled matrix) reaches the oracle's root."""
    nx, ny, nz = 33, 33, 9
    phys = synth.physics(2)
    xi = _xi(2, 2, seed=6)
    pb = _problem(phys, [(nx, ny, nz, 4, 2)], precision=precision, smoother=1)
    pb.set_parameters(xi)
    pb.set_tuning(0, 3)
    st = pb.step(DT)
    assert all(t["status"] == 0 for t in st), st
    box = elder.Box(nx, ny, nz, phys)
    for s in range(2):
        ref = newton.newton_solve(box, elder.coefficients(box, xi[s]),
                                  synth.initial_state(nx, ny, nz, phys), DT)
        got = pb.get_state(s)
        for f in range(2):
            assert _rel(got[..., f], ref[..., f]) < tol, (s, f)
    pb.destroy()


def test_matrix_free_product_equals_the_assembled_jacobian():
    """The matrix-free J~ x (directional derivative of the defect at the state, upwind
    frozen) against the product with the assembled exact Jacobian, at random states and
    directions, every field model: equal to rounding (1e-12 of the largest entry).  The
    second shape has columns of 19 vertices, walked in 3 segments; the third spans 4 x 2
    tiles of hexahedron columns (a ragged last tile each way) and 2 segments."""
    for (nx, ny, nz, levels), models in (((17, 13, 5, 3), (0, 1, 2, 3)), ((11, 9, 19, 2), (1, 2)),
                                         ((49, 29, 13, 3), (2, 3))):
        for model in models:
            phys = synth.physics(model)
            xi = _xi(model, 2, seed=21)
            ys = []
            for mf in (0, 1):
                pb = _problem(phys, [(nx, ny, nz, levels, 2)], matrix_free=mf)
                pb.set_parameters(xi)
                for s in range(2):
                    pb.set_state(s, synth.random_state(nx, ny, nz, phys, seed=40 + s))
                x = np.random.default_rng(7).standard_normal((2, nz, ny, nx, 2))
                pb.apply_vcycle(0, DT, x)  # assembles at the states with this step length
                ys.append(pb.apply_jacobian(0, x))
                pb.destroy()
            err = np.abs(ys[1] - ys[0]).max() / np.abs(ys[0]).max()
            print(f"{nx}x{ny}x{nz} model {model}: matrix-free vs assembled {err:.2e}", flush=True)
            assert err < 1e-12, (model, err)


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
def test_matrix_free_step_matches_oracle(precision, tol):
    nx, ny, nz = 33, 33, 9
    phys = synth.physics(2)
    xi = _xi(2, 2, seed=16)
    pb = _problem(phys, [(nx, ny, nz, 4, 2)], precision=precision, matrix_free=1)
    pb.set_parameters(xi)
    st = pb.step(DT)
    assert all(t["status"] == 0 for t in st), st
    box = elder.Box(nx, ny, nz, phys)
    for s in range(2):
        ref = newton.newton_solve(box, elder.coefficients(box, xi[s]),
                                  synth.initial_state(nx, ny, nz, phys), DT)
        for f in range(2):
            assert _rel(pb.get_state(s)[..., f], ref[..., f]) < tol, (s, f)
    pb.destroy()


def test_autotuned_step_matches_default():
    """Autotuning times the V-cycle for every fused-bottom choice, keeps the fastest,
    leaves the states alone, and the step then solves the same system to the same
    state."""
    nx, ny, nz = 33, 33, 9
    phys = synth.physics(2)
    xi = _xi(2, 2, seed=12)
    out = {}
    for tune in (0, 1):
        pb = _problem(phys, [(nx, ny, nz, 4, 2)])
        pb.set_parameters(xi)
        if tune:
            pb.autotune(DT)
            assert _rel(pb.get_state(1), synth.initial_state(nx, ny, nz, phys)) < 1e-14
        st = pb.step(DT)
        assert all(x["status"] == 0 for x in st)
        out[tune] = np.stack([pb.get_state(s) for s in range(2)])
        l0, ms = pb.tuning(0)
        print(f"autotune {tune}: fused from level {l0}, V-cycle ms {ms}", flush=True)
        if tune:
            assert all(ms[l] > 0 for l in (1, 2, 3)) and ms[0] == -1.0
            assert ms[l0] == min(ms[1:])
        else:
            assert l0 == 3 and all(ms == -1.0)  # 2 samples: only the coarse solve fused
        pb.destroy()
    assert _rel(out[1], out[0]) < 1e-12


@pytest.mark.parametrize("conc,precision,groups", [
    (1, 0, [(9, 9, 3, 2, 3), (17, 17, 5, 3, 2), (33, 33, 9, 4, 2)]),
    (2, 0, [(9, 9, 3, 2, 3), (17, 17, 5, 3, 2), (33, 33, 9, 4, 2)]),
    (2, 1, [(9, 9, 3, 2, 3), (17, 17, 5, 3, 2), (33, 33, 9, 4, 2)]),
    (2, 0, [(17, 13, 5, 3, 3), (33, 33, 9, 4, 2), (33, 33, 9, 3, 2)])])
def test_concurrent_groups_give_the_serial_result(conc, precision, groups):
    """Groups advanced at the same time reach bitwise the states and solver counts of groups
    advanced one after the other: with one host thread and stream each (1), and with one
    thread each on a shared stream where the V-cycles of the groups inside BiCGStab run
    together, each level that groups share (same grid, same role) swept by one launch over
    all their samples (2).  The last grid set has levels that do not line up (a 17x13x5
    group, two 33x33x9 groups whose hierarchies end at different depths), which run as
    separate launches.  Merging only removes launches: with edf_profile on, the merged
    run counts no more smoother launches than the serial one."""
    phys = synth.physics(2)
    S = sum(g[4] for g in groups)
    xi = _xi(2, S, seed=21)
    xi[3] = 0.9  # a high-permeability sample that needs sub-steps at 4 months
    out, launches = {}, {}
    for c in (0, conc):
        pb = _problem(phys, groups, concurrent_groups=c, dt_max_halvings=4, precision=precision,
                      check_every=1)
        pb.set_parameters(xi)
        pb.profile(True)
        sts = [pb.step(4 * DT) for _ in range(2)]
        launches[c] = pb.profile(False)["all_launches"]
        out[c] = ([pb.get_state(s) for s in range(S)],
                  [[(x["status"], x["newton_its"], x["lin_its"], x["substeps"]) for x in st]
                   for st in sts])
        pb.destroy()
    print("sub-steps", [x[3] for x in out[conc][1][1]], "smoother launches", launches,
          flush=True)
    assert out[conc][1] == out[0][1]
    for s in range(S):
        assert np.array_equal(out[conc][0][s], out[0][0][s]), s
    assert launches[conc] <= launches[0]


def _zero_start_blocks(c):
    """Stencil blocks of vertex colour c that a forward sweep from x = 0 needs: those of
    the neighbours whose colour (c with the parity bit of each odd offset flipped) was
    swept before c."""
    n = 0
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                m = (dx != 0) | ((dy != 0) << 1) | ((dz != 0) << 2)
                n += (c ^ m) < c
    return n


def _colour_counts(nx, ny, nz):
    """Vertices of each colour (i % 2) + 2 (j % 2) + 4 (k % 2)."""
    return [((nx + 1 - (c & 1)) // 2) * ((ny + 1 - ((c >> 1) & 1)) // 2)
            * ((nz + 1 - (c >> 2)) // 2) for c in range(8)]


@pytest.mark.parametrize("precision,concurrent", [(0, 0), (1, 0), (0, 1)])
def test_graph_vcycle_gives_the_eager_result(precision, concurrent):
    """V-cycles captured as HIP graphs and replayed (graph_vcycle = 1) give bitwise the
    states, solver counts and V-cycle outputs of the V-cycles launched one by one: three
    steps of a mixed-resolution batch (each replaying the captured graphs many times, with
    other launches and host synchronisations between the replays, and with the sample
    list shrinking as samples converge), then two applications of one V-cycle; also with
    the groups captured and replayed from their own host threads at the same time."""
    phys = synth.physics(2)
    groups = [(17, 17, 5, 3, 3), (33, 33, 9, 4, 4)]
    xi = _xi(2, 7, seed=23)
    b = np.random.default_rng(9).standard_normal((4, 9, 33, 33, 2))
    b[..., 1][:, -1] = 0.0
    out = {}
    for graph in (0, 1):
        pb = _problem(phys, groups, precision=precision, graph_vcycle=graph, check_every=1,
                      dt_max_halvings=4, concurrent_groups=concurrent * graph)
        pb.set_parameters(xi)
        sts = [pb.step(DT) for _ in range(3)]
        ys = [pb.apply_vcycle(1, DT, b) for _ in range(2)]
        out[graph] = ([pb.get_state(s) for s in range(7)],
                      [[(x["status"], x["newton_its"], x["lin_its"], x["substeps"]) for x in st]
                       for st in sts], ys)
        pb.destroy()
    print("lin its", [sum(x[2] for x in st) for st in out[1][1]], flush=True)
    assert out[1][1] == out[0][1]
    for s in range(7):
        assert np.array_equal(out[1][0][s], out[0][0][s]), s
    for y1, y0 in zip(out[1][2], out[0][2]):
        assert np.array_equal(y1, y0)
    assert np.array_equal(out[1][2][0], out[1][2][1])


def test_profile_counts_launches_and_algorithmic_bytes():
    """edf_profile: every smoother launch is counted with its algorithmic bytes (118
    values per vertex of the swept colour and active sample; the first forward sweep of a
    level, from x = 0, 4 per stencil block of an already swept neighbour colour plus 8,
    its colour 0 done by the kernel that writes b, not by a smoother launch), every 13th
    is timed, and every V-cycle is timed."""
    nx, ny, nz, L, S = 33, 33, 9, 4, 2
    phys = synth.physics(2)
    pb = _problem(phys, [(nx, ny, nz, L, S)], smoother=0)
    pb.set_parameters(_xi(2, S))
    pb.set_tuning(0, L - 1)  # levels 0..2 smoothed by separate launches
    b = np.random.default_rng(1).standard_normal((S, nz, ny, nx, 2))
    pb.profile(True)
    pb.apply_vcycle(0, DT, b)
    pr = pb.profile(False)
    grids = [(33, 33, 9), (17, 17, 5), (9, 9, 3)]
    assert sum(_zero_start_blocks(c) for c in range(8)) == 8 * 13
    expect = 0
    for g in grids:
        cnt = _colour_counts(*g)
        assert sum(cnt) == g[0] * g[1] * g[2]
        expect += S * 8 * sum(n * (118 + (4 * _zero_start_blocks(c) + 8 if c > 0 else 0))
                              for c, n in enumerate(cnt))
    assert pr["all_launches"] == 3 * 15
    assert pr["launches"] == len(range(0, 45, 13))
    assert pr["all_bytes"] == expect
    assert pr["vcycles"] == 1 and pr["vcycle_ms"] > 0 and pr["ms"] > 0
    # two 33x33x9 samples: no launch and no V-cycle beyond the 256 MiB last-level cache
    assert pr["large_vcycles"] == 0 and pr["large_all_launches"] == 0
    pb.destroy()


def test_profile_counts_line_smoother_launches():
    """edf_profile with the vertical-line smoother: 4 column colours per sweep, each
    vertex of a colour's columns counted with the blocks towards the other columns (24,
    or from x = 0 the 0, 6, 18, 24 towards the colours already swept), the block above,
    the 8 factor values, b, and x written, read and written again (116 values)."""
    nx, ny, nz, L, S = 33, 33, 9, 4, 2
    phys = synth.physics(2)
    pb = _problem(phys, [(nx, ny, nz, L, S)], smoother=1)
    pb.set_parameters(_xi(2, S))
    pb.set_tuning(0, L - 1)  # levels 0..2 line-smoothed by separate launches
    b = np.random.default_rng(1).standard_normal((S, nz, ny, nx, 2))
    pb.profile(True)
    pb.apply_vcycle(0, DT, b)
    pr = pb.profile(False)
    zs_blocks = [0, 6, 18, 24]
    expect = 0
    for (gx, gy, gz) in [(33, 33, 9), (17, 17, 5), (9, 9, 3)]:
        for cc in range(4):
            ncol = ((gx + 1 - (cc & 1)) // 2) * ((gy + 1 - (cc >> 1)) // 2)
            per = (4 * (zs_blocks[cc] + 1) + 16) + (4 * 25 + 16)  # pre (from zero), post
            expect += S * ncol * gz * per * 8
    assert pr["all_launches"] == 3 * 8
    assert pr["all_bytes"] == expect
    pb.destroy()


@pytest.mark.parametrize("precision", [1, 2])
def test_mixed_precision_step_matches_fp64_oracle(precision):
    nx, ny, nz = 33, 33, 9
    phys = synth.physics(2)
    xi = _xi(2, 1, seed=6)
    pb = _problem(phys, [(nx, ny, nz, 4, 1)], precision=precision)
    pb.set_parameters(xi)
    pb.step(DT)
    box = elder.Box(nx, ny, nz, phys)
    ref = newton.newton_solve(box, elder.coefficients(box, xi[0]),
                              synth.initial_state(nx, ny, nz, phys), DT)
    got = pb.get_state(0)
    for f in range(2):
        assert _rel(got[..., f], ref[..., f]) < 1e-6
    pb.destroy()


def test_single_level_and_thinnest_grid():
    """Edge cases: one grid only (the dense coarse solve is the whole preconditioner)
    and the thinnest grid nz = 2."""
    for shape, levels in [((5, 5, 3), 1), ((9, 9, 2), 1), ((5, 5, 2), 1), ((9, 9, 5), 3)]:
        nx, ny, nz = shape
        phys = synth.physics(0)
        pb = _problem(phys, [(nx, ny, nz, levels, 1)])
        pb.set_parameters(np.zeros((1, 0)))
        pb.step(DT)
        box = elder.Box(nx, ny, nz, phys)
        ref = newton.newton_solve(box, elder.coefficients(box, []),
                                  synth.initial_state(nx, ny, nz, phys), DT)
        got = pb.get_state(0)
        for f in range(2):
            assert _rel(got[..., f], ref[..., f]) < 1e-10, (shape, f)
        pb.destroy()


def test_invalid_arguments_are_rejected():
    from paper_1906_01632_amd import EDFError
    phys = synth.physics(2)
    with pytest.raises(EDFError):
        _problem(phys, [(10, 9, 3, 2, 1)])        # 9 not divisible by 2
    with pytest.raises(EDFError):
        _problem(phys, [(65, 65, 17, 2, 1)])      # coarsest grid too large for the dense solve
    pb = _problem(phys, [(9, 9, 3, 2, 1)])
    with pytest.raises(EDFError):
        pb.step(DT)                               # parameters not set
    with pytest.raises(EDFError):
        pb.set_parameters(np.full((1, 4), 1.5))   # |xi| > 1
    pb.set_parameters(np.zeros((1, 4)))
    with pytest.raises(EDFError):
        pb.step(-1.0)
    with pytest.raises(EDFError):
        pb.moments((4, 9, 3))                     # not nested
    with pytest.raises(EDFError):
        pb.moments((9, 9, 3), weights=[-0.5])     # weights summing to a non-positive value
    pb.destroy()
    with pytest.raises(EDFError):
        _problem(phys, [(9, 9, 3, 2, 0)])         # no samples
    with pytest.raises(EDFError):
        _problem(phys, [(9, 9, 3, 0, 1)])         # no levels
    with pytest.raises(EDFError):
        _problem(phys, [(1, 9, 3, 1, 1)])         # a dimension of one vertex


def test_failed_step_is_redone_as_equal_substeps():
    """A 4-month step of a high-permeability sample lands on a spurious root (c < 0)
    in one Newton solve; the library redoes it as 2^h equal sub-steps, and the oracle
    replaying the same sub-steps gives the same state.  The other sample of the batch
    takes the step whole."""
    nx, ny, nz = 17, 17, 5
    phys = synth.physics(2)
    xi = np.array([[0.0, 0.0, 0.0, 0.0], [0.9, 0.9, 0.9, 0.9]])
    dt = 4 * DT
    pb = _problem(phys, [(nx, ny, nz, 3, 2)], dt_max_halvings=4)
    pb.set_parameters(xi)
    st = pb.step(dt)
    print("substeps", [s["substeps"] for s in st], "status", [s["status"] for s in st], flush=True)
    assert [s["status"] for s in st] == [0, 0]
    assert st[0]["substeps"] == 1 and st[1]["substeps"] >= 2
    box = elder.Box(nx, ny, nz, phys)
    for s in range(2):
        coef = elder.coefficients(box, xi[s])
        u = synth.initial_state(nx, ny, nz, phys)
        m = st[s]["substeps"]
        for _ in range(m):
            u = newton.newton_solve(box, coef, u, dt / m)
        got = pb.get_state(s)
        assert got[..., 1].min() >= -1e-9
        for f in range(2):
            assert _rel(got[..., f], u[..., f]) < 1e-10, (s, f)
    pb.destroy()


def test_sample_failure_is_reported_and_left_out_of_moments():
    """Without step halving the spurious root is rejected: that sample reports the
    failure, keeps its state, and the moments use the other sample only."""
    nx, ny, nz = 17, 17, 5
    phys = synth.physics(2)
    xi = np.array([[0.0, 0.0, 0.0, 0.0], [0.9, 0.9, 0.9, 0.9]])
    pb = _problem(phys, [(nx, ny, nz, 3, 2)], dt_max_halvings=0)
    pb.set_parameters(xi)
    before = pb.get_state(1)
    st = pb.step(4 * DT)
    assert st[0]["status"] == 0 and st[1]["status"] != 0
    np.testing.assert_array_equal(pb.get_state(1), before)
    mean, var, exc = pb.moments((9, 9, 3))
    c0 = stats.inject(pb.get_state(0)[..., 1], (9, 9, 3))
    assert np.abs(mean - c0).max() < 1e-15 and np.abs(var).max() < 1e-30
    pb.destroy()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_line_tile_shapes_give_the_same_vcycle(precision, tmp_path):
    """The line sweep's tile shapes (8, 16, 32 columns per workgroup) compute every column
    the same way: one V-cycle gives bitwise the same output with each shape.  Invalid
    shapes are rejected with nothing changed, and an autotuning stored in a JSON cache is
    applied again by a second problem of the same key."""
    from paper_1906_01632_amd import EDFError
    phys = synth.physics(2)
    groups = [(33, 33, 9, 4, 3)]
    b = np.random.default_rng(5).standard_normal((3, 9, 33, 33, 2))
    b[..., 1][:, -1] = 0.0
    pb = _problem(phys, groups, precision=precision)
    pb.set_parameters(_xi(2, 3, seed=4))
    pb.set_tuning(0, 3)  # levels 0-2 swept by their own launches
    ys = {}
    for c in (8, 16, 32):
        pb.set_line_tiles(0, [c, c, c, 0])
        assert pb.line_tiles(0) == [c, c, c, 0]
        ys[c] = pb.apply_vcycle(0, DT, b)
    assert np.array_equal(ys[8], ys[16]) and np.array_equal(ys[32], ys[16])
    for bad in ([12, 16, 16, 0], [16, 16, 16, 8]):
        with pytest.raises(EDFError):
            pb.set_line_tiles(0, bad)
    assert pb.line_tiles(0) == [32, 32, 32, 0]
    cache = str(tmp_path / "tuning.json")
    assert pb.autotune(DT, cache=cache) is True
    tuned = (pb.tuning(0)[0], pb.line_tiles(0))
    pb.destroy()
    pb2 = _problem(phys, groups, precision=precision)
    pb2.set_parameters(_xi(2, 3, seed=4))
    assert pb2.autotune(DT, cache=cache) is False
    assert (pb2.tuning(0)[0], pb2.line_tiles(0)) == tuned
    pb2.destroy()


def test_joint_tuning_gives_groups_one_fused_bottom():
    """With merged V-cycles (concurrent_groups = 2) the autotuner fuses the same number of
    levels in every group (the groups' coarse grids are the same), so that their bottoms
    share one launch; the tuned problem steps to bitwise the result of the serial one."""
    phys = synth.physics(2)
    groups = [(17, 17, 5, 3, 3), (33, 33, 9, 4, 2)]
    xi = _xi(2, 5, seed=31)
    pb = _problem(phys, groups, concurrent_groups=2, check_every=1)
    pb.set_parameters(xi)
    pb.autotune(DT)
    fused = [g[3] - pb.tuning(i)[0] for i, g in enumerate(groups)]
    assert fused[0] == fused[1], fused
    pb.step(DT)
    got = [pb.get_state(s) for s in range(5)]
    pb.destroy()
    ref = _problem(phys, groups, check_every=1)
    ref.set_parameters(xi)
    for i, g in enumerate(groups):
        ref.set_tuning(i, g[3] - fused[i])
    ref.step(DT)
    for s in range(5):
        assert np.array_equal(ref.get_state(s), got[s]), s
    ref.destroy()
