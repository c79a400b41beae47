"""Parity at the benchmark sizes (129x129x33, 257x257x65, the three qMC grids), in the
launch configuration bench.py times (Eisenstat-Walker forcing, one convergence check
per BiCGStab iteration).  The oracle cannot run Newton with direct solves at these
sizes; it checks every output through properties that hold at any size: its own
residual evaluated at the GPU's converged states, element-wise defect parity, and
the statistics of the injected fields.  GPU."""
import numpy as np
import pytest

import synth
from oracle import elder, stats

pytestmark = pytest.mark.gpu

DT = synth.MONTH_S
BENCH_OPTS = dict(lin_rtol=1e-6, lin_max_it=100, newton_max_it=20, check_every=1, forcing=1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _problem(phys, groups, **opts):
    from paper_1906_01632_amd import Problem
    o = dict(BENCH_OPTS)
    o.update(opts)
    return Problem(phys, groups, o)


def _oracle_scaled_norm(box, coef, u, u_old, dt=DT):
    F = elder.residual(box, coef, u, u_old, dt) * elder.row_scale(box, dt)
    return float(np.linalg.norm(F))


def _substep_states(phys, group, xi, sub, opts):
    """The sub-step states of one sample's split step: the sample alone, stepped `sub`
    times by DT / sub (each of those steps is the Newton solve of the split step's
    sub-step, bitwise)."""
    pb = _problem(phys, [group[:4] + (1,)], **opts)
    pb.set_parameters(xi[None])
    states = [pb.get_state(0)]
    for _ in range(sub):
        st = pb.step(DT / sub)
        assert st[0]["status"] == 0 and st[0]["substeps"] == 1, st
        states.append(pb.get_state(0))
    pb.destroy()
    return states


def test_defect_parity_129_every_vertex():
    nx, ny, nz = 129, 129, 33
    phys = synth.physics(2)
    xi = synth.lattice_points(512, 4, 0)[1:2]
    pb = _problem(phys, [(nx, ny, nz, 6, 1)])
    pb.set_parameters(xi)
    u = synth.random_state(nx, ny, nz, phys, seed=3)
    uo = synth.random_state(nx, ny, nz, phys, seed=4)
    got = pb.residual(0, u, uo, DT)
    box = elder.Box(nx, ny, nz, phys)
    ref = elder.residual(box, elder.coefficients(box, xi[0]), u, uo, DT) * elder.row_scale(box, DT)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
    pb.destroy()


def test_qmc_groups_step_solves_the_oracle_system():
    """Two lattice samples of each resolution of the qMC workload in one problem: every
    converged state zeroes the oracle's residual to the Newton tolerance, and the pooled
    moments on the 33x33x9 grid are the oracle statistics of the same fields."""
    wl = synth.workload("qmc512_mixedres")
    phys = synth.physics(wl.field_model)
    groups, xis, off = [], [], 0
    for g in wl.groups:
        groups.append((g.nx, g.ny, g.nz, g.levels, 2))
        xis.append(wl.xi[off:off + 2])
        off += g.samples
    xi = np.concatenate(xis)
    pb = _problem(phys, groups, newton_rtol=wl.newton_rtol)
    pb.set_parameters(xi)
    st = pb.step(DT)
    fields = []
    for s in range(6):
        nx, ny, nz = groups[s // 2][:3]
        box = elder.Box(nx, ny, nz, phys)
        coef = elder.coefficients(box, xi[s])
        u0 = synth.initial_state(nx, ny, nz, phys)
        u = pb.get_state(s)
        sub = st[s]["substeps"]
        # a split step is replayed sub-step by sub-step; every sub-step's state zeroes the
        # oracle's residual of that sub-step
        states = [u0, u] if sub == 1 else _substep_states(
            phys, groups[s // 2], xi[s], sub, dict(newton_rtol=wl.newton_rtol))
        np.testing.assert_array_equal(states[-1], u)
        for k in range(1, len(states)):
            r0 = _oracle_scaled_norm(box, coef, states[k - 1], states[k - 1], DT / sub)
            r = _oracle_scaled_norm(box, coef, states[k], states[k - 1], DT / sub)
            print(f"sample {s} {nx}x{ny}x{nz} sub-step {k}/{sub}: oracle |F~| {r:.3e} of {r0:.3e}",
                  flush=True)
            assert r <= 2 * wl.newton_rtol * r0 + 1e-10
        assert -0.05 <= u[..., 1].min() and u[..., 1].max() <= 1.05
        fields.append(stats.inject(u[..., 1], (33, 33, 9)))
    mean, var, exc = pb.moments((33, 33, 9), threshold=0.5)
    m, v, e = stats.moments(np.array(fields), threshold=0.5)
    assert np.abs(mean - m).max() < 1e-14 and np.abs(var - v).max() < 1e-14
    assert np.abs(exc - e).max() < 1e-14
    pb.destroy()


def test_single_129_cosine_field_step_solves_the_oracle_system():
    """The plain single-sample FP64 path of the 129x129x33 workload (one cosine mode of
    phi, Kozeny-Carman K, xi1 from the seed): its first step zeroes the oracle's residual
    to the Newton tolerance (replayed sub-step by sub-step if it was split)."""
    wl = synth.workload("elder129_f64")
    phys = synth.physics(wl.field_model)
    g = wl.groups[0]
    group = (g.nx, g.ny, g.nz, g.levels, 1)
    pb = _problem(phys, [group], newton_rtol=wl.newton_rtol)
    pb.set_parameters(wl.xi)
    st = pb.step(DT)
    assert st[0]["status"] == 0, st
    u = pb.get_state(0)
    pb.destroy()
    box = elder.Box(g.nx, g.ny, g.nz, phys)
    coef = elder.coefficients(box, wl.xi[0])
    sub = st[0]["substeps"]
    states = ([synth.initial_state(g.nx, g.ny, g.nz, phys), u] if sub == 1 else
              _substep_states(phys, group, wl.xi[0], sub, dict(newton_rtol=wl.newton_rtol)))
    for k in range(1, len(states)):
        r0 = _oracle_scaled_norm(box, coef, states[k - 1], states[k - 1], DT / sub)
        r = _oracle_scaled_norm(box, coef, states[k], states[k - 1], DT / sub)
        print(f"129 cosine field, xi1 = {wl.xi[0, 0]:.4f}, sub-step {k}/{sub}: |F~| {r:.3e} of "
              f"{r0:.3e}", flush=True)
        assert r <= 2 * wl.newton_rtol * r0 + 1e-10
    assert -0.05 <= u[..., 1].min() and u[..., 1].max() <= 1.05


def test_qmc_batch_mixed_precision_matches_fp64():
    """A slice of the qMC workload (8 lattice samples of each of its three grids, in one
    problem, the benchmark's options): two steps with the FP32 V-cycle, and with the
    finest matrix in FP16, against the FP64 V-cycle.  Samples that took the same
    sub-steps in both runs agree to 1e-6 relative L2 per field (the bar of the mixed
    path); every state is admissible."""
    wl = synth.workload("qmc512_mixedres")
    phys = synth.physics(wl.field_model)
    groups, xis, off = [], [], 0
    for g in wl.groups:
        groups.append((g.nx, g.ny, g.nz, g.levels, 8))
        xis.append(wl.xi[off:off + 8])
        off += g.samples
    xi = np.concatenate(xis)
    out = {}
    for prec in (0, 1, 2):
        pb = _problem(phys, groups, newton_rtol=wl.newton_rtol, precision=prec)
        pb.set_parameters(xi)
        subs = []
        for _ in range(2):
            st = pb.step(DT)
            assert all(t["status"] == 0 for t in st), st
            subs.append([t["substeps"] for t in st])
        out[prec] = ([pb.get_state(s) for s in range(24)], np.array(subs))
        pb.destroy()
    compared = 0
    for prec in (1, 2):
        for s in range(24):
            if not np.array_equal(out[prec][1][:, s], out[0][1][:, s]):
                print(f"precision {prec} sample {s}: sub-steps {out[prec][1][:, s]} vs "
                      f"{out[0][1][:, s]}, not compared", flush=True)
                continue
            compared += 1
            for f in range(2):
                a, b = out[prec][0][s][..., f], out[0][0][s][..., f]
                rel = np.linalg.norm(a - b) / np.linalg.norm(b)
                assert rel <= 1e-6, (prec, s, f, rel)
            assert -0.05 <= out[prec][0][s][..., 1].min() <= out[prec][0][s][..., 1].max() <= 1.05
    print(f"{compared} of 48 mixed/FP64 sample pairs compared", flush=True)
    assert compared >= 40


def test_mixed_257_matches_fp64_and_solves_the_oracle_system():
    """The mixed-precision workload's shapes: a 257x257x65 sample and a 129x129x33 sample,
    FP32 V-cycle (and FP32 with the finest matrix stored in FP16); each result agrees
    with the FP64-V-cycle result to 1e-6 relative L2 per field, and the oracle's
    residual at the mixed result meets the Newton tolerance."""
    wl = synth.workload("mixed257")
    phys = synth.physics(wl.field_model)
    groups = [(257, 257, 65, 7, 1), (129, 129, 33, 6, 1)]
    xi = wl.xi[:2]
    out = {}
    for prec in (2, 1, 0):
        pb = _problem(phys, groups, newton_rtol=wl.newton_rtol, precision=prec)
        pb.set_parameters(xi)
        st = pb.step(DT)
        assert all(s["status"] == 0 for s in st), st
        out[prec] = [pb.get_state(s) for s in range(2)]
        out[("sub", prec)] = [s["substeps"] for s in st]
        pb.destroy()
    for prec in (1, 2):  # FP32 V-cycle; FP32 with the finest matrix in FP16
        assert out[("sub", 0)] == out[("sub", prec)]
        for s in range(2):
            for f in range(2):
                a, b = out[prec][s][..., f], out[0][s][..., f]
                rel = np.linalg.norm(a - b) / np.linalg.norm(b)
                print(f"precision {prec} sample {s} field {f}: vs FP64 rel L2 {rel:.2e}",
                      flush=True)
                assert rel <= 1e-6
    if out[("sub", 1)][0] != 1:
        return  # the step was split; the state does not solve the full-step system
    nx, ny, nz = 257, 257, 65
    box = elder.Box(nx, ny, nz, phys)
    coef = elder.coefficients(box, xi[0])
    u0 = synth.initial_state(nx, ny, nz, phys)
    r0 = _oracle_scaled_norm(box, coef, u0, u0)
    r = _oracle_scaled_norm(box, coef, out[1][0], u0)
    print(f"257: oracle |F~| at the mixed result {r:.3e} of {r0:.3e}", flush=True)
    assert r <= 2 * wl.newton_rtol * r0 + 1e-10
