"""Pins of the oracle against things other than itself.

Each test checks the oracle against a value the paper prints, a closed form, a
conservation identity, a symmetry, a textbook routine or brute force, chosen so
that a dropped term, a wrong sign or index, or a transposed operand fails one of
them.  CPU only.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import elder, newton, stats

GOLD = os.path.join(os.path.dirname(__file__), "golden")
DT = synth.MONTH_S


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- counts ---

def test_paper_grid_counts():
    """Section 2.1: 524,288 hexahedra and 1,098,306 DoFs; Conclusion: 4,194,304 cells."""
    g = _load("paper_counts.json")
    ph = synth.physics()
    nx, ny, nz = 129, 129, 33
    assert (nx - 1) * (ny - 1) * (nz - 1) == g["box_coarse_hexahedra"]
    assert 2 * nx * ny * nz == g["box_coarse_dofs"]
    assert 256 * 256 * 64 == g["box_fine_cells"]
    # equal spacing in all directions for the paper's box
    box = elder.Box(5, 5, 2, ph)
    assert box.h == (150.0, 150.0, 150.0)
    assert math.isclose(g["box_steps"] * g["box_dt_years"], g["box_total_years"])


def test_table1_and_rayleigh():
    """Table 1 values; D_m = 3.565e-6 gives the Elder Rayleigh number 400."""
    t = _load("table1.json")
    ph = synth.physics()
    for key in ("phi_mean", "K_mean", "g", "rho0", "rho1", "mu"):
        assert ph[key] == t[key]
    ra = ph["K_mean"] * (ph["rho1"] - ph["rho0"]) * ph["g"] * ph["lz"] / (
        ph["phi_mean"] * ph["Dm"] * ph["mu"])
    assert abs(ra - 400.0) < 0.05
    ra_printed = ra * ph["Dm"] / t["Dm_printed"]
    assert ra_printed > 2000  # the printed value would not be the Elder problem


def test_kozeny_carman_normalisation():
    """Section 2.2: the scaling constant makes K(E phi) = E K."""
    ph = synth.physics(1)
    assert elder.kozeny_carman(np.array(0.1), ph) == pytest.approx(4.845e-13, rel=1e-15)
    # monotone and cubic for small phi
    r = elder.kozeny_carman(np.array(0.02), ph) / elder.kozeny_carman(np.array(0.01), ph)
    assert 8.0 < r < 8.2


def test_kozeny_carman_denominator():
    """K at phi = 0.08 and 0.12 from the perturbed-field workload's law (phi/0.1)^3
    ((1-0.1)/(1-phi))^2, hand-computed; the paper's printed phi^3/(1-phi^2) (normalised
    the same way) differs by 2-4 % there, so the reading is pinned, not only K(E phi)."""
    g = _load("field_values.json")["kozeny_carman"]
    ph = synth.physics(1)
    for phi, want, printed in zip(g["phi"], g["K_over_Kmean"], g["K_over_Kmean_printed_form"]):
        got = elder.kozeny_carman(np.array(phi), ph) / ph["K_mean"]
        assert got == pytest.approx(want, rel=1e-14)
        assert abs(got - printed) > 0.02 * printed


@pytest.mark.parametrize("model", [1, 2, 3])
def test_field_models_at_exact_points(model):
    """phi and K per hexahedron on small grids whose centroids make every trigonometric
    factor exact (+-1/2, +-sqrt(2)/2, +-sqrt(3)/2, 0, 1), hand-computed from the field
    formulas (model 3: the paper's eq. poro-paral3RVS).  The grids give the x, y and z
    factors different values, so a swapped coordinate, a sin for a cos, a dropped
    cross term or a wrong amplitude changes some entry."""
    g = _load("field_values.json")[f"model{model}"]
    nx, ny, nz = g["grid"]
    box = elder.Box(nx, ny, nz, synth.physics(model))
    np.testing.assert_allclose(box.xc[0, 0, :], g["centroid_x"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(box.yc[0, :, 0], g["centroid_y"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(box.zc[:, 0, 0], g["centroid_z"], rtol=0, atol=1e-12)
    phi, K = elder.coefficients(box, g["xi"])
    np.testing.assert_allclose(phi.ravel(), g["phi"], rtol=1e-14)
    np.testing.assert_allclose(K.ravel(), g["K"], rtol=1e-13)


@pytest.mark.parametrize("shape", [(33, 33, 9), (65, 65, 17)])
def test_boundary_vertex_sets(shape):
    """The closed top patch [150, 450]^2 (its edge vertices included), the bottom face and
    the four pinned top corners, counted on the workloads' grids."""
    g = _load("field_values.json")["patch_vertices"]["x".join(map(str, shape))]
    box = elder.Box(*shape, synth.physics(0))
    cmask, cval = box.dirichlet_c()
    assert int((cmask & (cval == 1.0)).sum()) == g["patch"]
    assert int((cmask & (cval == 0.0)).sum()) == g["bottom"]
    assert int(cmask.sum()) == g["patch"] + g["bottom"]
    assert int(box.pinned_p().sum()) == g["pinned_p"]
    u0 = synth.initial_state(*shape, synth.physics(0))
    assert int((u0[..., 1] == 1.0).sum()) == g["patch"]


# -------------------------------------------------------------- jacobian ---

@pytest.mark.parametrize("shape,model", [((5, 5, 2), 0), ((5, 5, 3), 2), ((7, 5, 3), 1),
                                         ((5, 7, 4), 3)])
def test_jacobian_is_complex_step_derivative(shape, model):
    """Every entry of the analytic Jacobian equals the complex-step derivative of F."""
    ph = synth.physics(model)
    nx, ny, nz = shape
    box = elder.Box(nx, ny, nz, ph)
    xi = np.random.default_rng(7).uniform(-1, 1, synth.N_XI[model])
    coef = elder.coefficients(box, xi)
    u = synth.random_state(nx, ny, nz, ph, seed=11)
    u_old = synth.random_state(nx, ny, nz, ph, seed=12)
    J = elder.jacobian(box, coef, u, DT).toarray()
    n = 2 * box.N
    h = 1e-30
    Jcs = np.zeros((n, n))
    flat = u.reshape(-1).astype(complex)
    for col in range(n):
        uc = flat.copy()
        uc[col] += 1j * h
        Jcs[:, col] = elder.residual(box, coef, uc.reshape(u.shape), u_old, DT).imag.ravel() / h
    scale = np.abs(J).max(axis=1, keepdims=True)
    assert np.max(np.abs(J - Jcs) / scale) < 1e-13


def test_stencil_is_27_point_2x2_block():
    """Every row couples only the 3x3x3 vertex neighbourhood (2x2 blocks)."""
    ph = synth.physics(2)
    box = elder.Box(7, 7, 5, ph)
    coef = elder.coefficients(box, [0.3, -0.2, 0.5, 0.1])
    u = synth.random_state(7, 7, 5, ph, seed=3)
    J = elder.jacobian(box, coef, u, DT).tocoo()
    vr, vc = J.row // 2, J.col // 2
    ir, jr, kr = vr % 7, (vr // 7) % 7, vr // 49
    ic, jc, kc = vc % 7, (vc // 7) % 7, vc // 49
    assert max(np.abs(ir - ic).max(), np.abs(jr - jc).max(), np.abs(kr - kc).max()) == 1
    # an interior vertex row has all 27 neighbours
    v = 3 + 7 * (3 + 7 * 2)
    assert len(set(vc[vr == v])) == 27


# ------------------------------------------------------- closed forms ------

@pytest.mark.parametrize("model", [0, 2])
def test_hydrostatic_state_is_a_fixed_point(model):
    """c = 0 everywhere (patch switched off), p = rho0 g z: no flow, F = 0, and one
    Newton-solved step returns the same state."""
    ph = synth.physics(model, patch=(-10.0, -5.0, -10.0, -5.0))
    nx, ny, nz = 9, 9, 3
    box = elder.Box(nx, ny, nz, ph)
    coef = elder.coefficients(box, [0.7, -0.4, 0.9, -1.0][:synth.N_XI[model]])
    u = np.zeros((nz, ny, nx, 2))
    u[..., 0] = ph["rho0"] * ph["g"] * box.z
    F = elder.residual(box, coef, u, u, DT)
    assert np.abs(F * elder.row_scale(box, DT)).max() < 1e-11
    u1 = newton.newton_solve(box, coef, u, DT)
    assert np.abs(u1[..., 1]).max() < 1e-13
    assert np.abs(u1[..., 0] - u[..., 0]).max() < 1e-9 * ph["rho0"] * ph["g"] * ph["lz"]


def _stratified_hydrostatic(box, ph, cz):
    """c = c(z) laterally uniform, p from the trapezoid rule of dp/dz = rho(c) g down each
    column (p = 0 at the top)."""
    rho = ph["rho0"] + (ph["rho1"] - ph["rho0"]) * np.asarray(cz)
    p = np.concatenate([[0.0], np.cumsum(ph["g"] * box.h[2] * 0.5 * (rho[1:] + rho[:-1]))])
    u = np.zeros((box.nz, box.ny, box.nx, 2))
    u[..., 0] = p[:, None, None]
    u[..., 1] = np.asarray(cz)[:, None, None]
    return u


@pytest.mark.parametrize("model", [0, 2, 3])
def test_stratified_hydrostatic_state_has_no_darcy_flux(model):
    """Consistent velocity (Section 4, the flux that keeps hydrostatic states free of
    spurious flow): with a non-uniform, non-monotone stratification c(z) and the discrete
    hydrostatic pressure, every face's Darcy flux vanishes for any per-hex K, so the
    liquid rows are zero and the salt rows are pure vertical diffusion (the same rows as
    with the permeability switched off)."""
    ph = synth.physics(model)
    box = elder.Box(9, 7, 6, ph)
    coef = elder.coefficients(box, [0.7, -0.4, 0.9, -1.0][:synth.N_XI[model]])
    u = _stratified_hydrostatic(box, ph, [0.0, 0.3, 0.35, 0.9, 0.1, 0.6])
    qscale = coef[1].max() / ph["mu"] * ph["rho1"] * ph["g"] * box.h[0] * box.h[1]
    for face in elder.SCVFS:
        Q = elder._face_quantities(box, coef, u[..., 0], u[..., 1], face)[3]
        assert np.abs(Q).max() < 1e-13 * qscale
    Fl, Fs = elder.fv_rows(box, coef, u, u, DT)
    Fl0, Fs0 = elder.fv_rows(box, (coef[0], coef[1] * 0.0), u, u, DT)
    s = elder.row_scale(box, DT)[..., 0]
    assert np.abs(Fl * s).max() < 1e-12
    assert np.abs(Fl0 * s).max() == 0.0
    assert np.abs((Fs - Fs0) * s).max() < 1e-12 * np.abs(Fs0 * s).max()
    assert np.abs(Fs0 * s).max() > 1e-6  # diffusion across the stratification is there
    # a lateral density contrast is not in equilibrium: flux appears
    u2 = u.copy()
    u2[:, :, : box.nx // 2, 1] += 0.2
    Q2 = max(np.abs(elder._face_quantities(box, coef, u2[..., 0], u2[..., 1], f)[3]).max()
             for f in elder.SCVFS)
    assert Q2 > 1e-3 * qscale


@pytest.mark.parametrize("c0", [0.0, 0.37, 1.0])
def test_uniform_salt_is_consistent(c0):
    """c = c0 everywhere, p = rho(c0) g z: both FV rows vanish at every vertex, i.e.
    the salt flux is c0 times the liquid flux and gravity balances the pressure."""
    ph = synth.physics(2)
    box = elder.Box(9, 7, 5, ph)
    coef = elder.coefficients(box, [0.5, 0.5, -0.5, 1.0])
    rho = ph["rho0"] + (ph["rho1"] - ph["rho0"]) * c0
    u = np.zeros((5, 7, 9, 2))
    u[..., 0] = rho * ph["g"] * box.z
    u[..., 1] = c0
    Fl, Fs = elder.fv_rows(box, coef, u, u, DT)
    s = elder.row_scale(box, DT)[..., 0]
    assert np.abs(Fl * s).max() < 1e-11
    assert np.abs(Fs * s).max() < 1e-11


def _thomas(a, b, c, d):
    """Textbook tridiagonal (Thomas) solve: a sub-, b main, c super-diagonal."""
    n = len(b)
    cp, dp = np.zeros(n), np.zeros(n)
    cp[0], dp[0] = c[0] / b[0], d[0] / b[0]
    for i in range(1, n):
        m = b[i] - a[i] * cp[i - 1]
        cp[i] = c[i] / m if i < n - 1 else 0.0
        dp[i] = (d[i] - a[i] * dp[i - 1]) / m
    x = np.zeros(n)
    x[-1] = dp[-1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


def _heat_1d(nz, H, D, dt, n_steps):
    """Implicit-Euler 3-point scheme (hz/dt)(c_k - c_k^old) = D (c_{k+1} - 2c_k + c_{k-1})/hz,
    c_0 = 1, c_{nz-1} = 0, c = 0 initially inside."""
    hz = H / (nz - 1)
    c = np.zeros(nz)
    c[0] = 1.0
    r = D * dt / hz ** 2
    n = nz - 2
    for _ in range(n_steps):
        rhs = c[1:-1].copy()
        rhs[0] += r * 1.0
        c[1:-1] = _thomas(np.full(n, -r), np.full(n, 1 + 2 * r), np.full(n, -r), rhs)
    return c


def test_thomas_heat_matches_fourier_series():
    """The 1D reference converges to c = 1 - z/H - sum 2/(n pi) sin(n pi z/H) e^{-D n^2 pi^2 t/H^2}
    at first order in dt (h^2 is negligible here)."""
    H, D, T = 150.0, 1e-4, 4.0e7
    z = np.linspace(0.0, H, 201)
    exact = 1.0 - z / H
    for n in range(1, 400):
        exact -= 2.0 / (n * np.pi) * np.sin(n * np.pi * z / H) * np.exp(-D * n * n * np.pi ** 2 * T / H ** 2)
    errs = []
    for steps in (100, 200, 400):
        c = _heat_1d(201, H, D, T / steps, steps)
        errs.append(np.abs(c - exact).max())
    assert errs[2] < 2e-3
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3


@pytest.mark.parametrize("shape", [(5, 5, 9), (7, 5, 17)])
def test_pure_diffusion_reduces_to_1d_scheme(shape):
    """g = 0, rho1 = rho0, uniform phi, c = 1 on the whole top: the 3D solution is
    independent of x, y and equals the 1D implicit-Euler three-point scheme."""
    nx, ny, nz = shape
    D, dt, steps = 1e-4, 2.0e6, 4
    ph = synth.physics(0, g=0.0, rho1=1000.0, Dm=D, patch=(0.0, 600.0, 0.0, 600.0))
    box = elder.Box(nx, ny, nz, ph)
    coef = elder.coefficients(box, [])
    u = np.zeros((nz, ny, nx, 2))
    u[0, :, :, 1] = 1.0
    for _ in range(steps):
        u = newton.newton_solve(box, coef, u, dt)
    ref = _heat_1d(nz, ph["lz"], D, dt, steps)
    assert np.abs(u[..., 1] - ref[:, None, None]).max() < 1e-12
    assert np.abs(u[..., 0]).max() < 1e-6


# ------------------------------------------------------- conservation ------

@pytest.mark.parametrize("model", [0, 2])
def test_global_mass_balance(model):
    """Interior face fluxes cancel and boundary faces carry none, so the change of
    total salt (liquid) mass over a step equals dt times the FV rows summed over the
    salt-Dirichlet (pressure-pinned) vertices, whose rows are not solved."""
    ph = synth.physics(model)
    nx, ny, nz = 9, 9, 5
    box = elder.Box(nx, ny, nz, ph)
    coef = elder.coefficients(box, [0.4, -0.9, 0.3, 0.8][:synth.N_XI[model]])
    u0 = synth.initial_state(nx, ny, nz, ph)
    u1 = newton.newton_solve(box, coef, u0, DT)
    u2 = newton.newton_solve(box, coef, u1, DT)
    Fl, Fs = elder.fv_rows(box, coef, u2, u1, DT)
    m = elder.storage_weight(box, coef[0])
    rho = lambda c: ph["rho0"] + (ph["rho1"] - ph["rho0"]) * c
    c1, c2 = u1[..., 1], u2[..., 1]
    dsalt = np.sum(m * (rho(c2) * c2 - rho(c1) * c1))
    dliq = np.sum(m * (rho(c2) - rho(c1)))
    cmask, _ = box.dirichlet_c()
    pmask = box.pinned_p()
    assert dsalt > 0  # brine enters through the patch
    assert abs(DT * Fs[cmask].sum() - dsalt) <= 1e-9 * abs(dsalt)
    assert abs(DT * Fl[pmask].sum() - dliq) <= 1e-9 * abs(dliq)
    # the solved rows are zero
    s = elder.row_scale(box, DT)[..., 0]
    assert np.abs((Fs * s)[~cmask]).max() < 1e-11
    assert np.abs((Fl * s)[~pmask]).max() < 1e-11
    bal = elder.mass_balance(box, coef, u2, u1, DT)
    assert bal["salt"]["dM"] == pytest.approx(dsalt, rel=1e-14)
    assert bal["salt"]["err"] < 1e-9 and bal["liquid"]["err"] < 1e-9


def test_mass_balance_detects_a_planted_imbalance():
    """Adding salt by hand at one interior vertex with no Dirichlet vertex among its 27
    neighbours (so no Dirichlet row sees it) changes the storage by m_v [rho(c+d)(c+d) - rho(c) c] with
    m_v = phi hx hy hz (constant phi, all 8 octants) and leaves the boundary exchange
    alone, so dM - B of mass_balance grows by exactly that amount; the liquid balance
    grows by m_v (rho1 - rho0) d."""
    ph = synth.physics(0)
    nx, ny, nz = 9, 9, 7
    box = elder.Box(nx, ny, nz, ph)
    coef = elder.coefficients(box, [])
    u0 = synth.initial_state(nx, ny, nz, ph)
    u1 = newton.newton_solve(box, coef, u0, DT)
    base = elder.mass_balance(box, coef, u1, u0, DT)
    k, j, i, d = 3, 1, 4, 0.05   # no Dirichlet vertex among its 27 neighbours (checked)
    cmask, _ = box.dirichlet_c()
    near = cmask[max(k - 1, 0):k + 2, max(j - 1, 0):j + 2, max(i - 1, 0):i + 2]
    assert not near.any() and not box.pinned_p()[k, j, i]
    u2 = u1.copy()
    u2[k, j, i, 1] += d
    bal = elder.mass_balance(box, coef, u2, u0, DT)
    m = ph["phi_mean"] * np.prod(box.h)
    rho = lambda c: ph["rho0"] + (ph["rho1"] - ph["rho0"]) * c
    c = u1[k, j, i, 1]
    planted = m * (rho(c + d) * (c + d) - rho(c) * c)
    for eq, amount in (("salt", planted), ("liquid", m * (ph["rho1"] - ph["rho0"]) * d)):
        got = (bal[eq]["dM"] - bal[eq]["B"]) - (base[eq]["dM"] - base[eq]["B"])
        assert got == pytest.approx(amount, rel=1e-9), eq
        assert bal[eq]["err"] > 1e3 * base[eq]["err"]


# ------------------------------------------------------------- symmetry ----

def test_box_symmetry_at_mean_parameters():
    """At xi = 0 the box, the patch and the boundary data are invariant under
    x -> 600 - x, y -> 600 - y and x <-> y; so is the solution after two steps."""
    ph = synth.physics(0)
    n = 9
    box = elder.Box(n, n, 5, ph)
    coef = elder.coefficients(box, [])
    u = synth.initial_state(n, n, 5, ph)
    for _ in range(2):
        u = newton.newton_solve(box, coef, u, DT)
    scale = np.array([ph["rho0"] * ph["g"] * ph["lz"], 1.0])
    v = u / scale
    assert np.abs(v - v[:, :, ::-1]).max() < 1e-10
    assert np.abs(v - v[:, ::-1, :]).max() < 1e-10
    assert np.abs(v - v.transpose(0, 2, 1, 3)).max() < 1e-10
    assert u[..., 1].max() > 0.0 and np.abs(u[1, :, :, 1]).max() > 1e-3  # not trivial


def test_cosine_field_symmetry():
    """The one-mode field phi = 0.1(1 + 0.2 xi cos(pi x/600) cos(pi y/600)) is invariant
    under the half-turn (x, y) -> (600 - x, 600 - y) and under x <-> y."""
    ph = synth.physics(1)
    n = 9
    box = elder.Box(n, n, 5, ph)
    coef = elder.coefficients(box, [0.8])
    assert np.abs(coef[0] - coef[0][:, ::-1, ::-1]).max() < 1e-15
    u = synth.initial_state(n, n, 5, ph)
    for _ in range(2):
        u = newton.newton_solve(box, coef, u, DT)
    v = u / np.array([ph["rho0"] * ph["g"] * ph["lz"], 1.0])
    assert np.abs(v - v[:, ::-1, ::-1]).max() < 1e-10
    assert np.abs(v - v.transpose(0, 2, 1, 3)).max() < 1e-10
    assert np.abs(v - v[:, :, ::-1]).max() > 1e-8  # the field breaks the single mirror


# ------------------------------------------------------ linear algebra -----

@pytest.mark.parametrize("shape", [(5, 5, 2), (5, 5, 3), (9, 9, 3)])
def test_dense_and_sparse_newton_agree(shape):
    """Newton with numpy.linalg.solve equals Newton with the sparse LU."""
    ph = synth.physics(2)
    nx, ny, nz = shape
    box = elder.Box(nx, ny, nz, ph)
    coef = elder.coefficients(box, [0.2, 0.6, -0.3, 0.9])
    u0 = synth.initial_state(nx, ny, nz, ph)
    a = newton.newton_solve(box, coef, u0, DT, dense=True)
    b = newton.newton_solve(box, coef, u0, DT)
    sc = np.array([ph["rho0"] * ph["g"] * ph["lz"], 1.0])
    assert np.abs((a - b) / sc).max() < 1e-12


def test_root_does_not_depend_on_start():
    """The step's root near u^{n-1} is reached from different starting guesses."""
    ph = synth.physics(2)
    box = elder.Box(9, 9, 3, ph)
    coef = elder.coefficients(box, [0.2, 0.6, -0.3, 0.9])
    u0 = synth.initial_state(9, 9, 3, ph)
    a = newton.newton_solve(box, coef, u0, DT)
    start = u0.copy()
    start[..., 0] += 500.0 * np.random.default_rng(1).standard_normal(start.shape[:3])
    b = newton.newton_solve(box, coef, u0, DT, u0=start)
    sc = np.array([ph["rho0"] * ph["g"] * ph["lz"], 1.0])
    assert np.abs((a - b) / sc).max() < 1e-11


# ---------------------------------------------------- upwinding ------------

def _elder_extremes(nx, ny, nz, dt, steps):
    ph = synth.physics(0)
    box = elder.Box(nx, ny, nz, ph)
    coef = elder.coefficients(box, [])
    u = synth.initial_state(nx, ny, nz, ph)
    for _ in range(steps):
        u = newton.newton_solve(box, coef, u, dt, max_it=60)
    return u[..., 1].min(), u[..., 1].max()


def test_upwinding_keeps_salt_in_range():
    """Implicit Euler with full upwinding keeps 0 <= c <= 1 (discrete maximum
    principle), here over three 3-month steps."""
    lo, hi = _elder_extremes(17, 17, 5, 3 * DT, 3)
    assert lo > -1e-9 and hi < 1.0 + 1e-9


def test_downwinding_would_violate_range(monkeypatch):
    """Sensitivity of the previous pin: swapping upstream and downstream vertices
    breaks the range after one 1-month step, so that pin detects the direction of
    upwinding."""
    monkeypatch.setattr(elder, "upwind_is_start", lambda Q: np.real(Q) < 0.0)
    lo, hi = _elder_extremes(17, 17, 5, DT, 1)
    assert lo < -1e-2 or hi > 1.0 + 1e-2


# --------------------------------------------------------------- stats -----

def test_moments_reduce_to_numpy():
    """Equal weights: mean and population variance are numpy's mean and var, the
    exceedance probability is the fraction of samples strictly above the threshold."""
    rng = np.random.default_rng(5)
    f = rng.random((37, 4, 5, 6))
    f[3, 0, 0, 0] = 0.5  # a tie at the threshold counts as not exceeding
    mean, var, exc = stats.moments(f, threshold=0.5)
    assert np.allclose(mean, f.mean(0), rtol=1e-14, atol=0)
    assert np.allclose(var, f.var(0), rtol=1e-12, atol=1e-16)
    assert np.array_equal(np.round(exc * 37), (f > 0.5).sum(0))
    assert exc[0, 0, 0] == pytest.approx(np.sum(np.delete(f[:, 0, 0, 0], 3) > 0.5) / 37, rel=1e-14)
    w = rng.random(37)
    w /= w.sum()
    mean_w, var_w, _ = stats.moments(f, weights=w)
    assert np.allclose(mean_w, np.average(f, axis=0, weights=w), rtol=1e-13)
    assert np.allclose(var_w, np.average((f - mean_w) ** 2, axis=0, weights=w), rtol=1e-12)


def test_injection_picks_nested_vertices():
    f = np.arange(17 * 65 * 65, dtype=float).reshape(17, 65, 65)
    g = stats.inject(f, (33, 33, 9))
    assert g.shape == (9, 33, 33)
    assert g[1, 2, 3] == f[2, 4, 6]


# ------------------------------------------------------------- gradient ----

def test_qoi_weights_are_exact_volumes():
    """With phi = 1 the octant weights integrate the box S exactly: sum W = |S|,
    also when S cuts hexahedra (200/75 and 100/37.5 are not integers)."""
    from oracle import gradient
    ph = synth.physics(0, phi_mean=0.5)
    box = elder.Box(9, 9, 5, ph)
    ones = np.ones((4, 8, 8))
    W = gradient.octant_weights(box, ones)
    assert W.sum() == pytest.approx(200 * 200 * 50, rel=1e-14)
    S = (0.0, 600.0, 0.0, 600.0, 0.0, 150.0)
    assert gradient.octant_weights(box, ones, S).sum() == pytest.approx(600 * 600 * 150, rel=1e-14)
    # uniform c: J = phi rho(c0) c0 |S|
    u = np.zeros((5, 9, 9, 2))
    u[..., 1] = 0.3
    coef = elder.coefficients(box, [])
    rho = ph["rho0"] + (ph["rho1"] - ph["rho0"]) * 0.3
    assert gradient.qoi(box, coef, u) == pytest.approx(0.5 * rho * 0.3 * 200 * 200 * 50, rel=1e-13)


@pytest.mark.parametrize("model,xi", [(1, [0.7]), (2, [0.3, -0.5, 0.2, 0.6]), (3, [0.6, -0.4, 0.9])])
def test_tangent_linear_gradient_matches_finite_differences(model, xi):
    """dJ/dxi from tangent-linear sensitivities equals central differences of the
    forward map (h = 1e-6), over three steps of a 9x9x5 box, for the one-mode, the
    four-mode and the paper's three-variable field."""
    from oracle import gradient
    ph = synth.physics(model)
    box = elder.Box(9, 9, 5, ph)
    S = (200.0, 400.0, 200.0, 400.0, 0.0, 60.0)
    xi = np.array(xi)
    u0 = synth.initial_state(9, 9, 5, ph)
    dts = [DT, DT, DT]
    J, g, _ = gradient.tangent_linear_gradient(box, xi, u0, dts, S)
    assert J > 0
    h = 1e-6
    for m in range(xi.size):
        e = np.zeros(xi.size)
        e[m] = h
        Jp = gradient.qoi(box, elder.coefficients(box, xi + e),
                          gradient.forward(box, xi + e, u0, dts)[-1], S)
        Jm = gradient.qoi(box, elder.coefficients(box, xi - e),
                          gradient.forward(box, xi - e, u0, dts)[-1], S)
        fd = (Jp - Jm) / (2 * h)
        assert abs(g[m] - fd) <= 1e-5 * np.abs(g).max(), (m, g[m], fd)


# ---------------------------------------------------- manufactured solution -----

def _mms_fields(ph, x, y, z, P=1.0e4):
    """A smooth manufactured state: p = rho0 g z + P cos cos cos, c = 0.5 + 0.3 sin sin
    cos (values in [0.2, 0.8]), with their exact gradients."""
    lx, ly, lz = ph["lx"], ph["ly"], ph["lz"]
    sx, cx = np.sin(np.pi * x / lx), np.cos(np.pi * x / lx)
    sy, cy = np.sin(np.pi * y / ly), np.cos(np.pi * y / ly)
    sz, cz = np.sin(np.pi * z / lz), np.cos(np.pi * z / lz)
    p = ph["rho0"] * ph["g"] * z + P * cx * cy * cz
    dp = (-P * np.pi / lx * sx * cy * cz, -P * np.pi / ly * cx * sy * cz,
          ph["rho0"] * ph["g"] - P * np.pi / lz * cx * cy * sz)
    c = 0.5 + 0.3 * sx * sy * cz
    dc = (0.3 * np.pi / lx * cx * sy * cz, 0.3 * np.pi / ly * sx * cy * cz,
          -0.3 * np.pi / lz * sx * sy * sz)
    return p, dp, c, dc


def _mms_exact_fluxes(ph, x, y, z):
    """The continuous liquid and salt flux vectors of Section 2.1 (eqs. e_cont_eq,
    e_tran_eq, e_Darcy_vel) at points, for constant phi and K."""
    _, dp, c, dc = _mms_fields(ph, x, y, z)
    rho = ph["rho0"] + (ph["rho1"] - ph["rho0"]) * c
    kmu = ph["K_mean"] / ph["mu"]
    q = (-kmu * dp[0], -kmu * dp[1], -kmu * (dp[2] - rho * ph["g"]))
    Fl = [rho * qd for qd in q]
    Fs = [rho * c * qd - rho * ph["phi_mean"] * ph["Dm"] * dcd for qd, dcd in zip(q, dc)]
    return Fl, Fs


def _mms_truncation(ph, n):
    """Finite-volume flux sums of the manufactured state minus the exact outward fluxes
    through the dual cells of the interior vertices (4x4 Gauss-Legendre per face),
    divided by the cell volume: the consistency error density of both rows."""
    nz = (n - 1) // 4 + 1
    box = elder.Box(n, n, nz, ph)
    coef = elder.coefficients(box, np.zeros(0))
    p, _, c, _ = _mms_fields(ph, box.x, box.y, box.z)
    u = np.stack([p, c], axis=-1)
    Fl, Fs = elder.fv_rows(box, coef, u, u, 1.0)  # u_old = u: no storage term
    sl = (slice(1, -1),) * 3
    ctr = [box.x[sl], box.y[sl], box.z[sl]]
    gx, gw = np.polynomial.legendre.leggauss(4)
    el, es = np.zeros_like(ctr[0]), np.zeros_like(ctr[0])
    for d in range(3):
        o = [e for e in range(3) if e != d]
        for sgn in (1.0, -1.0):
            for a, wa in zip(gx, gw):
                for b, wb in zip(gx, gw):
                    pt = list(ctr)
                    pt[d] = pt[d] + sgn * box.h[d] / 2
                    pt[o[0]] = pt[o[0]] + a * box.h[o[0]] / 2
                    pt[o[1]] = pt[o[1]] + b * box.h[o[1]] / 2
                    fl, fs = _mms_exact_fluxes(ph, *pt)
                    w = sgn * wa * wb * box.h[o[0]] * box.h[o[1]] / 4
                    el += w * fl[d]
                    es += w * fs[d]
    V = np.prod(box.h)
    return (Fl[sl] - el) / V, (Fs[sl] - es) / V


def test_manufactured_solution_consistency_orders():
    """Consistency of the discrete fluxes with the PDE under refinement (h = 37.5,
    18.75, 9.375 m): the liquid row (central, trilinear gradients at the face points)
    is second order, the salt row first order (full upwinding of the advected salt),
    and its diffusion part alone second order.  A dropped or mis-scaled flux term
    leaves an O(1) error and an order near zero."""
    ph = synth.physics(0)
    diff_only = dict(ph, K_mean=1e-30)
    el, es, ed = [], [], []
    for n in (17, 33, 65):
        tl, ts = _mms_truncation(ph, n)
        _, td = _mms_truncation(diff_only, n)
        el.append(np.abs(tl).max())
        es.append(np.sqrt(np.mean(ts ** 2)))
        ed.append(np.sqrt(np.mean(td ** 2)))
    order = lambda e: math.log2(e[-2] / e[-1])
    print("liquid", el, order(el), "salt", es, order(es), "salt diffusion", ed, order(ed))
    assert order(el) > 1.8
    assert order(es) > 0.9
    assert order(ed) > 1.8
    assert el[-1] < 0.05 * 7e-6 and es[-1] < 0.05 * 8e-6  # small against the flux divergence


# ---------------------------------------------------------- polynomial chaos -----

def test_legendre_matches_the_printed_polynomials():
    """psi_0..psi_5 of the recursion equal the appendix's list (psi_3 as the recursion
    gives it; the printed psi_3 is not a Legendre polynomial: it fails orthogonality)."""
    from oracle import gpc
    g = _load("legendre.json")
    x = np.linspace(-1.0, 1.0, 41)
    for n, c in g["psi"].items():
        ref = np.polynomial.polynomial.polyval(x, c)
        assert np.abs(gpc.legendre(int(n), x) - ref).max() < 1e-14
    printed = np.polynomial.polynomial.polyval(x, g["psi3_as_printed"])
    xq, wq = np.polynomial.legendre.leggauss(8)
    pr = np.polynomial.polynomial.polyval(xq, g["psi3_as_printed"])
    assert abs(np.sum(wq * pr * gpc.legendre(1, xq))) > 0.1   # printed form is not orthogonal
    assert np.abs(printed - gpc.legendre(3, x)).max() > 0.1


def test_legendre_orthogonality_and_norms():
    """<psi_m, psi_n> = delta_mn / (2n + 1) under the uniform density, with a
    Gauss-Legendre rule exact for degree <= 11."""
    from oracle import gpc
    nodes, w = gpc.tensor_gauss_legendre(1, 6)
    x = nodes[:, 0]
    assert abs(w.sum() - 1.0) < 1e-15
    for m in range(6):
        for n in range(6):
            got = np.sum(w * gpc.legendre(m, x) * gpc.legendre(n, x))
            assert abs(got - (1.0 / (2 * n + 1) if m == n else 0.0)) < 1e-14


def test_multi_index_sets():
    from oracle import gpc
    assert len(gpc.multi_indices(3, 4)) == math.comb(7, 4) == 35
    assert len(gpc.multi_indices(4, 4)) == math.comb(8, 4)
    assert len(gpc.multi_indices(3, 2, truncation=1)) == 27
    assert gpc.multi_indices(2, 2) == [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]
    J = gpc.multi_indices(3, 3, truncation=1)
    assert len(set(J)) == len(J) and max(max(b) for b in J) == 3
    assert [sum(b) for b in J] == sorted(sum(b) for b in J)


def test_projection_recovers_a_polynomial_field():
    """Fields that are gPC polynomials of degree <= p are projected back to their own
    coefficients by a tensor Gauss-Legendre rule with p + 1 points per direction."""
    from oracle import gpc
    rng = np.random.default_rng(7)
    for M, p, trunc in ((3, 4, 0), (2, 3, 1), (1, 5, 0)):
        J = gpc.multi_indices(M, p, trunc)
        true = rng.standard_normal((len(J), 5, 4))
        nodes, w = gpc.tensor_gauss_legendre(M, p + 1)
        fields = gpc.surrogate(true, J, nodes)
        got = gpc.project(fields, nodes, w, J)
        assert np.abs(got - true).max() < 1e-12


def test_gpc_moments_closed_form():
    """f = a + b th1 + c th1 th2 + d psi_2(th3): mean a, variance b^2/3 + c^2/9 + d^2/5,
    from the coefficients (eqs. PCEcoef2, var) and equal to the quadrature moments."""
    from oracle import gpc
    a, b, c, d = 0.4, -0.3, 0.7, 0.2
    J = gpc.multi_indices(3, 2)
    nodes, w = gpc.tensor_gauss_legendre(3, 3)
    t = nodes
    f = a + b * t[:, 0] + c * t[:, 0] * t[:, 1] + d * gpc.legendre(2, t[:, 2])
    coef = gpc.project(f[:, None], nodes, w, J)
    mean, var = gpc.moments(coef, J)
    assert abs(mean[0] - a) < 1e-15
    assert abs(var[0] - (b * b / 3 + c * c / 9 + d * d / 5)) < 1e-15
    m2, v2, _ = stats.moments(f[:, None], w)
    assert abs(m2[0] - a) < 1e-15 and abs(v2[0] - var[0]) < 1e-15


def test_surrogate_exceedance():
    """For c = th1, P(c > t) = (1 - t)/2: the sampled estimate (Section 3.2) lies within
    four standard errors, and equals a direct count."""
    from oracle import gpc
    J = gpc.multi_indices(2, 1)
    coef = np.zeros((len(J), 3))
    coef[1] = 1.0                                   # beta = (1, 0): psi_1(th1) = th1
    pts = np.random.default_rng(3).uniform(-1, 1, (200000, 2))
    t = np.array([-0.5, 0.1, 0.8])
    got = np.array([gpc.exceedance(coef[:, q:q + 1], J, pts, t[q])[0] for q in range(3)])
    ref = (1.0 - t) / 2.0
    se = np.sqrt(ref * (1 - ref) / len(pts))
    assert np.all(np.abs(got - ref) < 4 * se)
    assert np.array_equal(got, np.array([np.mean(pts[:, 0] > tq) for tq in t]))
