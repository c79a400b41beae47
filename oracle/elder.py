"""Vertex-centred finite-volume discretisation of the Elder problem, plain FP64.

TEST INFRASTRUCTURE ONLY.  This is the oracle that the HIP path is checked
against; nothing in the product imports it.  It is written to be read against
the paper, not to be fast.

What it follows (paper, Section 2 "Problem setup"):
  * liquid mass conservation  d_t(phi rho) + div(rho q) = 0          (eq. e_cont_eq)
  * salt transport            d_t(phi rho c) + div(rho c q - rho D grad c) = 0  (eq. e_tran_eq)
  * Darcy's law               q = -(K/mu)(grad p - rho g)            (eq. e_Darcy_vel)
  * scalar permeability K I (eq. e_scalar_perm), linear density
    rho(c) = rho0 + (rho1 - rho0) c (eq. e_lin_density), D = phi D_m I (eq. e_mol_diff)
  * vertex-centred FV with DoFs (p, c) at the grid nodes, implicit Euler in time
    (Section 2.3 "Solution of the stochastic flow model").
  * Boundary conditions of the box (Section 2.1, text under Table 1): c = 1 on the
    top patch, c = 0 at the bottom, zero flux elsewhere, p fixed to 0 at the four
    top corners (the reading adopted for the "edges" sentence).

The paper gives no formula for the discrete operator; the readings used here are:
  R1  vertices x_ijk = (i hx, j hy, k hz); z is depth; gravity = (0, 0, +g).
  R2  phi, K constant per hexahedron, evaluated at its centroid.
  R3  control volume of a vertex = union of its hex octants; storage weight
      m_v = sum over adjacent hexes of phi_e * (hx hy hz / 8).
  R4  one sub-control-volume face (SCVF) per hex edge: the quarter of the hex
      mid-plane normal to the edge, area = (product of the two other h)/4, normal +e_d,
      one integration point at the face centre (t_d = 1/2, others at 1/4 or 3/4).
  R5  trilinear (Q1) interpolation of c and of grad p, grad c at the integration point.
  R6  Darcy flux through the face Q = -(K_e/mu)(d_d p - rho(c_f) g_d) A_f.
  R7  full upwinding of the advected salt: upstream vertex = edge start if Q >= 0.
  R8  liquid flux rho(c_f) Q;  salt flux rho(c_up) c_up Q - rho(c_f) phi_e D_m d_d c A_f.
  R9  residual row = storage m_v [..]^{n} - [..]^{n-1} over dt + outgoing fluxes.
  R10 Dirichlet rows: salt row -> c - c_D on the patch (c_D = 1) and bottom (c_D = 0);
      liquid row -> p at the four top corners.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

CORNERS = [(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]  # (x, y, z) bits


class Box:
    """Structured vertex grid on [0,lx] x [0,ly] x [0,lz]; arrays are indexed [k, j, i]."""

    def __init__(self, nx: int, ny: int, nz: int, phys: dict):
        if min(nx, ny, nz) < 2:
            raise ValueError("need at least two vertices per direction")
        self.nx, self.ny, self.nz = nx, ny, nz
        self.phys = phys
        self.h = (phys["lx"] / (nx - 1), phys["ly"] / (ny - 1), phys["lz"] / (nz - 1))
        self.N = nx * ny * nz
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        self.k, self.j, self.i = k, j, i
        self.x, self.y, self.z = i * self.h[0], j * self.h[1], k * self.h[2]
        # hex centroids, shape (nz-1, ny-1, nx-1)
        kc, jc, ic = np.meshgrid(np.arange(nz - 1), np.arange(ny - 1), np.arange(nx - 1),
                                 indexing="ij")
        self.xc = (ic + 0.5) * self.h[0]
        self.yc = (jc + 0.5) * self.h[1]
        self.zc = (kc + 0.5) * self.h[2]
        self.vid = np.arange(self.N).reshape(nz, ny, nx)

    @property
    def n_hex(self) -> int:
        return (self.nx - 1) * (self.ny - 1) * (self.nz - 1)

    def corner(self, arr, bits):
        """View of a vertex array at corner `bits` = (a, b, c) of every hexahedron."""
        a, b, c = bits
        return arr[c:c + self.nz - 1, b:b + self.ny - 1, a:a + self.nx - 1]

    # -- boundary sets (R10) ------------------------------------------------
    def dirichlet_c(self):
        """(mask, value) of the salt Dirichlet vertices: closed top patch c = 1, bottom c = 0."""
        x0, x1, y0, y1 = self.phys["patch"]
        tol = 1e-9 * max(self.phys["lx"], self.phys["ly"])
        patch = ((self.k == 0) & (self.x >= x0 - tol) & (self.x <= x1 + tol)
                 & (self.y >= y0 - tol) & (self.y <= y1 + tol))
        bottom = self.k == self.nz - 1
        mask = patch | bottom
        value = np.where(patch, 1.0, 0.0)
        return mask, value

    def pinned_p(self):
        """Mask of the vertices where p = 0: the four top corners."""
        return ((self.k == 0) & ((self.i == 0) | (self.i == self.nx - 1))
                & ((self.j == 0) | (self.j == self.ny - 1)))


# ---------------------------------------------------------------------------
# Porosity and permeability (Section 2.2, eq. e_perm_Kozeny_Carman; Section 5)
# ---------------------------------------------------------------------------

def kozeny_carman(phi, phys):
    """K(phi) = K_mean (phi/phi_mean)^3 ((1 - phi_mean)/(1 - phi))^2, so K(phi_mean) = K_mean.

    The Kozeny-Carman scaling constant is fixed by K(E phi) = E K (Section 2.2); the
    (1 - phi)^2 denominator is the standard Kozeny-Carman form (the paper prints 1 - phi^2).
    """
    pm = phys["phi_mean"]
    return phys["K_mean"] * (phi / pm) ** 3 * ((1.0 - pm) / (1.0 - phi)) ** 2


def coefficients(box: Box, xi) -> tuple:
    """Per-hex (phi_e, K_e) at the hex centroids for the field model in box.phys."""
    ph = box.phys
    model = ph["field_model"]
    xi = np.asarray(xi, dtype=float).ravel()
    x, y, z = box.xc, box.yc, box.zc
    lx, ly, lz = ph["lx"], ph["ly"], ph["lz"]
    pm = ph["phi_mean"]
    if model == 0:
        phi = np.full(x.shape, pm)
        K = np.full(x.shape, ph["K_mean"])
    elif model == 1:
        phi = pm * (1.0 + 0.2 * xi[0] * np.cos(np.pi * x / lx) * np.cos(np.pi * y / ly))
        K = kozeny_carman(phi, ph)
    elif model == 2:
        phi = pm * (1.0 + 0.2 * xi[0] * np.cos(np.pi * x / lx) * np.cos(np.pi * y / ly)
                    + 0.2 * xi[1] * np.sin(np.pi * x / lx) * np.sin(np.pi * y / ly))
        logK = (np.log(kozeny_carman(phi, ph)) + 0.5 * xi[2] * np.cos(np.pi * z / lz)
                + 0.5 * xi[3] * np.sin(np.pi * x / lx) * np.cos(np.pi * z / lz))
        K = np.exp(logK)
    elif model == 3:
        # the paper's three-variable porosity of the box experiment (eq. poro-paral3RVS)
        sx, sy, sz = np.sin(np.pi * x / lx), np.sin(np.pi * y / ly), np.sin(np.pi * z / lz)
        phi = pm + 0.01 * (xi[0] * sx + xi[1] * sy + xi[2] * sz + xi[0] * sx * sy + xi[1] * sx * sz)
        K = kozeny_carman(phi, ph)
    else:
        raise ValueError(f"unknown field model {model}")
    return phi, K


# ---------------------------------------------------------------------------
# Sub-control-volume faces (R4, R5)
# ---------------------------------------------------------------------------

def scvf_list():
    """The 12 SCVFs of a hexahedron: (d, edge_bits, weights) where for each corner w
    weights[w] = (N_w(ip), dN_w/dt_d(ip)) in reference coordinates t in [0,1]^3."""
    faces = []
    for d in range(3):
        others = [e for e in range(3) if e != d]
        for s0 in (0, 1):
            for s1 in (0, 1):
                ip = [0.0, 0.0, 0.0]
                ip[d] = 0.5
                ip[others[0]] = 0.25 if s0 == 0 else 0.75
                ip[others[1]] = 0.25 if s1 == 0 else 0.75
                start = [0, 0, 0]
                start[others[0]] = s0
                start[others[1]] = s1
                end = list(start)
                end[d] = 1
                w = {}
                for bits in CORNERS:
                    f = [ip[e] if bits[e] == 1 else 1.0 - ip[e] for e in range(3)]
                    N = f[0] * f[1] * f[2]
                    dfd = 1.0 if bits[d] == 1 else -1.0
                    dN = dfd * np.prod([f[e] for e in range(3) if e != d])
                    w[bits] = (N, dN)
                faces.append((d, tuple(start), tuple(end), w))
    return faces


SCVFS = scvf_list()


def _rho(c, ph):
    return ph["rho0"] + (ph["rho1"] - ph["rho0"]) * c


def storage_weight(box: Box, phi_e):
    """m_v = sum over the hexes adjacent to v of phi_e * V/8 (R3)."""
    Vo = box.h[0] * box.h[1] * box.h[2] / 8.0
    m = np.zeros((box.nz, box.ny, box.nx), dtype=np.result_type(phi_e, float))
    for bits in CORNERS:
        box.corner(m, bits)[...] += phi_e * Vo
    return m


def _face_quantities(box, coef, p, c, face):
    """Interpolated c, d_d p, d_d c, Darcy flux Q at one SCVF of every hex."""
    ph = box.phys
    phi_e, K_e = coef
    d, start, end, w = face
    h = box.h
    area = np.prod([h[e] for e in range(3) if e != d]) / 4.0
    cf = sum(N * box.corner(c, b) for b, (N, _) in w.items())
    dp = sum(dN * box.corner(p, b) for b, (_, dN) in w.items()) / h[d]
    dc = sum(dN * box.corner(c, b) for b, (_, dN) in w.items()) / h[d]
    gd = ph["g"] if d == 2 else 0.0
    Q = -(K_e / ph["mu"]) * (dp - _rho(cf, ph) * gd) * area
    return cf, dp, dc, Q, area, gd


def upwind_is_start(Q):
    """Full upwinding (R7): the upstream vertex is the edge start when Q >= 0."""
    return np.real(Q) >= 0.0


def fv_rows(box: Box, coef, u, u_old, dt):
    """Liquid and salt finite-volume rows (R9) at every vertex, before Dirichlet rows.

    u, u_old: [nz, ny, nx, 2] with (p, c).  Complex u is allowed (complex-step tests);
    the upwind choice uses the real part.  Returns (F_liquid, F_salt), each [nz, ny, nx].
    """
    ph = box.phys
    phi_e, K_e = coef
    p, c = u[..., 0], u[..., 1]
    c_old = u_old[..., 1]
    m = storage_weight(box, phi_e)
    Fl = m * (_rho(c, ph) - _rho(c_old, ph)) / dt
    Fs = m * (_rho(c, ph) * c - _rho(c_old, ph) * c_old) / dt
    Fl = Fl.astype(np.result_type(Fl, u))
    Fs = Fs.astype(np.result_type(Fs, u))
    for face in SCVFS:
        d, start, end, w = face
        cf, dp, dc, Q, area, gd = _face_quantities(box, coef, p, c, face)
        ca, cb = box.corner(c, start), box.corner(c, end)
        cup = np.where(upwind_is_start(Q), ca, cb)
        phi_l = _rho(cf, ph) * Q
        phi_s = _rho(cup, ph) * cup * Q - _rho(cf, ph) * phi_e * ph["Dm"] * dc * area
        box.corner(Fl, start)[...] += phi_l
        box.corner(Fl, end)[...] -= phi_l
        box.corner(Fs, start)[...] += phi_s
        box.corner(Fs, end)[...] -= phi_s
    return Fl, Fs


def residual(box: Box, coef, u, u_old, dt):
    """Full nonlinear residual F(u; u_old) [nz, ny, nx, 2] with Dirichlet rows (R10)."""
    Fl, Fs = fv_rows(box, coef, u, u_old, dt)
    cmask, cval = box.dirichlet_c()
    pmask = box.pinned_p()
    F = np.stack([Fl, Fs], axis=-1)
    F[..., 1] = np.where(cmask, u[..., 1] - cval, Fs)
    F[..., 0] = np.where(pmask, u[..., 0], Fl)
    return F


def jacobian(box: Box, coef, u, dt):
    """Analytic Jacobian dF/du (upwind choice frozen) as a CSR matrix of size 2N x 2N.

    Unknown ordering: index 2*v + var with var 0 = p, 1 = c and
    v = i + nx (j + ny k); row 2*v + eq with eq 0 = liquid, 1 = salt.
    """
    ph = box.phys
    phi_e, K_e = coef
    p, c = u[..., 0], u[..., 1]
    drho = ph["rho1"] - ph["rho0"]
    rows, cols, vals = [], [], []

    def add(row_v, eq, col_v, var, val):
        rows.append((2 * row_v + eq).ravel())
        cols.append((2 * col_v + var).ravel())
        vals.append(np.broadcast_to(val, row_v.shape).ravel())

    for face in SCVFS:
        d, start, end, w = face
        cf, dp, dc, Q, area, gd = _face_quantities(box, coef, p, c, face)
        rho_f = _rho(cf, ph)
        ca, cb = box.corner(c, start), box.corner(c, end)
        is_a = upwind_is_start(Q)
        cup = np.where(is_a, ca, cb)
        rho_up = _rho(cup, ph)
        va, vb = box.corner(box.vid, start), box.corner(box.vid, end)
        for bits, (N, dN) in w.items():
            vw = box.corner(box.vid, bits)
            dQ_dp = -(K_e / ph["mu"]) * area * dN / box.h[d]
            dQ_dc = (K_e / ph["mu"]) * area * drho * gd * N
            dl_dp = rho_f * dQ_dp
            dl_dc = drho * N * Q + rho_f * dQ_dc
            ds_dp = rho_up * cup * dQ_dp
            ds_dc = (rho_up * cup * dQ_dc
                     - drho * N * phi_e * ph["Dm"] * dc * area
                     - rho_f * phi_e * ph["Dm"] * area * dN / box.h[d])
            if bits == start:
                ds_dc = ds_dc + np.where(is_a, (ph["rho0"] + 2.0 * drho * cup) * Q, 0.0)
            if bits == end:
                ds_dc = ds_dc + np.where(is_a, 0.0, (ph["rho0"] + 2.0 * drho * cup) * Q)
            for sign, vr in ((1.0, va), (-1.0, vb)):
                add(vr, 0, vw, 0, sign * dl_dp)
                add(vr, 0, vw, 1, sign * dl_dc)
                add(vr, 1, vw, 0, sign * ds_dp)
                add(vr, 1, vw, 1, sign * ds_dc)
    m = storage_weight(box, phi_e)
    v = box.vid
    add(v, 0, v, 1, m * drho / dt)
    add(v, 1, v, 1, m * (ph["rho0"] + 2.0 * drho * c) / dt)
    n = 2 * box.N
    J = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    # Dirichlet rows become identity rows
    cmask, _ = box.dirichlet_c()
    pmask = box.pinned_p()
    drow = np.zeros(n, dtype=bool)
    drow[2 * box.vid[pmask]] = True
    drow[2 * box.vid[cmask] + 1] = True
    keep = sp.diags((~drow).astype(float))
    J = (keep @ J + sp.diags(drow.astype(float))).tocsr()
    J.eliminate_zeros()
    return J


# ---------------------------------------------------------------------------
# Global conservation of one step (eqs. e_cont_eq and e_tran_eq summed over the box)
# ---------------------------------------------------------------------------

def mass_balance(box: Box, coef, u, u_old, dt):
    """Salt and liquid mass balance of one implicit-Euler step from u_old to u.

    Summing the FV rows (R9) over all vertices, every interior SCVF flux appears once
    with each sign and no-flow faces carry none, so the storage change of the whole box
    equals dt times the rows of the vertices whose equation is a Dirichlet condition
    (the boundary exchange): salt rows at the c-Dirichlet vertices, liquid rows at the
    pinned vertices.  Returns, per equation, the storage change dM, the sum of the
    vertices' absolute storage changes, the exchange B and the relative error
    |dM - B| / (sum |storage change| + |B|) (0 when both vanish)."""
    ph = box.phys
    Fl, Fs = fv_rows(box, coef, u, u_old, dt)
    m = storage_weight(box, coef[0])
    c, co = u[..., 1], u_old[..., 1]
    Ss = m * (_rho(c, ph) * c - _rho(co, ph) * co)
    Sl = m * (_rho(c, ph) - _rho(co, ph))
    cmask, _ = box.dirichlet_c()
    pmask = box.pinned_p()
    out = {}
    for name, S, F, mask in (("salt", Ss, Fs, cmask), ("liquid", Sl, Fl, pmask)):
        dM, gross, B = float(S.sum()), float(np.abs(S).sum()), float(dt * F[mask].sum())
        den = gross + abs(B)
        out[name] = {"dM": dM, "gross": gross, "B": B,
                     "err": abs(dM - B) / den if den > 0 else 0.0}
    return out


# ---------------------------------------------------------------------------
# Scaling used for norms (a dimensionless "change of c per step" for FV rows)
# ---------------------------------------------------------------------------

def row_scale(box: Box, dt):
    """Per-row factors turning F into a dimensionless residual.

    FV rows: dt / (rho0 phi_mean hx hy hz); salt Dirichlet rows: 1;
    pinned pressure rows: 1 / pressure_unit.  Shape [nz, ny, nx, 2]."""
    ph = box.phys
    V = box.h[0] * box.h[1] * box.h[2]
    s = np.full((box.nz, box.ny, box.nx, 2), dt / (ph["rho0"] * ph["phi_mean"] * V))
    cmask, _ = box.dirichlet_c()
    s[..., 1] = np.where(cmask, 1.0, s[..., 1])
    s[..., 0] = np.where(box.pinned_p(), 1.0 / pressure_unit(ph), s[..., 0])
    return s


def pressure_unit(ph):
    """rho0 g lz (the hydrostatic pressure at the bottom); g is taken as at least 1 m/s^2
    so that the unit stays positive in the gravity-free test cases."""
    return ph["rho0"] * max(ph["g"], 1.0) * ph["lz"]


def col_scale(box: Box):
    """Unknown scaling: p in units of pressure_unit, c as is.  Shape [2]."""
    return np.array([pressure_unit(box.phys), 1.0])
