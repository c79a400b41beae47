"""Salt mass in a subregion and its gradient with respect to the field parameters xi.

TEST INFRASTRUCTURE ONLY (oracle).

Quantity of interest: the salt mass in a box S at the final time, with the
lumped (vertex control volume) representation of the FV scheme,
    J = sum_v sum_{e ∋ v} phi_e |o(e, v) ∩ S| rho(c_v) c_v,
where o(e, v) is the octant of hexahedron e that belongs to vertex v (the mass
density phi rho c of Section 2.1, eq. e_tran_eq, integrated over S).  The reading
for the "lower-central subregion" of the workload is S = [200,400] x [200,400] x
[100,150] (depth), the bottom 50 m under the centre of the box.

Gradient: tangent-linear sensitivities.  Each implicit-Euler step solves
R(u^n; u^{n-1}, xi) = 0, so du^n/dxi = -(dR/du^n)^{-1} (dR/du^{n-1} du^{n-1}/dxi
+ dR/dxi), and dJ/dxi = dJ/du^N du^N/dxi + dJ/dxi|_explicit.  dR/dxi and the
explicit dJ/dxi come from complex-step differentiation through the coefficient
fields (phi, K are analytic in xi), dR/du^{n-1} times a direction from complex
step in u^{n-1}.  This is a different mode from the library's adjoint (reverse),
so the two are independent checks of each other.
"""
from __future__ import annotations

import numpy as np

from . import elder, newton

LOWER_CENTRAL = (200.0, 400.0, 200.0, 400.0, 100.0, 150.0)


def _overlap(lo, hi, s0, s1):
    return np.maximum(0.0, np.minimum(hi, s1) - np.maximum(lo, s0))


def octant_weights(box: elder.Box, phi_e, S=LOWER_CENTRAL):
    """W_v = sum over adjacent hexes of phi_e |o(e, v) ∩ S|, shape [nz, ny, nx]."""
    hx, hy, hz = box.h
    W = np.zeros((box.nz, box.ny, box.nx), dtype=np.result_type(phi_e, float))
    xv, yv, zv = box.xc - hx / 2, box.yc - hy / 2, box.zc - hz / 2  # hex lower corners
    for a, b, c in elder.CORNERS:
        # octant of corner (a, b, c): the half of the hex next to that corner in each direction
        x0 = xv + a * hx / 2
        y0 = yv + b * hy / 2
        z0 = zv + c * hz / 2
        vol = (_overlap(x0, x0 + hx / 2, S[0], S[1]) * _overlap(y0, y0 + hy / 2, S[2], S[3])
               * _overlap(z0, z0 + hz / 2, S[4], S[5]))
        box.corner(W, (a, b, c))[...] += phi_e * vol
    return W


def qoi(box: elder.Box, coef, u, S=LOWER_CENTRAL):
    ph = box.phys
    c = u[..., 1]
    rho = ph["rho0"] + (ph["rho1"] - ph["rho0"]) * c
    return np.sum(octant_weights(box, coef[0], S) * rho * c)


def _coef_cs(box, xi, m, h):
    """Coefficients at xi + i h e_m (complex step)."""
    x = np.asarray(xi, dtype=complex).copy()
    x[m] += 1j * h
    return _coefficients_complex(box, x)


def _coefficients_complex(box, xi):
    # elder.coefficients with complex parameters: the formulas are analytic in xi
    ph = box.phys
    model = ph["field_model"]
    x, y, z = box.xc, box.yc, box.zc
    lx, ly, lz = ph["lx"], ph["ly"], ph["lz"]
    pm = ph["phi_mean"]
    if model == 1:
        phi = pm * (1.0 + 0.2 * xi[0] * np.cos(np.pi * x / lx) * np.cos(np.pi * y / ly))
        K = elder.kozeny_carman(phi, ph)
    elif model == 2:
        phi = pm * (1.0 + 0.2 * xi[0] * np.cos(np.pi * x / lx) * np.cos(np.pi * y / ly)
                    + 0.2 * xi[1] * np.sin(np.pi * x / lx) * np.sin(np.pi * y / ly))
        K = np.exp(np.log(elder.kozeny_carman(phi, ph)) + 0.5 * xi[2] * np.cos(np.pi * z / lz)
                   + 0.5 * xi[3] * np.sin(np.pi * x / lx) * np.cos(np.pi * z / lz))
    elif model == 3:
        sx, sy, sz = np.sin(np.pi * x / lx), np.sin(np.pi * y / ly), np.sin(np.pi * z / lz)
        phi = pm + 0.01 * (xi[0] * sx + xi[1] * sy + xi[2] * sz + xi[0] * sx * sy + xi[1] * sx * sz)
        K = elder.kozeny_carman(phi, ph)
    else:
        raise ValueError("the constant field has no parameters")
    return phi, K


def forward(box, xi, u0, dts, rtol=1e-13):
    """States after each step of length dts[n] (list), starting from u0."""
    coef = elder.coefficients(box, xi)
    states = [u0]
    for dt in dts:
        states.append(newton.newton_solve(box, coef, states[-1], dt, rtol=rtol))
    return states


def tangent_linear_gradient(box, xi, u0, dts, S=LOWER_CENTRAL, rtol=1e-13, h=1e-30):
    """(J, dJ/dxi) by tangent-linear sensitivities along the trajectory from u0."""
    xi = np.asarray(xi, dtype=float)
    M = xi.size
    coef = elder.coefficients(box, xi)
    rs = elder.row_scale
    states = forward(box, xi, u0, dts, rtol)
    du = [np.zeros(u0.shape) for _ in range(M)]
    perm = newton.nested_dissection(box.nx, box.ny, box.nz)
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    for n, dt in enumerate(dts):
        u_old, u_new = states[n], states[n + 1]
        J = elder.jacobian(box, coef, u_new, dt).tocsr()
        lu = spla.splu(J[perm][:, perm].tocsc())
        for m in range(M):
            dR_dxi = elder.residual(box, _coef_cs(box, xi, m, h), u_new, u_old, dt).imag / h
            dR_dold = elder.residual(box, coef, u_new, u_old + 1j * h * du[m], dt).imag / h
            rhs = -(dR_dxi + dR_dold).ravel()
            y = np.empty_like(rhs)
            y[perm] = lu.solve(rhs[perm])
            du[m] = y.reshape(u0.shape)
    uN = states[-1]
    Jval = qoi(box, coef, uN, S)
    ph = box.phys
    c = uN[..., 1]
    dJ_dc = octant_weights(box, coef[0], S) * (ph["rho0"] + 2.0 * (ph["rho1"] - ph["rho0"]) * c)
    grad = np.zeros(M)
    for m in range(M):
        explicit = qoi(box, _coef_cs(box, xi, m, h), uN, S).imag / h
        grad[m] = np.sum(dJ_dc * du[m][..., 1]) + explicit
    return Jval, grad, states
