"""Implicit-Euler time step solved by Newton's method with a sparse direct solve.

TEST INFRASTRUCTURE ONLY (oracle).  Section 2.3 of the paper: every implicit
Euler step gives a nonlinear algebraic system, solved by Newton's method with a
line search.  The oracle only has to reach the root of F(u^n; u^{n-1}) = 0
near u^{n-1} tightly; it does so with an exact (SuperLU) solve of every Newton
system instead of the paper's preconditioned Krylov method.

Line search reading (the paper gives no rule): lambda = 1, 1/2, 1/4, ... (at most
`ls_max` halvings); the first lambda with ||F~(u + lambda d)|| <= (1 - lambda/4) ||F~(u)||
is taken, else the last one.  F~ is the residual scaled by `elder.row_scale`.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import elder


def nested_dissection(nx, ny, nz, leaf=32):
    """Geometric nested-dissection order of the unknowns of an nx*ny*nz vertex grid.

    Only a fill-reducing permutation for the sparse LU: the box is cut by a vertex
    plane through the middle of its longest side, both halves are ordered recursively
    and the plane goes last.  It does not change the solution of a linear system.
    """
    out = []

    def block(r):
        (i0, i1), (j0, j1), (k0, k1) = r
        k, j, i = np.meshgrid(np.arange(k0, k1), np.arange(j0, j1), np.arange(i0, i1),
                              indexing="ij")
        out.append((i + nx * (j + ny * k)).ravel())

    def rec(r):
        sizes = [hi - lo for lo, hi in r]
        if sizes[0] * sizes[1] * sizes[2] <= leaf or max(sizes) < 3:
            block(r)
            return
        d = int(np.argmax(sizes))
        lo, hi = r[d]
        mid = (lo + hi) // 2
        a, b, s = list(r), list(r), list(r)
        a[d], b[d], s[d] = (lo, mid), (mid + 1, hi), (mid, mid + 1)
        rec(a)
        rec(b)
        block(s)

    rec([(0, nx), (0, ny), (0, nz)])
    v = np.concatenate(out)
    return np.stack([2 * v, 2 * v + 1], axis=1).ravel()


def sparse_solve(A, rhs, perm):
    """x = A^{-1} rhs by SuperLU on the symmetrically permuted matrix."""
    Ap = A.tocsr()[perm][:, perm].tocsc()
    y = spla.splu(Ap, permc_spec="NATURAL").solve(rhs[perm])
    x = np.empty_like(y)
    x[perm] = y
    return x


def scaled_norm(box, F, dt):
    return float(np.linalg.norm((F * elder.row_scale(box, dt)).ravel()))


def newton_solve(box, coef, u_old, dt, u0=None, rtol=1e-13, atol=None, max_it=40,
                 ls_max=5, dense=False, stats=None):
    """Root of F(u; u_old) = 0 starting from u0 (default u_old).

    Stops when ||F~|| <= max(rtol ||F~(u0)||, atol) or when the scaled Newton update
    falls below 1e-15 in max norm.  `dense=True` uses numpy.linalg.solve (tiny grids).
    """
    n = 2 * box.N
    if atol is None:
        atol = 1e-15 * np.sqrt(n)
    rs = elder.row_scale(box, dt).reshape(-1)
    cs = np.tile(elder.col_scale(box), box.N)
    Dr, Dc = sp.diags(rs), sp.diags(cs)
    perm = nested_dissection(box.nx, box.ny, box.nz)
    u = (u_old if u0 is None else u0).copy()
    F = elder.residual(box, coef, u, u_old, dt)
    r = float(np.linalg.norm(F.ravel() * rs))
    r0 = r
    its = 0
    for its in range(1, max_it + 1):
        if r <= max(rtol * r0, atol):
            its -= 1
            break
        J = elder.jacobian(box, coef, u, dt)
        A = Dr @ J @ Dc
        rhs = -F.ravel() * rs
        if dense:
            dt_ = np.linalg.solve(A.toarray(), rhs)
        else:
            dt_ = sparse_solve(A, rhs, perm)
        delta = (dt_ * cs).reshape(u.shape)
        lam = 1.0
        for _ in range(ls_max + 1):
            ut = u + lam * delta
            Ft = elder.residual(box, coef, ut, u_old, dt)
            rt = float(np.linalg.norm(Ft.ravel() * rs))
            if rt <= (1.0 - lam / 4.0) * r:
                break
            lam *= 0.5
        else:
            lam *= 2.0
        u, F, r = ut, Ft, rt
        if np.max(np.abs(dt_)) * lam <= 1e-15:
            break
    if stats is not None:
        stats.update(newton_its=its, defect=r, defect0=r0)
    return u


def time_steps(box, coef, u0, dt, n_steps, rtol=1e-13, callback=None):
    """n_steps implicit-Euler steps from u0; returns the final state."""
    u = u0.copy()
    for n in range(n_steps):
        u = newton_solve(box, coef, u, dt, rtol=rtol)
        if callback is not None:
            callback(n + 1, u)
    return u
