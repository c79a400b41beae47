"""The algebra the V-cycle's zero-start forms rest on, checked with plain numpy on small
random block systems (CPU).  Block Gauss-Seidel over the 8 colours (i % 2, j % 2, k % 2)
of a 27-point stencil of 2x2 blocks, started from x = 0:

- the colour of the neighbour at offset o of a vertex of colour c is c with the parity
  bit of every odd component of o flipped, so the blocks a colour's first sweep needs
  (neighbours of colours already swept) are fixed per colour;
- after a single such sweep the residual b - A x of a vertex of colour c equals minus the
  sum of A_vo x_{v+o} over its neighbours of the colours swept after c.
"""
import itertools

import numpy as np

OFFS = list(itertools.product((-1, 0, 1), repeat=3))  # (dz, dy, dx)


def colour(i, j, k):
    return (i % 2) + 2 * (j % 2) + 4 * (k % 2)


def random_system(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    n = nx * ny * nz
    A = np.zeros((2 * n, 2 * n))
    idx = lambda i, j, k: i + nx * (j + ny * k)
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        v = idx(i, j, k)
        for dz, dy, dx in OFFS:
            ii, jj, kk = i + dx, j + dy, k + dz
            if not (0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz):
                continue
            w = idx(ii, jj, kk)
            blk = rng.uniform(-1, 1, (2, 2))
            if v == w:  # diagonally dominant diagonal blocks
                blk += np.diag([30.0, 30.0])
            A[2 * v:2 * v + 2, 2 * w:2 * w + 2] = blk
    b = rng.standard_normal(2 * n)
    return A, b, idx


def test_neighbour_colour_is_a_parity_flip():
    for c in range(8):
        i, j, k = c & 1, (c >> 1) & 1, c >> 2
        i, j, k = i + 2, j + 2, k + 2  # away from the edges
        for dz, dy, dx in OFFS:
            m = (dx != 0) | ((dy != 0) << 1) | ((dz != 0) << 2)
            assert colour(i + dx, j + dy, k + dz) == c ^ m


def test_zero_start_block_counts():
    """0, 2, 6, 8, 18, 20, 24, 26 of the 26 off-diagonal blocks, 13 on average: each
    coupling is read from exactly one of its two ends."""
    counts = []
    for c in range(8):
        n = 0
        for dz, dy, dx in OFFS:
            m = (dx != 0) | ((dy != 0) << 1) | ((dz != 0) << 2)
            n += (c ^ m) < c
        counts.append(n)
    assert counts == [0, 2, 6, 8, 18, 20, 24, 26]
    assert sum(counts) == 8 * 13


def test_residual_after_one_zero_start_sweep():
    nx, ny, nz = 6, 5, 4
    A, b, idx = random_system(nx, ny, nz, seed=5)
    verts = [(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]
    x = np.zeros_like(b)
    # one forward block Gauss-Seidel sweep over the colours, reading only the colours
    # already swept (the others are still zero)
    for c in range(8):
        for (i, j, k) in verts:
            if colour(i, j, k) != c:
                continue
            v = idx(i, j, k)
            r = b[2 * v:2 * v + 2].copy()
            for dz, dy, dx in OFFS:
                ii, jj, kk = i + dx, j + dy, k + dz
                if (dx, dy, dz) == (0, 0, 0) or not (0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz):
                    continue
                if colour(ii, jj, kk) >= c:
                    continue
                w = idx(ii, jj, kk)
                r -= A[2 * v:2 * v + 2, 2 * w:2 * w + 2] @ x[2 * w:2 * w + 2]
            x[2 * v:2 * v + 2] = np.linalg.solve(A[2 * v:2 * v + 2, 2 * v:2 * v + 2], r)
    # the same sweep written as the general one (every neighbour, x zero where not yet
    # swept) gives the same x
    x2 = np.zeros_like(b)
    for c in range(8):
        for (i, j, k) in verts:
            if colour(i, j, k) != c:
                continue
            v = idx(i, j, k)
            rv = b[2 * v:2 * v + 2] - A[2 * v:2 * v + 2] @ x2
            x2[2 * v:2 * v + 2] += np.linalg.solve(A[2 * v:2 * v + 2, 2 * v:2 * v + 2], rv)
    assert np.allclose(x, x2, rtol=1e-13, atol=1e-15)
    full = b - A @ x
    short = np.zeros_like(b)
    for (i, j, k) in verts:
        v, c = idx(i, j, k), colour(i, j, k)
        for dz, dy, dx in OFFS:
            ii, jj, kk = i + dx, j + dy, k + dz
            if not (0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz):
                continue
            if colour(ii, jj, kk) <= c:
                continue
            w = idx(ii, jj, kk)
            short[2 * v:2 * v + 2] -= A[2 * v:2 * v + 2, 2 * w:2 * w + 2] @ x[2 * w:2 * w + 2]
    assert np.abs(full - short).max() <= 1e-12 * np.abs(b).max()
    # colour 7, swept last, has zero residual
    for (i, j, k) in verts:
        if colour(i, j, k) == 7:
            v = idx(i, j, k)
            assert np.abs(full[2 * v:2 * v + 2]).max() <= 1e-12


# ---------------------------------------------------------------------------------------
# Vertical-line block Gauss-Seidel: every z-column (i, j) is solved exactly, the columns
# in 4 colours (i % 2, j % 2).  The column's block tridiagonal part is factored from the
# top (M_k = D_k - L_k C_{k-1}, C_k = M_k^{-1} U_k); a sweep solves d_k = M_k^{-1} (r_k -
# L_k d_{k-1}) downwards and x_k = d_k - C_k x_{k+1} upwards.
# ---------------------------------------------------------------------------------------

def column_colour(i, j):
    return (i % 2) + 2 * (j % 2)


def _blk(A, v, w):
    return A[2 * v:2 * v + 2, 2 * w:2 * w + 2]


def _column_solve(A, idx, i, j, nz, rhs):
    """The block-LU solve of the column (i, j) as the line kernels do it."""
    C = np.zeros((2, 2))
    Mi, Cs = [], []
    for k in range(nz):
        v = idx(i, j, k)
        L = _blk(A, v, idx(i, j, k - 1)) if k > 0 else np.zeros((2, 2))
        U = _blk(A, v, idx(i, j, k + 1)) if k + 1 < nz else np.zeros((2, 2))
        m_inv = np.linalg.inv(_blk(A, v, v) - L @ C)
        C = m_inv @ U
        Mi.append(m_inv)
        Cs.append(C)
    d, dprev = [], np.zeros(2)
    for k in range(nz):
        v = idx(i, j, k)
        L = _blk(A, v, idx(i, j, k - 1)) if k > 0 else np.zeros((2, 2))
        dprev = Mi[k] @ (rhs[k] - L @ dprev)
        d.append(dprev)
    x, y = [None] * nz, np.zeros(2)
    for k in range(nz - 1, -1, -1):
        y = d[k] - Cs[k] @ y
        x[k] = y
    return x


def test_column_block_lu_is_the_tridiagonal_solve():
    nx, ny, nz = 3, 3, 7
    A, b, idx = random_system(nx, ny, nz, seed=9)
    i, j = 1, 2
    rows = [2 * idx(i, j, k) + e for k in range(nz) for e in range(2)]
    T = A[np.ix_(rows, rows)]
    rhs = np.random.default_rng(3).standard_normal((nz, 2))
    x = np.concatenate(_column_solve(A, idx, i, j, nz, rhs))
    assert np.allclose(T @ x, rhs.ravel(), rtol=0, atol=1e-12)


def test_line_zero_start_block_counts():
    """The first line sweep of column colour cc reads the 3 blocks of every neighbour
    column of a colour below cc: 0, 6, 18, 24 (each coupling between columns once)."""
    counts = []
    for cc in range(4):
        i, j = 2 + (cc & 1), 2 + (cc >> 1)
        n = sum(3 for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                if (dx, dy) != (0, 0) and column_colour(i + dx, j + dy) < cc)
        counts.append(n)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                m = (dx != 0) | ((dy != 0) << 1)
                assert column_colour(i + dx, j + dy) == cc ^ m
    assert counts == [0, 6, 18, 24]


def test_residual_after_one_zero_start_line_sweep():
    nx, ny, nz = 5, 6, 5
    A, b, idx = random_system(nx, ny, nz, seed=7)
    cols = [(i, j) for j in range(ny) for i in range(nx)]

    def off_column(i, j, k, x, keep):
        r = b[2 * idx(i, j, k):2 * idx(i, j, k) + 2].copy()
        for dz, dy, dx in OFFS:
            ii, jj, kk = i + dx, j + dy, k + dz
            if (dx, dy) == (0, 0) or not (0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz):
                continue
            if keep(column_colour(ii, jj)):
                r -= _blk(A, idx(i, j, k), idx(ii, jj, kk)) @ x[2 * idx(ii, jj, kk):2 * idx(ii, jj, kk) + 2]
        return r

    x = np.zeros_like(b)   # zero-start form: only columns of the colours already swept
    x2 = np.zeros_like(b)  # general form from zero
    for cc in range(4):
        for (i, j) in cols:
            if column_colour(i, j) != cc:
                continue
            r = [off_column(i, j, k, x, lambda c: c < cc) for k in range(nz)]
            r2 = [off_column(i, j, k, x2, lambda c: True) for k in range(nz)]
            for k, (xk, xk2) in enumerate(zip(_column_solve(A, idx, i, j, nz, r),
                                              _column_solve(A, idx, i, j, nz, r2))):
                x[2 * idx(i, j, k):2 * idx(i, j, k) + 2] = xk
                x2[2 * idx(i, j, k):2 * idx(i, j, k) + 2] = xk2
    assert np.allclose(x, x2, rtol=1e-13, atol=1e-15)
    full = b - A @ x
    short = np.zeros_like(b)
    for (i, j) in cols:
        cc = column_colour(i, j)
        for k in range(nz):
            v = idx(i, j, k)
            for dz, dy, dx in OFFS:
                ii, jj, kk = i + dx, j + dy, k + dz
                if (dx, dy) == (0, 0) or not (0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz):
                    continue
                if column_colour(ii, jj) <= cc:
                    continue
                w = idx(ii, jj, kk)
                short[2 * v:2 * v + 2] -= _blk(A, v, w) @ x[2 * w:2 * w + 2]
    assert np.abs(full - short).max() <= 1e-12 * np.abs(b).max()
    for (i, j) in cols:  # the last column colour has zero residual
        if column_colour(i, j) == 3:
            for k in range(nz):
                v = idx(i, j, k)
                assert np.abs(full[2 * v:2 * v + 2]).max() <= 1e-12
