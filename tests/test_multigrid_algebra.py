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
