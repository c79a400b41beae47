"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the solver itself: it only produces the
physical constants of the 3D Elder box (Table 1 of the paper, with the readings
listed below), the workload shapes, the random parameter points xi, and random
states used as shared starting points for per-step parity.

Readings taken where the paper is ambiguous:
  * molecular diffusion D_m = 3.565e-6 m^2/s (Table 1 prints 0.565e-6; 3.565e-6
    gives the classical Elder Rayleigh number 400),
  * z is depth (k = 0 is the top face), gravity is +9.81 along +z,
  * one time step is one month = 365/12 days = 2,628,000 s,
  * porosity/permeability parameters xi are uniform on [-1, 1].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MONTH_S = 365.0 / 12.0 * 86400.0  # 2,628,000 s

# Table 1 of the paper (Section 2.1), with D_m and gravity read as stated above.
ELDER_BOX = {
    "lx": 600.0, "ly": 600.0, "lz": 150.0,
    "rho0": 1000.0, "rho1": 1200.0, "mu": 1.0e-3, "g": 9.81,
    "Dm": 3.565e-6, "phi_mean": 0.1, "K_mean": 4.845e-13,
    # closed top patch [x0, x1] x [y0, y1] at z = 0 where c = 1
    "patch": (150.0, 450.0, 150.0, 450.0),
}

# porosity / permeability field models (see oracle.elder.coefficients)
FIELD_CONST = 0      # phi = phi_mean, K = K_mean
FIELD_COS1 = 1       # one cosine mode of phi, Kozeny-Carman K
FIELD_LATTICE4 = 2   # two modes of phi + two modes of log K
FIELD_PAPER3 = 3     # the paper's three-variable sine field (Section 5, box with 3 RVs)

N_XI = {FIELD_CONST: 0, FIELD_COS1: 1, FIELD_LATTICE4: 4, FIELD_PAPER3: 3}


def physics(field_model: int = FIELD_CONST, **over) -> dict:
    """Physical constants of the Elder box plus the porosity field model."""
    p = dict(ELDER_BOX)
    p["field_model"] = int(field_model)
    p.update(over)
    return p


@dataclass
class Group:
    """One resolution group: `samples` realisations on an nx*ny*nz vertex grid."""
    nx: int
    ny: int
    nz: int
    samples: int
    levels: int

    @property
    def n_vertices(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class Workload:
    name: str
    groups: list
    field_model: int
    steps: int
    dt: float = MONTH_S
    precision: str = "f64"          # "f64" or "mixed" (FP32 V-cycle)
    newton_rtol: float = 1e-10
    xi: np.ndarray = field(default=None, repr=False)  # [S_total, n_xi]
    weights: np.ndarray = field(default=None, repr=False)  # quadrature weights (gPC)
    mlmc_levels: tuple = None       # samples per level of a multilevel workload

    @property
    def n_samples(self) -> int:
        return sum(g.samples for g in self.groups)


# --------------------------------------------------------------------------
# Rank-1 lattice (quasi-Monte Carlo points on [0,1)^s, shifted), built by the
# component-by-component rule that minimises the worst-case error of the
# unweighted Korobov space with smoothness 2.
# --------------------------------------------------------------------------

def _bernoulli2(x):
    return x * x - x + 1.0 / 6.0


def lattice_vector(n: int, s: int) -> np.ndarray:
    """Component-by-component generating vector for an n-point lattice in s dims."""
    cand = np.array([z for z in range(1, n) if math.gcd(z, n) == 1], dtype=np.int64)
    k = np.arange(n, dtype=np.int64)
    prod = np.ones(n)
    z = []
    for _ in range(s):
        best, best_err, best_col = None, None, None
        for zc in cand:
            col = 1.0 + 2.0 * math.pi ** 2 * _bernoulli2(((k * zc) % n) / n)
            err = np.mean(prod * col)
            if best_err is None or err < best_err - 1e-15:
                best, best_err, best_col = int(zc), err, col
        z.append(best)
        prod = prod * best_col
    return np.array(z, dtype=np.int64)


def lattice_points(n: int, s: int, seed: int = 0) -> np.ndarray:
    """xi_i = 2 frac(i z / n + shift) - 1, i = 0..n-1, shift ~ U[0,1)^s from `seed`."""
    z = lattice_vector(n, s)
    shift = np.random.default_rng(seed).random(s)
    i = np.arange(n, dtype=np.int64)[:, None]
    u = np.mod((i * z[None, :]) % n / n + shift[None, :], 1.0)
    return 2.0 * u - 1.0


# --------------------------------------------------------------------------
# Halton points (quasi-Monte Carlo on [0,1)^s): coordinate d of point i is the
# radical inverse of i in the d-th prime base
# --------------------------------------------------------------------------

PRIMES = (2, 3, 5, 7, 11, 13, 17, 19)


def radical_inverse(i: int, base: int) -> float:
    """The base-`base` digits of i written in reverse order after the radix point."""
    x, f = 0.0, 1.0 / base
    while i > 0:
        i, d = divmod(i, base)
        x += d * f
        f /= base
    return x


def halton_points(n: int, s: int, skip: int = 1) -> np.ndarray:
    """xi_i = 2 (phi_2(i), phi_3(i), phi_5(i), ...) - 1 for i = skip .. skip + n - 1 (the
    first index, 0, maps to the corner and is skipped by default)."""
    return np.array([[2.0 * radical_inverse(i, PRIMES[d]) - 1.0 for d in range(s)]
                     for i in range(skip, skip + n)])


def gauss_legendre_tensor(n: int, m: int):
    """Full tensor n^m Gauss-Legendre nodes on [-1, 1]^m (first coordinate slowest) and
    weights of the uniform probability measure (summing to 1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    grids = np.meshgrid(*([x] * m), indexing="ij")
    wg = np.meshgrid(*([w] * m), indexing="ij")
    nodes = np.stack([g.ravel() for g in grids], axis=1)
    weights = np.prod(np.stack([g.ravel() for g in wg], axis=1), axis=1) / 2.0 ** m
    return nodes, weights


YEAR_S = 365.0 * 86400.0
# the box experiment on two grids; on the paper's 129x129x33 mesh its 325 samples would
# need ~390 GB in FP64, more than one GPU holds
E1_GRIDS = {"e1box33": (33, 33, 9, 4), "e1box65": (65, 65, 17, 5)}


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def workload(name: str, seed: int = 0) -> Workload:
    """The five benchmark workloads of the Elder box, with seeded parameter points.

    g33 = 33x33x9 vertices, g65 = 65x65x17, g129 = 129x129x33, g257 = 257x257x65.
    """
    if name == "elder33_f64":          # one deterministic sample, 20 steps, FP64
        return Workload(name, [Group(33, 33, 9, 1, 4)], FIELD_CONST, 20,
                        newton_rtol=1e-10, xi=np.zeros((1, 0)))
    if name == "elder129_f64":         # one perturbed sample, 200 steps, FP64
        xi1 = np.random.default_rng(seed).uniform(-1.0, 1.0)
        return Workload(name, [Group(129, 129, 33, 1, 6)], FIELD_COS1, 200,
                        newton_rtol=1e-8, xi=np.array([[xi1]]))
    if name == "qmc512_mixedres":      # 512 lattice points, three resolutions, FP64
        pts = lattice_points(512, 4, seed)
        i = np.arange(512)
        sel33 = i[i % 2 == 0]
        sel129 = i[i % 8 == 1]
        sel65 = i[(i % 8 == 3) | (i % 8 == 5) | (i % 8 == 7)]
        xi = np.concatenate([pts[sel33], pts[sel65], pts[sel129]])
        return Workload(name, [Group(33, 33, 9, 256, 4), Group(65, 65, 17, 192, 5),
                               Group(129, 129, 33, 64, 6)], FIELD_LATTICE4, 100,
                        newton_rtol=1e-8, xi=xi)
    if name == "mixed257":             # FP32 V-cycle: one 257^2x65 sample + 32 129^2x33
        pts = lattice_points(512, 4, seed)
        i = np.arange(512)
        xi = np.concatenate([pts[:1], pts[i % 16 == 0]])
        return Workload(name, [Group(257, 257, 65, 1, 7), Group(129, 129, 33, 32, 6)],
                        FIELD_LATTICE4, 100, precision="mixed", newton_rtol=1e-8, xi=xi)
    if name == "adjoint65":            # 64 samples for the gradient workload
        pts = lattice_points(512, 4, seed)
        i = np.arange(512)
        return Workload(name, [Group(65, 65, 17, 64, 5)], FIELD_LATTICE4, 50,
                        newton_rtol=1e-10, xi=pts[i % 8 == 0])
    if name == "gpc125":               # the paper's 3-parameter box field at 125 nodes
        nodes, weights = gauss_legendre_tensor(5, 3)
        return Workload(name, [Group(65, 65, 17, 125, 5)], FIELD_PAPER3, 3,
                        newton_rtol=1e-8, xi=nodes, weights=weights)
    if name == "mlmc3":                # multilevel MC on the nested 33^3/65^3/129^3 grids:
        # group l holds the n_l samples of level l, then the coarse partners (same xi) of
        # the n_{l+1} samples of level l + 1; every level draws its own shifted lattice
        n = (256, 64, 16)
        pts = [lattice_points(k, 4, seed + 1 + l) for l, k in enumerate(n)]
        xi = np.concatenate([pts[0], pts[1], pts[1], pts[2], pts[2]])
        return Workload(name, [Group(33, 33, 9, n[0] + n[1], 4), Group(65, 65, 17, n[1] + n[2], 5),
                               Group(129, 129, 33, n[2], 6)], FIELD_LATTICE4, 100,
                        newton_rtol=1e-8, xi=xi, mlmc_levels=n)
    if name in E1_GRIDS:               # the paper's box experiment with 3 parameters:
        # 200 Halton qMC samples (group 0) beside the 125 tensor Gauss-Legendre nodes of the
        # degree-4 surrogate (group 1) on one grid, 1500 steps of 0.005 years
        nx, ny, nz, levels = E1_GRIDS[name]
        nodes, weights = gauss_legendre_tensor(5, 3)
        xi = np.concatenate([halton_points(200, 3), nodes])
        return Workload(name, [Group(nx, ny, nz, 200, levels), Group(nx, ny, nz, 125, levels)],
                        FIELD_PAPER3, 1500, dt=0.005 * YEAR_S, newton_rtol=1e-8, xi=xi,
                        weights=weights)
    raise KeyError(name)


WORKLOADS = ("elder33_f64", "elder129_f64", "qmc512_mixedres", "mixed257", "adjoint65", "gpc125",
             "e1box33", "e1box65", "mlmc3")


# --------------------------------------------------------------------------
# States
# --------------------------------------------------------------------------

def initial_state(nx: int, ny: int, nz: int, phys: dict) -> np.ndarray:
    """Pure water at rest below the brine patch: c = 0 except c = 1 on the closed top
    patch, p = rho0 g z (z = depth).  Shape [nz, ny, nx, 2] with (p, c) last."""
    hx, hy, hz = phys["lx"] / (nx - 1), phys["ly"] / (ny - 1), phys["lz"] / (nz - 1)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x, y, z = i * hx, j * hy, k * hz
    x0, x1, y0, y1 = phys["patch"]
    tol = 1e-9 * max(phys["lx"], phys["ly"])
    on_patch = (k == 0) & (x >= x0 - tol) & (x <= x1 + tol) & (y >= y0 - tol) & (y <= y1 + tol)
    u = np.zeros((nz, ny, nx, 2))
    u[..., 0] = phys["rho0"] * phys["g"] * z
    u[..., 1] = np.where(on_patch, 1.0, 0.0)
    return u


def random_state(nx: int, ny: int, nz: int, phys: dict, seed: int,
                 dp: float = 2.0e3) -> np.ndarray:
    """A generic state: hydrostatic p plus a random perturbation of size `dp` Pa and
    c uniform in [0, 1].  Used as a shared point for defect/Jacobian parity."""
    rng = np.random.default_rng(seed)
    hz = phys["lz"] / (nz - 1)
    k = np.arange(nz)[:, None, None] * np.ones((1, ny, nx))
    u = np.empty((nz, ny, nx, 2))
    u[..., 0] = phys["rho0"] * phys["g"] * k * hz + dp * rng.standard_normal((nz, ny, nx))
    u[..., 1] = rng.random((nz, ny, nx))
    return u
