"""Generalised polynomial chaos surrogate of the salt mass fraction.

TEST INFRASTRUCTURE ONLY (oracle).  Section 3.1 of the paper and its appendix:
  basis        Psi_beta(theta) = prod_j psi_{beta_j}(theta_j), psi_n the Legendre
               polynomials of the three-term recursion (appendix), uniform theta on
               [-1, 1]^M with density 2^-M
  truncation   J_{M,p}: total degree sum_j beta_j <= p (condition b) or every degree
               beta_j <= p (condition c)
  norms        Q_beta = <Psi_beta, Psi_beta> = prod_j 1 / (2 beta_j + 1)      (eq. spro)
  projection   c_beta(x) = (1 / Q_beta) sum_i w_i Psi_beta(theta_i) c(x, theta_i)
               with probability weights w_i (sum 1)                          (eq. PCEcoef)
  mean         c_0                                                            (eq. PCEcoef2)
  variance     sum_{beta != 0} Q_beta c_beta^2                                (eq. var)
  surrogate    c^(theta) = sum_beta c_beta Psi_beta(theta)                    (eq. PCEpoint)
  exceedance   #{s : c^(theta_s) > c*} / N_s over N_s points theta_s          (Section 3.2)

Multi-indices are ordered by total degree, then in decreasing lexicographic order
(for M = 2: (0,0), (1,0), (0,1), (2,0), (1,1), (0,2), ...).
"""
from __future__ import annotations

import itertools

import numpy as np


def legendre(n: int, x):
    """psi_n(x) by the recursion (k + 1) psi_{k+1} = (2k + 1) x psi_k - k psi_{k-1}."""
    x = np.asarray(x, dtype=float)
    p_prev, p = np.ones_like(x), x.copy()
    if n == 0:
        return p_prev
    for k in range(1, n):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    return p


def multi_indices(M: int, p: int, truncation: int = 0):
    """J_{M,p}: truncation 0 = total degree <= p, 1 = every component <= p."""
    out = []
    for t in range(0, M * p + 1):
        level = [b for b in itertools.product(range(p + 1), repeat=M) if sum(b) == t]
        if truncation == 0 and t > p:
            break
        out.extend(sorted(level, reverse=True))
    return out


def norms(indices):
    """Q_beta = prod_j 1 / (2 beta_j + 1)."""
    return np.array([np.prod([1.0 / (2 * b + 1) for b in beta]) for beta in indices])


def basis(indices, theta):
    """Psi_beta(theta_s) for points theta [N, M]: array [N, n_coef]."""
    theta = np.atleast_2d(np.asarray(theta, dtype=float))
    out = np.ones((theta.shape[0], len(indices)))
    for q, beta in enumerate(indices):
        for j, b in enumerate(beta):
            out[:, q] *= legendre(b, theta[:, j])
    return out


def tensor_gauss_legendre(M: int, q: int):
    """Full tensor Gauss-Legendre nodes [q^M, M] and probability weights (sum 1): the
    1D rule of q points (a library routine) in every direction, weights times 1/2 per
    direction for the uniform density."""
    x, w = np.polynomial.legendre.leggauss(q)
    nodes = np.array(list(itertools.product(x, repeat=M)))
    weights = np.array([np.prod(c) for c in itertools.product(w / 2.0, repeat=M)])
    return nodes, weights


def project(fields, theta, weights, indices):
    """gPC coefficients [n_coef, ...] of sample fields [S, ...] at nodes theta [S, M]
    with probability weights [S] (eq. PCEcoef)."""
    f = np.asarray(fields, dtype=float)
    B = basis(indices, theta)
    Q = norms(indices)
    coef = np.zeros((len(indices),) + f.shape[1:])
    for q in range(len(indices)):
        for i in range(f.shape[0]):
            coef[q] += weights[i] * B[i, q] * f[i]
        coef[q] /= Q[q]
    return coef


def moments(coef, indices):
    """(mean, variance) from the coefficients (eqs. PCEcoef2, var)."""
    Q = norms(indices)
    var = np.zeros(coef.shape[1:])
    for q in range(1, len(indices)):
        var += Q[q] * coef[q] ** 2
    return coef[0].copy(), var


def surrogate(coef, indices, theta):
    """c^(theta_s) at every vertex: [N, ...] (eq. PCEpoint)."""
    B = basis(indices, theta)
    return np.tensordot(B, coef, axes=(1, 0))


def exceedance(coef, indices, theta, threshold):
    """#{s : c^(theta_s) > c*} / N_s at every vertex (strict >)."""
    vals = surrogate(coef, indices, theta)
    return np.mean(vals > threshold, axis=0)
