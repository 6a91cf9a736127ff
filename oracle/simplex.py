"""Exact integration on simplices and P1 element geometry (oracle, test infrastructure).

The P1 basis restricted to a simplex T in R^m is the set of barycentric
coordinates lambda_0..lambda_m (Section 3, P1 Lagrange elements).  Every
integral the method needs (mass matrix, psi^2-weighted mass matrix, the cubic
load) is an integral of a product of barycentric coordinates, for which the
classical closed form holds:

    int_T prod_a lambda_a^{alpha_a} dx = |T| * m! * prod_a alpha_a! / (m + |alpha|)!

The oracle evaluates every element integral through this one formula, looping
over monomials; it does not use any pre-simplified element formula.

Pinned by tests/test_oracle_assembly.py: the formula against brute-force
quadrature on a reference triangle and tetrahedron, volumes against the
known cell volume, gradients against finite differences of the affine map.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def monomial_integral_factor(m: int, alpha) -> float:
    """m! * prod(alpha_a!) / (m + |alpha|)!, i.e. int_T prod lambda^alpha / |T|."""
    num = math.factorial(m)
    for a in alpha:
        num *= math.factorial(int(a))
    return num / math.factorial(m + int(sum(alpha)))


def product_table(m: int, degree: int) -> np.ndarray:
    """Table I[i_1, ..., i_degree] = int_T lambda_{i_1} ... lambda_{i_degree} / |T|.

    Indices range over the m+1 local vertices; repeated indices raise the
    exponent of that barycentric coordinate.
    """
    k = m + 1
    tab = np.zeros((k,) * degree)
    for idx in itertools.product(range(k), repeat=degree):
        alpha = [0] * k
        for a in idx:
            alpha[a] += 1
        tab[idx] = monomial_integral_factor(m, alpha)
    return tab


def simplex_geometry(coords: np.ndarray):
    """Volumes and barycentric gradients of a batch of simplices.

    coords: [E, m+1, m] vertex coordinates.
    Returns (vol [E], grad [E, m+1, m]) where grad[e, a] = grad lambda_a on element e.

    With the affine map x = X_0 + B xi (B columns X_a - X_0), lambda_a = xi_a
    for a >= 1, so grad lambda_a is row a-1 of B^{-1}; lambda_0 = 1 - sum xi.
    """
    coords = np.asarray(coords, dtype=np.float64)
    E, k, m = coords.shape
    assert k == m + 1
    B = np.transpose(coords[:, 1:, :] - coords[:, :1, :], (0, 2, 1))  # [E, m, m], columns X_a - X_0
    det = np.linalg.det(B)
    vol = np.abs(det) / math.factorial(m)
    Binv = np.linalg.inv(B)  # rows are gradients of xi_a
    grad = np.empty((E, k, m))
    grad[:, 1:, :] = Binv
    grad[:, 0, :] = -Binv.sum(axis=1)
    return vol, grad
