"""P2 (quadratic Lagrange) finite-element matrices of the PFC system (oracle, test infrastructure).

Section 3 takes V_h with local polynomials of degree p = 1, 2; the studies of
Section 7 (Tables 3-5) use p = 2.  On a simplex with barycentric coordinates
lambda_0..lambda_m the P2 basis is
    vertex a:          lambda_a (2 lambda_a - 1)
    edge (i, j):       4 lambda_i lambda_j
with the element's nodes ordered vertices first, then edges in the order of
workloads.P2_EDGES.  Every basis function is a polynomial in the barycentric
coordinates; products are multiplied out and integrated exactly with the
monomial formula of `oracle.simplex`; gradients follow from
grad phi = sum_i (d phi / d lambda_i) grad lambda_i.  The matrices M, K,
N(psi) = -3 Mpsi2 and the load g(psi) have the definitions of `oracle.assembly`
(their integrands are of degree 4, 2, 8 and 8 on each simplex).

Pinned by tests/test_oracle_p2.py: Lagrange property and partition of unity
of the basis; the element tables against a collapsed-coordinate Gauss rule;
sum of M = |Omega|, K 1 = 0, symmetry, M positive definite; constant psi gives
N = -3 c^2 M, Mpsi2 psi = g(psi); the discrete Laplace eigenvalues converge to
the exact ones at order h^4 (order h^2 for P1).
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np

from .assembly import _assemble, _assemble_vec
from .simplex import monomial_integral_factor, simplex_geometry

P2_EDGES = {2: ((0, 1), (1, 2), (0, 2)),
            3: ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))}


def _unit(k, i):
    e = [0] * k
    e[i] = 1
    return tuple(e)


def _add(a, b):
    return tuple(x + y for x, y in zip(a, b))


def basis(m: int):
    """The P2 basis on an m-simplex as polynomials {exponent tuple: coefficient} in lambda."""
    k = m + 1
    out = []
    for a in range(k):
        out.append({_add(_unit(k, a), _unit(k, a)): 2.0, _unit(k, a): -1.0})
    for i, j in P2_EDGES[m]:
        out.append({_add(_unit(k, i), _unit(k, j)): 4.0})
    return out


def pmul(p, q):
    r = {}
    for a, ca in p.items():
        for b, cb in q.items():
            e = _add(a, b)
            r[e] = r.get(e, 0.0) + ca * cb
    return r


def pdiff(p, i):
    """d p / d lambda_i."""
    r = {}
    for a, c in p.items():
        if a[i] > 0:
            e = list(a)
            e[i] -= 1
            r[tuple(e)] = r.get(tuple(e), 0.0) + c * a[i]
    return r


def pint(p, m):
    """int_T p / |T|."""
    return sum(c * monomial_integral_factor(m, a) for a, c in p.items())


def peval(p, lam):
    return sum(c * np.prod([l ** e for l, e in zip(lam, a)]) for a, c in p.items())


@lru_cache(maxsize=None)
def tables(m: int):
    """Reference tables (divided by |T|): M2[a,b], D[i,j,a,b] = int d_i phi_a d_j phi_b, C4[a,b,c,d]."""
    B = basis(m)
    q = len(B)
    k = m + 1
    M2 = np.array([[pint(pmul(B[a], B[b]), m) for b in range(q)] for a in range(q)])
    dB = [[pdiff(B[a], i) for i in range(k)] for a in range(q)]
    D = np.zeros((k, k, q, q))
    for i, j, a, b in itertools.product(range(k), range(k), range(q), range(q)):
        D[i, j, a, b] = pint(pmul(dB[a][i], dB[b][j]), m)
    prod2 = [[pmul(B[a], B[b]) for b in range(q)] for a in range(q)]
    C4 = np.zeros((q, q, q, q))
    for a, b, c, d in itertools.product(range(q), repeat=4):
        if a <= b and c <= d:
            C4[a, b, c, d] = pint(pmul(prod2[a][b], prod2[c][d]), m)
    # fill the symmetric entries
    for a, b, c, d in itertools.product(range(q), repeat=4):
        C4[a, b, c, d] = C4[min(a, b), max(a, b), min(c, d), max(c, d)]
    return M2, D, C4


def mass_stiffness_p2(mesh):
    m = mesh.dim
    vol, grad = simplex_geometry(mesh.elem_coords)
    M2, D, _ = tables(m)
    G = np.einsum("eik,ejk->eij", grad, grad)                   # grad lambda_i . grad lambda_j
    Me = vol[:, None, None] * M2[None]
    Ke = vol[:, None, None] * np.einsum("eij,ijab->eab", G, D)
    return _assemble(mesh.elem_nodes, Me, mesh.n), _assemble(mesh.elem_nodes, Ke, mesh.n)


def mass_psi2_p2(mesh, psi):
    vol, _ = simplex_geometry(mesh.elem_coords)
    _, _, C4 = tables(mesh.dim)
    pe = np.asarray(psi, dtype=np.float64)[mesh.elem_nodes]
    Ee = vol[:, None, None] * np.einsum("abcd,ec,ed->eab", C4, pe, pe)
    return _assemble(mesh.elem_nodes, Ee, mesh.n)


def load_psi3_p2(mesh, psi):
    vol, _ = simplex_geometry(mesh.elem_coords)
    _, _, C4 = tables(mesh.dim)
    pe = np.asarray(psi, dtype=np.float64)[mesh.elem_nodes]
    ge = vol[:, None] * np.einsum("abcd,eb,ec,ed->ea", C4, pe, pe, pe)
    return _assemble_vec(mesh.elem_nodes, ge, mesh.n)
