"""Pins of the oracle's simplex integration and P1 assembly (no GPU)."""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import assembly, simplex


def _duffy_rule(m, npts=8):
    """Quadrature on the reference simplex by collapsed Gauss-Legendre coordinates (independent of the monomial formula)."""
    g, w = np.polynomial.legendre.leggauss(npts)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    pts, wts = [], []
    if m == 2:
        for (u, wu), (v, wv) in itertools.product(zip(g, w), zip(g, w)):
            pts.append((u, v * (1 - u)))
            wts.append(wu * wv * (1 - u))
    else:
        for (u, wu), (v, wv), (s, ws) in itertools.product(zip(g, w), zip(g, w), zip(g, w)):
            pts.append((u, v * (1 - u), s * (1 - u) * (1 - v)))
            wts.append(wu * wv * ws * (1 - u) ** 2 * (1 - v))
    return np.array(pts), np.array(wts)


@pytest.mark.parametrize("m", [2, 3])
def test_monomial_table_matches_quadrature(m):
    pts, wts = _duffy_rule(m)
    lam = np.concatenate([1.0 - pts.sum(axis=1, keepdims=True), pts], axis=1)  # barycentric
    vol_ref = 1.0 / math.factorial(m)
    tab = simplex.product_table(m, 4)
    for idx in itertools.product(range(m + 1), repeat=4):
        q = np.sum(wts * np.prod(lam[:, list(idx)], axis=1)) / vol_ref
        assert abs(q - tab[idx]) < 1e-14


@pytest.mark.parametrize("m", [2, 3])
def test_geometry_volume_and_gradients(m):
    rng = np.random.default_rng(3)
    X = rng.normal(size=(1, m + 1, m))
    vol, grad = simplex.simplex_geometry(X)
    # volume from the Cayley-Menger-free determinant of edge vectors
    E = X[0, 1:] - X[0, 0]
    assert abs(vol[0] - abs(np.linalg.det(E)) / math.factorial(m)) < 1e-14
    # gradients: lambda_a(X_b) = delta_ab with lambda affine
    for a in range(m + 1):
        for b in range(m + 1):
            val = (1.0 if a == 0 else 0.0) + grad[0, a] @ (X[0, b] - X[0, 0])
            assert abs(val - (1.0 if a == b else 0.0)) < 1e-12


@pytest.mark.parametrize("dim,N,jit", [(2, 8, 0.0), (2, 8, 0.2), (3, 4, 0.0), (3, 4, 0.2)])
def test_mass_sum_and_stiffness_kernel(dim, N, jit):
    mesh = wl.make_mesh(dim, N, jitter=jit, seed=5)
    M, K = assembly.mass_stiffness(mesh)
    assert abs(M.sum() - mesh.L ** dim) < 1e-11 * mesh.L ** dim
    assert np.abs(K @ np.ones(mesh.n)).max() < 1e-13
    assert abs(M - M.T).max() < 1e-15 and abs(K - K.T).max() < 1e-14
    Md = M.toarray()
    Kd = K.toarray()
    assert np.linalg.eigvalsh(Md).min() > 0
    ek = np.linalg.eigvalsh(Kd)
    assert ek[0] > -1e-12 and ek[1] > 1e-8  # PSD with a one-dimensional kernel
    # P1 pattern: 7 entries per row in 2D, 15 in 3D
    assert set(np.diff(M.indptr)) == {7 if dim == 2 else 15}


def test_2d_unjittered_stencil_closed_form():
    h = 0.7
    N = 6
    mesh = wl.periodic_mesh_2d(N, h)
    M, K = assembly.mass_stiffness(mesh)
    i0 = 2 + N * 3
    def node(di, dj):
        return ((2 + di) % N) + N * ((3 + dj) % N)
    assert abs(K[i0, i0] - 4.0) < 1e-13
    for di, dj in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
        assert abs(K[i0, node(di, dj)] + 1.0) < 1e-13
    for di, dj in [(1, 1), (-1, -1)]:
        assert abs(K[i0, node(di, dj)]) < 1e-13
    assert abs(M[i0, i0] - h * h / 2) < 1e-14
    for di, dj in [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)]:
        assert abs(M[i0, node(di, dj)] - h * h / 12) < 1e-14


def test_2d_generalized_eigenvalues_closed_form():
    h = 0.45
    N = 6
    mesh = wl.periodic_mesh_2d(N, h)
    M, K = assembly.mass_stiffness(mesh)
    ev = np.sort(sla.eigh(K.toarray(), M.toarray(), eigvals_only=True))
    th = 2 * np.pi * np.arange(N) / N
    t1, t2 = np.meshgrid(th, th, indexing="ij")
    mu = (4 - 2 * np.cos(t1) - 2 * np.cos(t2)) / (h * h * (0.5 + (np.cos(t1) + np.cos(t2) + np.cos(t1 + t2)) / 6))
    assert np.abs(ev - np.sort(mu.ravel())).max() < 1e-11 * mu.max()


@pytest.mark.parametrize("dim,N", [(2, 5), (3, 3)])
def test_N_and_g_identities(dim, N):
    mesh = wl.make_mesh(dim, N, jitter=0.2, seed=2)
    M, K = assembly.mass_stiffness(mesh)
    c = -0.37
    Nc = assembly.N_matrix(mesh, np.full(mesh.n, c))
    assert abs(Nc - (-3 * c * c) * M).max() < 1e-15
    psi = wl.psi0(mesh.n, -0.3, 0.2, seed=4)
    Mp = assembly.mass_psi2(mesh, psi)
    g = assembly.load_psi3(mesh, psi)
    assert np.abs(Mp @ psi - g).max() < 1e-14
    assert abs(Mp.sum() - psi @ (M @ psi)) < 1e-13
    assert abs(Mp - Mp.T).max() < 1e-16
    Nm = assembly.N_matrix(mesh, psi)
    assert abs(Nm - (-3.0) * Mp).max() == 0.0


def test_element_psi2_integral_by_quadrature():
    """One jittered triangle: int psi_h^2 lambda_i lambda_j by direct quadrature in physical coordinates."""
    mesh = wl.periodic_mesh_2d(3, 1.0, jitter=0.2, seed=9)
    psi = wl.psi0(mesh.n, 0.1, 0.5, seed=1)
    e = 4
    X = mesh.elem_coords[e]
    pts, wts = _duffy_rule(2)
    lam = np.concatenate([1.0 - pts.sum(axis=1, keepdims=True), pts], axis=1)
    area = abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0]], axis=1))) / 2
    ph = lam @ psi[mesh.elem_nodes[e]]
    Mp = assembly.mass_psi2(mesh, psi).toarray()
    # element contributions: compare against the assembled matrix minus the other elements
    others = wl.Mesh(2, mesh.n, np.delete(mesh.elem_nodes, e, axis=0), np.delete(mesh.elem_coords, e, axis=0), mesh.N, mesh.h)
    Mo = assembly.mass_psi2(others, psi).toarray()
    for a in range(3):
        for b in range(3):
            q = 2 * area * np.sum(wts * ph ** 2 * lam[:, a] * lam[:, b])
            ia, ib = mesh.elem_nodes[e, a], mesh.elem_nodes[e, b]
            assert abs((Mp - Mo)[ia, ib] - q) < 1e-14
