"""Pins of the oracle's P2 (quadratic Lagrange) matrices (Section 3, p = 2); no GPU."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import assembly, p2
from oracle.simplex import simplex_geometry


def _nodes_bary(m):
    """Barycentric coordinates of the P2 nodes: vertices, then edge midpoints."""
    k = m + 1
    pts = [np.eye(k)[a] for a in range(k)]
    for i, j in p2.P2_EDGES[m]:
        pts.append(0.5 * (np.eye(k)[i] + np.eye(k)[j]))
    return pts


@pytest.mark.parametrize("m", [2, 3])
def test_basis_lagrange_and_partition_of_unity(m):
    B = p2.basis(m)
    pts = _nodes_bary(m)
    V = np.array([[p2.peval(B[a], lam) for a in range(len(B))] for lam in pts])
    assert np.abs(V - np.eye(len(B))).max() < 1e-14
    rng = np.random.default_rng(0)
    for _ in range(5):
        lam = rng.dirichlet(np.ones(m + 1))
        assert abs(sum(p2.peval(b, lam) for b in B) - 1.0) < 1e-14
    # the edge order of the oracle is the mesh generator's
    assert p2.P2_EDGES[m] == wl.P2_EDGES[m]


def _collapsed_rule(m, npts=6):
    """Points (reference coordinates xi) and weights of a collapsed Gauss rule on the unit simplex."""
    g, w = np.polynomial.legendre.leggauss(npts)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    X, W = [], []
    if m == 2:
        for u, wu in zip(g, w):
            for v, wv in zip(g, w):
                X.append([u, (1 - u) * v])
                W.append(wu * wv * (1 - u))
    else:
        for u, wu in zip(g, w):
            for v, wv in zip(g, w):
                for t, wt in zip(g, w):
                    X.append([u, (1 - u) * v, (1 - u) * (1 - v) * t])
                    W.append(wu * wv * wt * (1 - u) ** 2 * (1 - v))
    return np.array(X), np.array(W)


@pytest.mark.parametrize("m", [2, 3])
def test_element_tables_against_quadrature(m):
    rng = np.random.default_rng(4)
    X = rng.normal(size=(m + 1, m)) + 2.0 * np.eye(m + 1, m)      # a generic simplex
    B = (X[1:] - X[0]).T
    vol = abs(np.linalg.det(B)) / math.factorial(m)
    basis = p2.basis(m)
    q = len(basis)
    psi = rng.normal(size=q)
    xi, wq = _collapsed_rule(m)
    M_e = np.zeros((q, q))
    K_e = np.zeros((q, q))
    Mp_e = np.zeros((q, q))
    g_e = np.zeros(q)
    Binv = np.linalg.inv(B)
    eps = 1e-6
    for x, w in zip(xi, wq):
        lam = np.concatenate([[1.0 - x.sum()], x])
        phi = np.array([p2.peval(b, lam) for b in basis])
        # physical gradients by central differences in physical coordinates
        grad = np.zeros((q, m))
        for d in range(m):
            dx = np.zeros(m)
            dx[d] = eps
            dxi = Binv @ dx
            lp = np.concatenate([[1.0 - (x + dxi).sum()], x + dxi])
            lm = np.concatenate([[1.0 - (x - dxi).sum()], x - dxi])
            grad[:, d] = [(p2.peval(b, lp) - p2.peval(b, lm)) / (2 * eps) for b in basis]
        ps = phi @ psi
        jw = w * vol * math.factorial(m)   # |det B| d xi
        M_e += jw * np.outer(phi, phi)
        K_e += jw * grad @ grad.T
        Mp_e += jw * ps * ps * np.outer(phi, phi)
        g_e += jw * ps ** 3 * phi
    M2, D, C4 = p2.tables(m)
    _, gl = simplex_geometry(X[None])
    G = gl[0] @ gl[0].T
    assert np.abs(vol * M2 - M_e).max() < 1e-13 * np.abs(M_e).max()
    assert np.abs(vol * np.einsum("ij,ijab->ab", G, D) - K_e).max() < 1e-7 * np.abs(K_e).max()
    assert np.abs(vol * np.einsum("abcd,c,d->ab", C4, psi, psi) - Mp_e).max() < 1e-12 * np.abs(Mp_e).max()
    assert np.abs(vol * np.einsum("abcd,b,c,d->a", C4, psi, psi, psi) - g_e).max() < 1e-12 * np.abs(g_e).max()


@pytest.mark.parametrize("dim,N", [(2, 5), (3, 3)])
def test_global_p2_matrices(dim, N):
    mesh = wl.p2_mesh(wl.make_mesh(dim, N, jitter=0.2, seed=3))
    M, K = assembly.mass_stiffness(mesh)
    vol = simplex_geometry(mesh.elem_coords)[0].sum()
    assert abs(M.sum() - vol) < 1e-12 * vol
    assert np.abs(K @ np.ones(mesh.n)).max() < 1e-12 * abs(K).max()
    assert abs(M - M.T).max() < 1e-15 and abs(K - K.T).max() < 1e-13
    ev = sla.eigvalsh(M.toarray())
    assert ev.min() > 0.0
    evK = sla.eigvalsh(K.toarray())
    assert evK.min() > -1e-12 and np.sum(evK < 1e-10 * evK.max()) == 1
    psi = wl.psi0(mesh.n, -0.3, 0.3, seed=2)
    c = 0.7
    Mc = assembly.mass_psi2(mesh, np.full(mesh.n, c))
    assert abs(Mc - c * c * M).max() < 1e-14 * abs(M).max()
    Mp = assembly.mass_psi2(mesh, psi)
    g = assembly.load_psi3(mesh, psi)
    assert np.abs(Mp @ psi - g).max() < 1e-13 * np.abs(g).max()
    assert abs(Mp.sum() - psi @ (M @ psi)) < 1e-12 * abs(Mp.sum())
    N_ = assembly.N_matrix(mesh, psi)
    assert abs(N_ + 3.0 * Mp).max() == 0.0


def test_laplace_eigenvalues_converge_at_order_h4():
    """Lowest nonzero eigenvalue of K x = lam M x on the periodic square of side L: the exact
    value is (2 pi / L)^2; P2 errors fall 16x per halving of h, P1 errors 4x."""
    L = 6.0
    exact = (2 * math.pi / L) ** 2
    e1, e2 = [], []
    for N in (4, 8, 16):
        base = wl.make_mesh(2, N, h=L / N)
        for deg, errs in ((1, e1), (2, e2)):
            mesh = base if deg == 1 else wl.p2_mesh(base)
            M, K = assembly.mass_stiffness(mesh)
            lam = sla.eigh(K.toarray(), M.toarray(), eigvals_only=True)
            errs.append(abs(np.sort(lam)[1] - exact) / exact)
    r1 = [a / b for a, b in zip(e1, e1[1:])]
    r2 = [a / b for a, b in zip(e2, e2[1:])]
    assert all(3.0 < r < 5.0 for r in r1), r1
    assert all(12.0 < r < 20.0 for r in r2), r2
    assert e2[-1] < 1e-3 * e1[-1] * 10


def test_p2_stage_solve_matches_dense():
    from oracle import pfc, solve
    from oracle.reference import dense_solve
    mesh = wl.p2_mesh(wl.make_mesh(2, 6, jitter=0.1, seed=5))
    M, K = assembly.mass_stiffness(mesh)
    psi = wl.psi0(mesh.n, -0.3, 0.05, seed=5)
    N_ = assembly.N_matrix(mesh, psi)
    b = np.random.default_rng(7).normal(size=3 * mesh.n)
    m11 = 1.0 / pfc.ROS3PW_GAMMA
    y, info = solve.solve_stage(M, K, N_, -0.35, 0.5, m11, b, tol=1e-12)
    yd = dense_solve(pfc.AR_sparse(M, K, N_, -0.35, 0.5, m11), b)
    assert info["converged"] and np.linalg.norm(y - yd) <= 1e-9 * np.linalg.norm(yd)
