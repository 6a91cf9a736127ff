"""Pins of the oracle's PFC1 model (mobility psi^+, Section 2 and eq. rosenbrock_matrix); no GPU."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import assembly, mobility as mob, pfc, solve
from oracle.reference import dense_solve
from oracle.simplex import simplex_geometry


def _tiny(dim=2, N=4, h=0.9, jitter=0.15, seed=11):
    mesh = wl.make_mesh(dim, N, h=h, jitter=jitter, seed=seed)
    M, K = assembly.mass_stiffness(mesh)
    return mesh, M, K


@pytest.mark.parametrize("dim", [2, 3])
def test_Kplus_constant_psi_and_structure(dim):
    mesh, M, K = _tiny(dim=dim, N=3 if dim == 3 else 5)
    c = 0.37
    Kp = mob.K_plus(mesh, np.full(mesh.n, c))
    assert abs(Kp - (c - mob.PSI_MIN) * K).max() <= 1e-13 * abs(K).max()
    psi = wl.psi0(mesh.n, -0.3, 0.5, seed=2)
    Kp = mob.K_plus(mesh, psi)
    assert abs(Kp - Kp.T).max() <= 1e-15 * abs(Kp).max()
    assert np.abs(Kp @ np.ones(mesh.n)).max() <= 1e-13 * abs(Kp).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_F_row_and_column_sums(dim):
    mesh, M, K = _tiny(dim=dim, N=3 if dim == 3 else 5)
    mu = np.random.default_rng(3).normal(size=mesh.n)
    Fm = mob.F_mu(mesh, mu)
    one = np.ones(mesh.n)
    # row sums: int grad mu . grad phi_i = (K mu)_i;  column sums: sum_i phi_i = 1 has no gradient
    assert np.abs(Fm @ one - K @ mu).max() <= 1e-12 * np.abs(K @ mu).max()
    assert np.abs(Fm.T @ one).max() <= 1e-12 * abs(Fm).max()
    assert abs(mob.F_mu(mesh, np.full(mesh.n, 2.5))).max() <= 1e-13
    # F is not symmetric in general (the mobility derivative is a convection-like term)
    assert abs(Fm - Fm.T).max() > 1e-3 * abs(Fm).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_element_matrices_against_centroid_rule(dim):
    """Both integrands are linear on a simplex, so the one-point centroid rule is exact."""
    mesh, M, K = _tiny(dim=dim, N=2, jitter=0.2)
    rng = np.random.default_rng(5)
    psi = rng.normal(size=mesh.n)
    mu = rng.normal(size=mesh.n)
    e = 0
    X = mesh.elem_coords[e]                         # [k, dim] vertices
    k = dim + 1
    B = (X[1:] - X[0]).T                            # affine map columns
    vol = abs(np.linalg.det(B)) / math.factorial(dim)
    Binv = np.linalg.inv(B)
    G = np.vstack([-Binv.sum(axis=0), Binv])        # grad of each barycentric coordinate [k, dim]
    nodes = mesh.elem_nodes[e]
    pplus_c = np.mean(psi[nodes] - mob.PSI_MIN)     # psi^+ at the centroid
    gmu = G.T @ mu[nodes]
    lam_c = np.full(k, 1.0 / k)                     # barycentric coordinates of the centroid
    Kp_e = vol * pplus_c * (G @ G.T)
    F_e = vol * np.outer(G @ gmu, lam_c)            # [a (test), b (trial)]
    # compare with the element's contribution: assemble only element e
    class One:
        pass
    one = One()
    one.dim, one.n = dim, mesh.n
    one.elem_nodes = mesh.elem_nodes[e:e + 1]
    one.elem_coords = mesh.elem_coords[e:e + 1]
    Kp = mob.K_plus(one, psi).toarray()[np.ix_(nodes, nodes)]
    Fm = mob.F_mu(one, mu).toarray()[np.ix_(nodes, nodes)]
    assert np.abs(Kp - Kp_e).max() <= 1e-13 * np.abs(Kp_e).max()
    assert np.abs(Fm - F_e).max() <= 1e-13 * np.abs(F_e).max()
    assert abs(simplex_geometry(one.elem_coords)[0][0] - vol) <= 1e-15


def test_AR1_is_scaled_jacobian_of_F1():
    """Block row 1 of A^R is tau times the negative Jacobian of -K_+(psi) mu, plus m11 M."""
    mesh, M, K = _tiny()
    r, tau = -0.35, 0.3
    n = mesh.n
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=n), -0.3 + 0.4 * rng.normal(size=n), rng.normal(size=n)])
    v = rng.normal(size=3 * n)
    eps = 1e-5
    Jv = (mob.F_weak1(mesh, M, K, r, x + eps * v) - mob.F_weak1(mesh, M, K, r, x - eps * v)) / (2 * eps)
    N = assembly.N_matrix(mesh, x[n:2 * n])
    Kp = mob.K_plus(mesh, x[n:2 * n])
    Fm = mob.F_mu(mesh, x[:n])
    m11 = 1.0 / pfc.ROS3PW_GAMMA
    W = -Jv
    W[n:2 * n] = tau * W[n:2 * n] + m11 * (M @ v[n:2 * n])
    AR = mob.apply_AR1(M, K, N, Kp, Fm, r, tau, m11, v)
    assert np.abs(AR - W).max() < 1e-8 * np.abs(AR).max()
    # dropping F, or using its transpose, breaks the identity
    bad = mob.apply_AR1(M, K, N, Kp, Fm.T.tocsr(), r, tau, m11, v)
    assert np.abs(bad - W).max() > 1e-4 * np.abs(AR).max()
    assert np.allclose(mob.AR1_sparse(M, K, N, Kp, Fm, r, tau, m11) @ v, AR, rtol=0, atol=1e-12 * np.abs(AR).max())


def _run1(mesh, M, K, x0, r, tau, steps):
    x, _ = mob.rosenbrock_run1(mesh, M, K, x0, r, tau, steps, solver="dense")
    return x


def test_pfc1_rosenbrock_order_and_conservation():
    mesh, M, K = _tiny(N=4, h=4.0)
    r = -0.35
    psi = wl.psi0(mesh.n, -0.2, 0.4, seed=8)
    x0 = pfc.consistent_init(mesh, M, K, r, psi)
    T = 2.0
    ref = _run1(mesh, M, K, x0, r, T / 1024, 1024)
    n = mesh.n
    errs = []
    for k in (8, 16, 32, 64):
        x = _run1(mesh, M, K, x0, r, T / k, k)
        errs.append(np.linalg.norm(x[n:2 * n] - ref[n:2 * n]))
        assert abs(np.sum(M @ x[n:2 * n]) - np.sum(M @ psi)) < 1e-12 * max(1.0, abs(np.sum(M @ psi)))
    orders = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert min(orders[1:]) > 2.8, (errs, orders)
    # the mobility changes the dynamics: PFC1 and PFC2 runs differ
    x2 = __import__("oracle.solve", fromlist=["x"]).rosenbrock_run(mesh, M, K, x0, r, T / 16, 16, solver="dense")[0]
    assert np.linalg.norm(x2[n:2 * n] - _run1(mesh, M, K, x0, r, T / 16, 16)[n:2 * n]) > 1e-3 * np.linalg.norm(psi)


def test_stage_rhs1_and_consistent_init():
    mesh, M, K = _tiny()
    r, tau = -0.3, 0.7
    n = mesh.n
    rng = np.random.default_rng(4)
    xi = np.concatenate([rng.normal(size=n), -0.3 + 0.2 * rng.normal(size=n), rng.normal(size=n)])
    ys = [rng.normal(size=3 * n) for _ in range(2)]
    c = [pfc.ROS3PW_C[(3, 1)], pfc.ROS3PW_C[(3, 2)]]
    b = mob.stage_rhs_R1(mesh, M, K, r, tau, xi, [y[n:2 * n] for y in ys], c)
    prob = mob.PFC1Problem(mesh, M, K, r)
    gen = prob.F(xi) + sum((cc / tau) * prob.mass_apply(y) for cc, y in zip(c, ys))
    gen[n:2 * n] *= tau
    assert np.abs(b - gen).max() < 1e-13 * np.abs(gen).max()
    # blocks 0 and 2 of the operator do not involve the mobility
    psi = wl.psi0(n, -0.25, 0.3, seed=3)
    x0 = pfc.consistent_init(mesh, M, K, r, psi)
    F = mob.F_weak1(mesh, M, K, r, x0)
    assert np.abs(F[:n]).max() < 1e-12 and np.abs(F[2 * n:]).max() < 1e-12


def test_mobility_mean():
    mesh, M, K = _tiny(jitter=0.2)
    psi = wl.psi0(mesh.n, -0.3, 0.2, seed=6)
    m0 = mob.mobility_mean(M, psi)
    # the mean of the P1 interpolant: int psi_h / |Omega|, int psi_h = sum of the element integrals
    vol, _ = simplex_geometry(mesh.elem_coords)
    integral = float(np.sum(vol * psi[mesh.elem_nodes].mean(axis=1)))
    assert abs(m0 - (integral / vol.sum() - mob.PSI_MIN)) <= 1e-14 * abs(m0)


def test_constant_state_pfc1_equals_pfc2_at_scaled_step():
    """psi and mu constant: K_+ = M0 K and F = 0, so the PFC1 system and its preconditioner are
    the PFC2 ones at time step M0 tau; the solve and its whole schedule must coincide."""
    mesh, M, K = _tiny(N=6, jitter=0.1)
    n = mesh.n
    r, tau, m11 = -0.35, 0.4, 1.0 / pfc.ROS3PW_GAMMA
    psi = np.full(n, -0.3)
    N = assembly.N_matrix(mesh, psi)
    Kp = mob.K_plus(mesh, psi)
    Fm = mob.F_mu(mesh, np.full(n, 0.8))
    m0 = mob.mobility_mean(M, psi)
    assert abs(m0 - 1.2) < 1e-14
    b = np.random.default_rng(9).normal(size=3 * n)
    y1, i1 = solve.solve_stage(M, K, N, r, tau, m11, b, Kp=Kp, Fm=Fm, m0=m0)
    y2, i2 = solve.solve_stage(M, K, N, r, m0 * tau, m11, b)
    assert i1["schedule"].inner == i2["schedule"].inner and i1["cycles"] == i2["cycles"]
    assert np.linalg.norm(y1 - y2) <= 1e-12 * np.linalg.norm(y2)
    # the preconditioner without the mobility mean takes more iterations here
    y3, i3 = solve.solve_stage(M, K, N, r, tau, m11, b, Kp=Kp, Fm=Fm, m0=1.0)
    assert i3["schedule"].inner != i1["schedule"].inner


def test_pfc1_fgmres_matches_dense():
    mesh, M, K = _tiny(N=6, jitter=0.1)
    n = mesh.n
    r, tau, m11 = -0.35, 0.5, 1.0 / pfc.ROS3PW_GAMMA
    rng = np.random.default_rng(12)
    x = np.concatenate([rng.normal(size=n), wl.psi0(n, -0.3, 0.3, seed=1), rng.normal(size=n)])
    N = assembly.N_matrix(mesh, x[n:2 * n])
    Kp = mob.K_plus(mesh, x[n:2 * n])
    Fm = mob.F_mu(mesh, x[:n])
    b = rng.normal(size=3 * n)
    y, info = solve.solve_stage(M, K, N, r, tau, m11, b, tol=1e-12, Kp=Kp, Fm=Fm,
                                m0=mob.mobility_mean(M, x[n:2 * n]))
    yd = dense_solve(mob.AR1_sparse(M, K, N, Kp, Fm, r, tau, m11), b)
    assert info["converged"] and np.linalg.norm(y - yd) <= 1e-9 * np.linalg.norm(yd)
