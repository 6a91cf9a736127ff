"""Pins of the oracle's Rosenbrock stage system (no GPU)."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import assembly, pfc
from oracle.reference import dense_solve

GOLD = __import__("json").load(open(__file__.rsplit("/", 1)[0] + "/golden/paper_values.json"))


def _scalar_R(z):
    """Stability function of the generic step on y' = lam y with tau = 1, z = lam."""
    lam = z
    F = lambda x: lam * x
    mass = lambda y: y
    solve = lambda rhs, i, xi: rhs / (1.0 / pfc.ROS3PW_GAMMA - lam)
    x1, _, _ = pfc.ros3pw_step(np.array([1.0]), 1.0, F, mass, solve)
    return float(x1[0])


def test_ros3pw_third_order_stability_function():
    errs = [abs(_scalar_R(z) - math.exp(z)) for z in (0.1, 0.05, 0.025)]
    # local error of an order-3 method is O(z^4): ratio 16 per halving
    for a, b in zip(errs, errs[1:]):
        assert 12.0 < a / b < 20.0
    assert abs(_scalar_R(-1e9) - GOLD["ros3pw_R_inf"]["value"]) < 1e-6
    # strongly A-stable: |R| <= 1 on the negative axis
    assert all(abs(_scalar_R(-x)) <= 1.0 for x in np.logspace(-3, 6, 50))


def _tiny(dim=2, N=4, h=0.9):
    mesh = wl.make_mesh(dim, N, h=h, jitter=0.15, seed=11)
    M, K = assembly.mass_stiffness(mesh)
    return mesh, M, K


def test_AR_is_scaled_jacobian_of_F():
    mesh, M, K = _tiny()
    r, tau = -0.35, 0.3
    n = mesh.n
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=n), -0.3 + 0.4 * rng.normal(size=n), rng.normal(size=n)])
    v = rng.normal(size=3 * n)
    eps = 1e-5
    Jv = (pfc.F_weak(mesh, M, K, r, x + eps * v) - pfc.F_weak(mesh, M, K, r, x - eps * v)) / (2 * eps)
    N = assembly.N_matrix(mesh, x[n:2 * n])
    W = -Jv
    W[n:2 * n] += (M @ v[n:2 * n]) / (tau * pfc.ROS3PW_GAMMA)
    W[n:2 * n] *= tau
    AR = pfc.apply_AR(M, K, N, r, tau, 1.0 / pfc.ROS3PW_GAMMA, v)
    assert np.abs(AR - W).max() < 1e-8 * np.abs(AR).max()


def test_consistent_init_zeroes_algebraic_rows():
    mesh, M, K = _tiny()
    r = -0.3
    psi = wl.psi0(mesh.n, -0.25, 0.3, seed=3)
    x0 = pfc.consistent_init(mesh, M, K, r, psi)
    F = pfc.F_weak(mesh, M, K, r, x0)
    n = mesh.n
    assert np.abs(F[:n]).max() < 1e-12 and np.abs(F[2 * n:]).max() < 1e-12
    assert np.array_equal(x0[n:2 * n], psi)
    # the mass solves agree with a sparse LU solve
    import scipy.sparse.linalg as spla
    om = spla.spsolve(M.tocsc(), -(K @ psi))
    assert np.abs(x0[2 * n:] - om).max() <= 1e-13 * np.abs(om).max()


def _run(mesh, M, K, x0, r, tau, steps):
    prob = pfc.PFCProblem(mesh, M, K, r)
    m11 = 1.0 / pfc.ROS3PW_GAMMA

    def lin(N, tau_, bR, i):
        return dense_solve(pfc.AR_sparse(M, K, N, r, tau_, m11), bR)

    x = x0.copy()
    for _ in range(steps):
        x, _, _ = prob.step(x, tau, lin)
    return x


def test_pfc_rosenbrock_order_and_conservation():
    """Third order in the non-stiff regime (coarse mesh, h = 4), conservation of int psi_h."""
    mesh, M, K = _tiny(N=4, h=4.0)
    r = -0.35
    psi = wl.psi0(mesh.n, -0.2, 0.4, seed=8)
    x0 = pfc.consistent_init(mesh, M, K, r, psi)
    T = 2.0
    ref = _run(mesh, M, K, x0, r, T / 1024, 1024)
    n = mesh.n
    errs = []
    for k in (8, 16, 32, 64):
        x = _run(mesh, M, K, x0, r, T / k, k)
        errs.append(np.linalg.norm(x[n:2 * n] - ref[n:2 * n]))
        # conservation of int psi_h = 1^T M psi
        assert abs(np.sum(M @ x[n:2 * n]) - np.sum(M @ psi)) < 1e-12 * max(1.0, abs(np.sum(M @ psi)))
    orders = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert min(orders[1:]) > 2.8, (errs, orders)


def test_stage_rhs_matches_generic_form():
    mesh, M, K = _tiny()
    r, tau = -0.3, 0.7
    n = mesh.n
    rng = np.random.default_rng(4)
    xi = np.concatenate([rng.normal(size=n), -0.3 + 0.2 * rng.normal(size=n), rng.normal(size=n)])
    ys = [rng.normal(size=3 * n) for _ in range(2)]
    c = [pfc.ROS3PW_C[(3, 1)], pfc.ROS3PW_C[(3, 2)]]
    b = pfc.stage_rhs_R(mesh, M, K, r, tau, xi, [y[n:2 * n] for y in ys], c)
    prob = pfc.PFCProblem(mesh, M, K, r)
    gen = prob.F(xi) + sum((cc / tau) * prob.mass_apply(y) for cc, y in zip(c, ys))
    gen[n:2 * n] *= tau
    assert np.abs(b - gen).max() < 1e-13 * np.abs(gen).max()
