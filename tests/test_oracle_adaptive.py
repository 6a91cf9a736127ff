"""Pins of the embedded Ros3Pw solution and the step-size controller (no GPU)."""
import math

import numpy as np

import workloads as wl
from oracle import adaptive, assembly, pfc
from oracle.reference import dense_solve


def _ode_run(k, embedded):
    F = lambda x: np.array([-x[0] ** 2 + x[1], -x[1] - x[0] * x[1]])
    J = lambda x: np.array([[-2 * x[0], 1.0], [-x[1], -1 - x[0]]])
    x = np.array([1.0, 0.5])
    tau = 1.0 / k
    for _ in range(k):
        W = np.eye(2) / (tau * pfc.ROS3PW_GAMMA) - J(x)
        xn, xh, _ = pfc.ros3pw_step(x, tau, F, lambda y: y, lambda rhs, i, xi: np.linalg.solve(W, rhs))
        x = xh if embedded else xn
    return x


def test_embedded_solution_is_second_order():
    ref = _ode_run(4096, False)
    e = [np.linalg.norm(_ode_run(k, True) - ref) for k in (16, 32, 64, 128)]
    orders = [math.log2(a / b) for a, b in zip(e, e[1:])]
    assert min(orders) > 1.9 and max(orders) < 2.1, orders


def _pfc_setup(h=4.0, N=4, amp=0.4):
    mesh = wl.make_mesh(2, N, h=h, jitter=0.15, seed=11)
    M, K = assembly.mass_stiffness(mesh)
    r = -0.35
    psi = wl.psi0(mesh.n, -0.2, amp, seed=8)
    x0 = pfc.consistent_init(mesh, M, K, r, psi)
    prob = pfc.PFCProblem(mesh, M, K, r)
    m11 = 1.0 / pfc.ROS3PW_GAMMA

    def lin(N_, tau_, bR, i):
        return dense_solve(pfc.AR_sparse(M, K, N_, r, tau_, m11), bR)

    return mesh, prob, x0, lin


def test_adaptive_run_meets_tolerance_and_rejects():
    mesh, prob, x0, lin = _pfc_setup()
    n = mesh.n
    T = 2.0
    # reference: fine fixed steps
    xr = x0.copy()
    for _ in range(512):
        xr, _, _ = prob.step(xr, T / 512, lin)
    errs = []
    for rtol in (1e-3, 1e-4, 1e-5):
        x, taus, rej = adaptive.rosenbrock_adaptive(prob, x0, 1.0, T, rtol, rtol, lin)
        assert abs(sum(taus) - T) <= 1e-12
        errs.append(np.linalg.norm(x[n:2 * n] - xr[n:2 * n]) / np.linalg.norm(xr[n:2 * n]))
    # the global error follows the requested tolerance
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] <= 1e-4
    # a too large first step (tau0 = 1 at rtol 1e-5) is rejected at least once
    _, taus, rej = adaptive.rosenbrock_adaptive(prob, x0, 1.0, T, 1e-5, 1e-5, lin)
    assert rej >= 1 and max(taus) < 1.0


def test_controller_safeguards():
    """No growth right after a rejection; a failed linear solve rejects the step and shrinks tau by facmin."""
    mesh, prob, x0, lin = _pfc_setup()
    T, cap = 2.0, 0.3

    def capped(N_, tau_, bR, i):
        if tau_ > cap:
            raise adaptive.LinearSolveFailed()
        return lin(N_, tau_, bR, i)

    log = []
    x, taus, rej = adaptive.rosenbrock_adaptive(prob, x0, 1.0, T, 1e-4, 1e-4, capped, log=log)
    assert abs(sum(taus) - T) <= 1e-12 and max(taus) <= cap
    kinds = [k for _, k in log]
    assert kinds[0] == "failed" and kinds.count("failed") >= 1
    assert rej == kinds.count("failed") + kinds.count("rejected")
    for (h0, k0), (h1, k1) in zip(log, log[1:]):
        if k0 == "failed":
            assert h1 == h0 * adaptive.FACMIN or h1 < h0 * adaptive.FACMIN  # the end time may clip it
        if k0 == "rejected":
            assert h1 < h0
    for a, b, c in zip(log, log[1:], log[2:]):
        if a[1] != "accepted" and b[1] == "accepted":
            assert c[0] <= b[0] * (1 + 1e-15)
    # without failures the log holds the same steps as the accepted taus
    log2 = []
    _, taus2, rej2 = adaptive.rosenbrock_adaptive(prob, x0, 1.0, T, 1e-5, 1e-5, lin, log=log2)
    assert [h for h, k in log2 if k == "accepted"] == taus2 and rej2 == sum(k == "rejected" for _, k in log2)
