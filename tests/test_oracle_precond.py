"""Pins of the oracle's block preconditioner (no GPU)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import assembly, pfc, precond


def _mk(dim, N, h=0.6, jitter=0.1):
    mesh = wl.make_mesh(dim, N, h=h, jitter=jitter, seed=21)
    M, K = assembly.mass_stiffness(mesh)
    return mesh, M, K


@pytest.mark.parametrize("dim,N,tau", [(2, 4, 0.1), (2, 5, 1.3), (3, 3, 0.5)])
def test_five_steps_equal_dense_PCH_inverse(dim, N, tau):
    mesh, M, K = _mk(dim, N)
    inner = precond.InnerSolvers(M, K, tau, mode="exact")
    P3 = precond.P3_dense(M, K, tau)
    rng = np.random.default_rng(1)
    for _ in range(3):
        v = rng.normal(size=3 * mesh.n)
        z = precond.pch_apply(inner, v)
        z_ref = np.linalg.solve(P3, v)
        assert np.linalg.norm(z - z_ref) <= 1e-12 * np.linalg.norm(z_ref)


@pytest.mark.parametrize("tau", [0.05, 0.8, 3.0])
def test_LU_factorisation_of_P_of_S(tau):
    mesh, M, K = _mk(2, 4)
    Md, Kd, B = precond.dense_blocks(M, K)
    for S in (precond.schur_exact(Md, Kd, B, tau), precond.schur_ch(Md, Kd, B, tau)):
        L, U = precond.L_U_of_S(Md, Kd, tau, S)
        P = precond.P_of_S(Md, Kd, tau, S)
        assert np.abs(L @ U - P).max() < 1e-12 * np.abs(P).max()
    # the Schur form of P(S) with the exact S is the paper's P (eq. pfc-preconditioner)
    d = math.sqrt(tau)
    Pex = np.block([[Md, 2 * Kd - B], [tau * Kd, Md - d * Kd + d * B]])
    assert np.abs(precond.P_of_S(Md, Kd, tau, precond.schur_exact(Md, Kd, B, tau)) - Pex).max() < 1e-12 * np.abs(Pex).max()


@pytest.mark.parametrize("tau,psibar,r,m11", [(0.1, -0.3, -0.35, 1.0), (1.0, -0.25, -0.3, 1.0),
                                              (0.5, -0.3, -0.35, 1.0 / pfc.ROS3PW_GAMMA)])
def test_spectrum_of_preconditioned_system(tau, psibar, r, m11):
    """Constant state: sigma(A P_CH^{-1}) = {1 (2n times)} u {lambda(mu)}, mu in sigma(M^{-1} K)."""
    mesh, M, K = _mk(2, 4, jitter=0.0)
    n = mesh.n
    N = assembly.N_matrix(mesh, np.full(n, psibar))
    tau_s = tau / m11  # block row 1 divided by m11
    A = pfc.AR_sparse(M, K, N, r, tau_s, 1.0).toarray()
    P3 = precond.P3_dense(M, K, tau_s)
    Q = A @ np.linalg.inv(P3)
    mu = sla.eigh(K.toarray(), M.toarray(), eigvals_only=True)
    d = math.sqrt(tau_s)
    c = 3 * psibar ** 2 + 1 + r
    lam = (1 + tau_s * (c * mu - 2 * mu ** 2 + mu ** 3)) / ((1 + d * mu) * (1 + math.sqrt(d) * mu) ** 2)
    # trace = sum of all eigenvalues (insensitive to the defective unit eigenvalue)
    assert abs(np.trace(Q) - (2 * n + lam.sum())) < 1e-10 * (2 * n + abs(lam).sum())
    # every predicted non-unit eigenvalue makes A - lambda P3 singular
    for l in lam:
        s = np.linalg.svd(A - l * P3, compute_uv=False)
        assert s[-1] < 1e-11 * s[0]
    # the same numbers are the printed third eigenvalue of Q_CH with k^2 -> mu (eq. eigenvalues_B_ch)
    from oracle.symbols import eig_printed_QCH
    # the printed set uses tau for the time step; here psibar enters through c
    lam_p = np.array([eig_printed_QCH(m, tau_s, r, psibar) for m in mu])
    assert np.abs(lam_p - lam).max() < 1e-12


@pytest.mark.parametrize("tau", [0.01, 0.1, 0.5])
def test_lemma2_interval(tau):
    mesh, M, K = _mk(2, 6, h=0.5)
    Md, Kd, B = precond.dense_blocks(M, K)
    S = precond.schur_exact(Md, Kd, B, tau)
    Sch = precond.schur_ch(Md, Kd, B, tau)
    ev = np.sort(sla.eigh(S, Sch, eigvals_only=True))
    d = math.sqrt(tau)
    assert ev.min() >= (1 - math.sqrt(d)) / 2 - 1e-12 and ev.max() <= 1 + 1e-12
    # reading of the garbled proof: lambda(mu) = (1 - 2 d mu + d mu^2) / (1 + sqrt(d) mu)^2
    mu = sla.eigh(Kd, Md, eigvals_only=True)
    lam = np.sort((1 - 2 * d * mu + d * mu ** 2) / (1 + math.sqrt(d) * mu) ** 2)
    assert np.abs(ev - lam).max() < 1e-10


def test_printed_PCH_block_does_not_reproduce_printed_spectrum():
    """Documents the reading: with the printed (0,1) block -2 sqrt(delta) K - B the trace identity fails."""
    mesh, M, K = _mk(2, 4, jitter=0.0)
    n = mesh.n
    tau, psibar, r = 0.3, -0.3, -0.35
    Md, Kd, B = precond.dense_blocks(M, K)
    d = math.sqrt(tau)
    P2 = np.block([[Md, -2 * math.sqrt(d) * Kd - B], [tau * Kd, Md + (d + 2 * math.sqrt(d)) * Kd + d * B]])
    P3 = np.zeros((3 * n, 3 * n))
    P3[:2 * n, :2 * n] = P2
    P3[2 * n:, n:2 * n] = Kd
    P3[2 * n:, 2 * n:] = Md
    A = pfc.AR_sparse(M, K, assembly.N_matrix(mesh, np.full(n, psibar)), r, tau, 1.0).toarray()
    mu = sla.eigh(Kd, Md, eigvals_only=True)
    c = 3 * psibar ** 2 + 1 + r
    lam = (1 + tau * (c * mu - 2 * mu ** 2 + mu ** 3)) / ((1 + d * mu) * (1 + math.sqrt(d) * mu) ** 2)
    assert abs(np.trace(A @ np.linalg.inv(P3)) - (2 * n + lam.sum())) > 1e-3


@pytest.mark.parametrize("dim,N,tau", [(2, 4, 0.1), (3, 3, 0.5)])
def test_SD_five_steps_equal_dense_inverse(dim, N, tau):
    mesh, M, K = _mk(dim, N)
    inner = precond.InnerSolvers(M, K, tau, mode="exact", schur="D")
    P3 = precond.P3_dense(M, K, tau, schur="D")
    v = np.random.default_rng(2).normal(size=3 * mesh.n)
    z = precond.pch_apply(inner, v)
    assert np.linalg.norm(z - np.linalg.solve(P3, v)) <= 1e-11 * np.linalg.norm(z)


@pytest.mark.parametrize("tau", [0.01, 0.1, 0.3])
def test_lemma1_interval_3d(tau):
    """Lemma 1 with the printed tetrahedral bound: eig(S_D^{-1} S) in [0.3924, 2.5]."""
    mesh, M, K = _mk(3, 4, h=0.7, jitter=0.0)
    Md, Kd, B = precond.dense_blocks(M, K)
    S = precond.schur_exact(Md, Kd, B, tau)
    SD = precond.schur_D_dense(Md, Kd, tau)
    ev = sla.eigh(S, SD, eigvals_only=True)
    assert ev.min() >= 0.3924 - 1e-12 and ev.max() <= 2.5 + 1e-12


def test_SD_preconditioned_fgmres_converges():
    from oracle import assembly, solve
    import workloads as wl
    mesh = wl.make_mesh(2, 12, jitter=0.1, seed=3)
    M, K = assembly.mass_stiffness(mesh)
    psi = wl.psi0(mesh.n, -0.3, 0.05, seed=3)
    Nm = assembly.N_matrix(mesh, psi)
    b = np.random.default_rng(1).normal(size=3 * mesh.n)
    y, info = solve.solve_stage(M, K, Nm, -0.35, 0.1, 1.0, b, tol=1e-8, schur="D")
    A = pfc.AR_sparse(M, K, Nm, -0.35, 0.1, 1.0)
    assert info["converged"] and np.linalg.norm(b - A @ y) <= 1e-8 * np.linalg.norm(b)
    assert all(c[2] == 20 and c[3] == 0 for c in info["schedule"].inner)
