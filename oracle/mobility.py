"""The PFC1 model: Wasserstein gradient flow with mobility psi^+ (oracle, test infrastructure).

Model (Section 2): d_t psi = div(psi^+ grad mu) with psi^+ = psi - psi_min,
psi_min = -1.5; mu and omega as in PFC2.  The matrices of Section 3 that the
mobility brings in:
    K_+(psi)_ij = (psi^+ grad phi_j, grad phi_i)        mobility matrix
    F(mu)_ij    = (phi_j grad mu, grad phi_i)          derivative of the mobility term
Weak-form operator (Section 3.1): blocks 0 and 2 as in PFC2, block 1
    F1(x) = -K_+(psi) mu.
Its Jacobian in block 1 is -K_+(psi) dmu - F(mu) dpsi, so the stage matrix
(eq. rosenbrock_matrix) is
    A^R = [[ M,              -(1+r) M + 2K + N(psi_k),   K ],
           [ tau K_+(psi_k),  m11 M + tau F(mu_k),        0 ],
           [ 0,               K,                          M ]]
and the stage right-hand side carries -tau K_+(psi_i) mu_i in block 1.

Preconditioner (Section 4): the constant-mobility approximation K_+ ~ M0 K
with M0 the mean of psi^+ and F dropped turns block (1,0) into tau M0 K, so
P_CH is built for the time step M0 tau (after the gamma scaling of block row
1: M0 tau / m11).  Reading: M0 = (1^T M psi)/(1^T M 1) - psi_min.  The scheme
conserves int psi_h (1^T K_+ = 0 and 1^T F = 0), so M0 is a constant of the
run; a Rosenbrock run evaluates it once from its initial state.

Element integrals (P1, exact): grad lambda is constant on a simplex, so
    int_T psi^+ grad l_a . grad l_b = (grad l_a . grad l_b) sum_c psi^+_c int_T l_c
    int_T l_b grad mu . grad l_a    = (sum_c mu_c grad l_c . grad l_a) int_T l_b
with int_T l_c = |T| / (m+1) from the monomial table of `oracle.simplex`.

Pinned by tests/test_oracle_mobility.py: constant psi gives K_+ = (c - psi_min) K;
K_+ symmetric with zero row sums; F(mu) 1 = K mu, 1^T F(mu) = 0, F(const) = 0;
both element matrices against a centroid rule computed from the affine map;
the stage matrix against central differences of the weak operator; psi-mass
conservation and third-order convergence of Rosenbrock runs; with constant
psi and mu the PFC1 solve equals the PFC2 solve at time step M0 tau, schedule
included.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .assembly import N_matrix, _assemble, load_psi3
from .pfc import PFCProblem, ROS3PW_GAMMA, ros3pw_step, split
from .simplex import product_table, simplex_geometry

PSI_MIN = -1.5


def K_plus(mesh, psi, psi_min=PSI_MIN) -> sp.csr_matrix:
    """K_+(psi)_ij = (psi^+ grad phi_j, grad phi_i), psi^+ = psi - psi_min."""
    m = mesh.dim
    vol, grad = simplex_geometry(mesh.elem_coords)
    I1 = product_table(m, 1)                                    # int l_c / |T|
    pp = (np.asarray(psi, dtype=np.float64) - psi_min)[mesh.elem_nodes]  # [E, k]
    mean = pp @ I1                                              # sum_c psi^+_c int l_c / |T|
    Ke = (vol * mean)[:, None, None] * np.einsum("eak,ebk->eab", grad, grad)
    return _assemble(mesh.elem_nodes, Ke, mesh.n)


def F_mu(mesh, mu) -> sp.csr_matrix:
    """F(mu)_ij = (phi_j grad mu, grad phi_i); row i is the test function."""
    m = mesh.dim
    vol, grad = simplex_geometry(mesh.elem_coords)
    I1 = product_table(m, 1)
    me = np.asarray(mu, dtype=np.float64)[mesh.elem_nodes]    # [E, k]
    gmu = np.einsum("ec,eck->ek", me, grad)                     # grad mu_h on each element
    ga = np.einsum("ek,eak->ea", gmu, grad)                     # grad mu . grad l_a
    Fe = vol[:, None, None] * ga[:, :, None] * I1[None, None, :]  # [E, a (row), b (column)]
    return _assemble(mesh.elem_nodes, Fe, mesh.n)


def mobility_mean(M, psi, psi_min=PSI_MIN) -> float:
    """M0 = mean of psi^+ over the domain = (1^T M psi) / (1^T M 1) - psi_min."""
    one = np.ones(M.shape[0])
    return float(one @ (M @ psi)) / float(one @ (M @ one)) - psi_min


def apply_AR1(M, K, N, Kp, Fm, r, tau, m11, y):
    """A^R y of the PFC1 stage matrix, y = (mu, psi, omega) stacked [3n]."""
    n = M.shape[0]
    mu, ps, om = split(y, n)
    out = np.empty(3 * n)
    out[:n] = M @ mu - (1.0 + r) * (M @ ps) + 2.0 * (K @ ps) + N @ ps + K @ om
    out[n:2 * n] = tau * (Kp @ mu) + m11 * (M @ ps) + tau * (Fm @ ps)
    out[2 * n:] = K @ ps + M @ om
    return out


def AR1_sparse(M, K, N, Kp, Fm, r, tau, m11):
    return sp.bmat([[M, -(1.0 + r) * M + 2.0 * K + N, K],
                    [tau * Kp, m11 * M + tau * Fm, None],
                    [None, K, M]], format="csr")


def F_weak1(mesh, M, K, r, x, psi_min=PSI_MIN):
    """Weak-form operator of PFC1 over the P1 basis."""
    n = M.shape[0]
    mu, ps, om = split(x, n)
    out = np.empty(3 * n)
    out[:n] = -(M @ mu) + (1.0 + r) * (M @ ps) - 2.0 * (K @ ps) - K @ om + load_psi3(mesh, ps)
    out[n:2 * n] = -(K_plus(mesh, ps, psi_min) @ mu)
    out[2 * n:] = -(M @ om) - K @ ps
    return out


def stage_rhs_R1(mesh, M, K, r, tau, x_i, y_prev_psi, c_row, psi_min=PSI_MIN):
    """b_i^R of PFC1: F(x_i) with block 1 times tau, plus sum_j c_ij M y_j^psi on block 1."""
    n = M.shape[0]
    b = F_weak1(mesh, M, K, r, x_i, psi_min)
    b[n:2 * n] *= tau
    for c, yp in zip(c_row, y_prev_psi):
        b[n:2 * n] += c * (M @ yp)
    return b


class PFC1Problem(PFCProblem):
    """A PFC1 instance: N(psi_k), K_+(psi_k) and F(mu_k) rebuilt each step."""

    def __init__(self, mesh, M, K, r, psi_min=PSI_MIN):
        super().__init__(mesh, M, K, r)
        self.psi_min = psi_min

    def F(self, x):
        return F_weak1(self.mesh, self.M, self.K, self.r, x, self.psi_min)

    def step(self, x, tau, linear_solve):
        """One Ros3Pw step.  linear_solve(N, Kp, Fm, tau, b_R, i) solves the PFC1 A^R y = b^R (m11 = 1/gamma)."""
        n = self.n
        mu, ps, _ = split(x, n)
        N = N_matrix(self.mesh, ps)
        Kp = K_plus(self.mesh, ps, self.psi_min)
        Fm = F_mu(self.mesh, mu)

        def stage_solve(rhs, i, xi):
            bR = rhs.copy()
            bR[n:2 * n] *= tau
            return linear_solve(N, Kp, Fm, tau, bR, i)

        return ros3pw_step(x, tau, self.F, self.mass_apply, stage_solve)


def rosenbrock_run1(mesh, M, K, x0, r, tau, n_steps, solver="fgmres", replays=None, psi_min=PSI_MIN, **kw):
    """n_steps Ros3Pw steps of PFC1 from x0 ('fgmres': the method, 'dense': LU reference).

    The preconditioner's mobility mean M0 is taken from x0 (conserved by the scheme).
    """
    from .reference import dense_solve
    from .solve import solve_stage

    prob = PFC1Problem(mesh, M, K, r, psi_min)
    n = M.shape[0]
    m0 = mobility_mean(M, x0[n:2 * n], psi_min)
    m11 = 1.0 / ROS3PW_GAMMA
    infos = []

    def lin(N, Kp, Fm, tau_, bR, i):
        if solver == "dense":
            infos.append(None)
            return dense_solve(AR1_sparse(M, K, N, Kp, Fm, r, tau_, m11), bR)
        rp = None if replays is None else replays[len(infos)]
        y, info = solve_stage(M, K, N, r, tau_, m11, bR, replay=rp, Kp=Kp, Fm=Fm, m0=m0, **kw)
        infos.append(info)
        return y

    x = x0.copy()
    for _ in range(n_steps):
        x, _, _ = prob.step(x, tau, lin)
    return x, infos
