"""The PFC2 Rosenbrock stage system (oracle, test infrastructure).

Model: the H^{-1} gradient flow of the Swift-Hohenberg energy, split into
second-order equations for x = (mu, psi, omega) (Section 2, PFC2: mobility
psi^+ = 1, hence K_+ = K and F(mu) = 0 in the stage matrix).

Weak-form operator (Section 3.1, linear form of the operator F):
    F0(x) = -M mu + (1+r) M psi - 2 K psi - K omega + g(psi)
    F1(x) = -K mu
    F2(x) = -M omega - K psi
Stage matrix (eq. rosenbrock_matrix with K_+ = K, F = 0):
    A^R = [[ M,   -(1+r) M + 2K + N(psi_k),  K ],
           [ tau K,         m11 M,           0 ],
           [ 0,               K,             M ]]
with m11 = 1/gamma for the Rosenbrock stages and m11 = 1 for the linearised
Euler system (eq. systemmatrix).  The stage right-hand side is the weak form
of F(x_i) + sum_j (c_ij/tau) Mbb y_j with its second block multiplied by tau
(Section 3.1, sentence after eq. rosenbrock_matrix), Mbb = diag(0, M, 0):
    b0 = F0(x_i),  b1 = tau F1(x_i) + sum_j c_ij M y_j^psi,  b2 = F2(x_i).

Ros3Pw coefficients: Table rosenbrock_scheme.  a_22, a_33 and c_11, c_22, c_33
in that table are stage-time nodes and diagonal sums of the standard form;
they do not enter the autonomous stage equations, and a_32 = 0.

Pinned by tests/test_oracle_pfc.py:
  * the generic step applied to y' = lambda y reproduces exp(z) to O(z^4)
    (third order) and R(-inf) = 1 - sqrt(3)
  * PFC run on a tiny mesh with dense stage solves converges with order 3
  * conservation of int psi_h from step to step (K annihilates constants)
  * A^R equals the Jacobian of the discrete operator (finite differences)
  * consistent initial values zero blocks 0 and 2 of F
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assembly import N_matrix, load_psi3

# Table rosenbrock_scheme (Ros3Pw in the modified form of eq. rosenbrock).
ROS3PW_GAMMA = 0.78867513459481287
ROS3PW_A = {(2, 1): 2.0, (3, 1): 0.633974596215561, (3, 2): 0.0}
ROS3PW_C = {(2, 1): -2.53589838486225, (3, 1): -1.62740473580836, (3, 2): -0.274519052838329}
ROS3PW_M = (1.63397459621556, 0.294228634059948, 1.07179676972449)
ROS3PW_MHAT = (1.99444650053487, 0.654700538379252, 1.07179676972449)


def split(x: np.ndarray, n: int):
    return x[:n], x[n:2 * n], x[2 * n:]


def apply_AR(M, K, N, r, tau, m11, y):
    """A^R y for y = (mu, psi, omega) stacked [3n]."""
    n = M.shape[0]
    mu, ps, om = split(y, n)
    out = np.empty(3 * n)
    out[:n] = M @ mu - (1.0 + r) * (M @ ps) + 2.0 * (K @ ps) + N @ ps + K @ om
    out[n:2 * n] = tau * (K @ mu) + m11 * (M @ ps)
    out[2 * n:] = K @ ps + M @ om
    return out


def AR_sparse(M, K, N, r, tau, m11):
    """A^R as one sparse 3n x 3n matrix (for direct solves on small meshes)."""
    Z = None
    return sp.bmat([[M, -(1.0 + r) * M + 2.0 * K + N, K],
                    [tau * K, m11 * M, Z],
                    [Z, K, M]], format="csr")


def F_weak(mesh, M, K, r, x):
    """The vector of the weak-form operator F(x)[theta] over the P1 basis."""
    n = M.shape[0]
    mu, ps, om = split(x, n)
    out = np.empty(3 * n)
    out[:n] = -(M @ mu) + (1.0 + r) * (M @ ps) - 2.0 * (K @ ps) - K @ om + load_psi3(mesh, ps)
    out[n:2 * n] = -(K @ mu)
    out[2 * n:] = -(M @ om) - K @ ps
    return out


def stage_rhs_R(mesh, M, K, r, tau, x_i, y_prev_psi, c_row):
    """b_i^R: F(x_i) with block 1 multiplied by tau, plus sum_j c_ij M y_j^psi on block 1.

    y_prev_psi: list of psi-blocks of earlier stage solutions y_1..y_{i-1};
    c_row: the matching coefficients c_i1..c_i,i-1.
    """
    n = M.shape[0]
    b = F_weak(mesh, M, K, r, x_i)
    b[n:2 * n] *= tau
    for c, yp in zip(c_row, y_prev_psi):
        b[n:2 * n] += c * (M @ yp)
    return b


def consistent_init(mesh, M, K, r, psi0):
    """mu_0, omega_0 that zero blocks 0 and 2 of F at t = 0.

    M omega_0 = -K psi_0;  M mu_0 = (1+r) M psi_0 - 2 K psi_0 - K omega_0 + g(psi_0).
    The two mass solves are taken to rounding level (Jacobi CG, relative
    residual 1e-15; M is SPD with a mesh-independent condition number), which
    agrees with a sparse LU solve to rounding (pinned in the tests).
    """
    from .krylov import pcg

    dinv = 1.0 / M.diagonal()

    def msolve(rhs):
        return pcg(lambda v: M @ v, rhs, dinv, tol=1e-15, maxit=1000)[0]

    om = msolve(-(K @ psi0))
    mu = msolve((1.0 + r) * (M @ psi0) - 2.0 * (K @ psi0) - K @ om + load_psi3(mesh, psi0))
    return np.concatenate([mu, psi0, om])


def ros3pw_step(x, tau, F, mass_apply, stage_solve, coeffs=None):
    """One step of the Rosenbrock scheme in modified form (eqs. rosenbrock, rosenbrock-update).

    stage i:   (1/(tau gamma)) Mbb y_i - J y_i = F(x_i) + sum_{j<i} (c_ij/tau) Mbb y_j
               x_i = x + sum_{j<i} a_ij y_j
    update:    x_new = x + sum m_j y_j,   x_hat = x + sum mhat_j y_j
    `stage_solve(rhs, i)` must solve ((1/(tau gamma)) Mbb - J(x)) y = rhs.
    Returns (x_new, x_hat, [y_1, y_2, y_3]).
    """
    a, c, m, mh = (ROS3PW_A, ROS3PW_C, ROS3PW_M, ROS3PW_MHAT) if coeffs is None else coeffs
    ys = []
    for i in (1, 2, 3):
        xi = x.copy()
        rhs_extra = 0.0
        for j in range(1, i):
            xi = xi + a[(i, j)] * ys[j - 1]
            rhs_extra = rhs_extra + (c[(i, j)] / tau) * mass_apply(ys[j - 1])
        rhs = F(xi) + rhs_extra
        ys.append(stage_solve(rhs, i, xi))
    x_new = x + sum(mj * yj for mj, yj in zip(m, ys))
    x_hat = x + sum(mj * yj for mj, yj in zip(mh, ys))
    return x_new, x_hat, ys


class PFCProblem:
    """A PFC2 instance on one mesh: M, K fixed, N(psi_k) rebuilt each step."""

    def __init__(self, mesh, M, K, r):
        self.mesh, self.M, self.K, self.r = mesh, M, K, r
        self.n = M.shape[0]

    def F(self, x):
        return F_weak(self.mesh, self.M, self.K, self.r, x)

    def mass_apply(self, y):
        n = self.n
        out = np.zeros(3 * n)
        out[n:2 * n] = self.M @ y[n:2 * n]
        return out

    def step(self, x, tau, linear_solve):
        """One Ros3Pw step.  linear_solve(N, tau, b_R, stage_index) solves A^R y = b^R with m11 = 1/gamma."""
        n = self.n
        N = N_matrix(self.mesh, x[n:2 * n])

        def stage_solve(rhs, i, xi):
            bR = rhs.copy()
            bR[n:2 * n] *= tau  # second block of the weak form times tau
            return linear_solve(N, tau, bR, i)

        return ros3pw_step(x, tau, self.F, self.mass_apply, stage_solve)
