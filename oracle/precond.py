"""The block preconditioner P_CH and its five-step apply (oracle, test infrastructure).

Section 4: for the reduced 2x2 system, P(S) = L U(S) with
    L    = [[M, 0], [tau K, M + delta K]],  delta = sqrt(tau)
    U(S) = [[I, delta^{-1} M^{-1} (M - S)], [0, M^{-1} S]]
so that (eq. preconditioner_S) P(S) = [[M, delta^{-1}(M - S)], [tau K, delta K + S]].
The Cahn-Hilliard approximation of the Schur complement is
    S_CH = (M + sqrt(delta) K) M^{-1} (M + sqrt(delta) K)   (eq. cahn_hilliard_precon_2)
and P_CH = P(S_CH).  The third block row of the 3x3 system is handled by
M x2 = b2 - K x1, giving the 3x3 preconditioner [[P_CH, 0], [[0, K], M]].

Apply of P_CH^{-1} to (b0, b1, b2):
    (1)   M y0 = b0
    (2)   (M + delta K) y1 = b1 - tau K y0
    (3.1) (M + sqrt(delta) K) z  = M y1
    (3.2) (M + sqrt(delta) K) x1 = M z
    (4)   x0 = y0 + (y1 - x1)/delta
    (5)   M x2 = b2 - K x1
Readings (listed in the design notes): step (2) uses y0 on the right (the
printed y1 contradicts the factorisation L); the (0,1) block of P_CH is
-(2/sqrt(delta)) K - B, which is what P(S_CH) gives and what reproduces the
printed spectrum of A P_CH^{-1}; the printed -2 sqrt(delta) K - B does not.
`tau` here is the coefficient of K in block row 1 after that row has been
divided by its mass coefficient m11 (tau/m11 = gamma tau for Rosenbrock).

Pinned by tests/test_oracle_precond.py: the five steps with exact inner
solves equal solve(P3, b) for the dense P3 built from P(S_CH); L U(S) = P(S)
for S = S_CH and the exact S; the spectrum of A P_CH^{-1} on a constant
state equals the closed form derived from the symbols (two unit eigenvalues
per mode and (1 + tau(c mu - 2 mu^2 + mu^3)) / ((1 + delta mu)(1 + sqrt(delta) mu)^2));
Lemma 2's interval for eig(S_CH^{-1} S).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla

from .krylov import pcg

STEP_NAMES = ("1:M", "2:M+dK", "3.1:M+sqrt(d)K", "3.2:M+sqrt(d)K", "5:M")


def schur_D_sparse(M, K, tau):
    """S_D = M - 2 delta K + delta K M_D^{-1} K with M_D = diag(M) (Section 4.1)."""
    import scipy.sparse as sp
    d = math.sqrt(tau)
    return (M - 2.0 * d * K + d * (K @ sp.diags(1.0 / M.diagonal()) @ K)).tocsr()


class InnerSolvers:
    """Inner solves of the five preconditioner steps.

    mode 'exact': sparse LU of M, M + delta K, M + sqrt(delta) K.
    mode 'pcg'  : Jacobi PCG, tol relative (1e-3 in the paper), maxit cap;
                  records the counts of every apply; with `replay_counts`
                  (list of 5-lists) runs exactly those counts; with
                  `fixed_counts` (one 5-list) every apply runs those counts
                  where they are positive.
    """

    def __init__(self, M, K, tau, mode="pcg", tol=1e-3, maxit=500, replay_counts=None, schur="CH", sd_iters=20,
                 fixed_counts=None):
        self.M, self.K = M, K
        self.tau = tau
        self.delta = math.sqrt(tau)
        self.sdelta = math.sqrt(self.delta)
        self.schur = schur
        self.sd_iters = sd_iters
        self.mats = [M, (M + self.delta * K).tocsr(), (M + self.sdelta * K).tocsr()]
        if schur == "D":
            self.mats.append(schur_D_sparse(M, K, tau))
        self.mode = mode
        self.tol, self.maxit = tol, maxit
        self.replay = replay_counts
        self.fixed_counts = fixed_counts  # per step: a fixed iteration count, or 0 for the tolerance
        self.counts: list[list[int]] = []
        self._cur: list[int] = []
        if mode == "exact":
            self.lu = [spla.splu(A.tocsc()) for A in self.mats]
        else:
            self.dinv = [1.0 / A.diagonal() for A in self.mats]

    def begin(self):
        self._cur = []

    def end(self):
        self.counts.append(self._cur)

    def solve(self, which_mat, step, rhs):
        if self.mode == "exact":
            self._cur.append(0)
            return self.lu[which_mat].solve(rhs)
        A = self.mats[which_mat]
        fixed = None
        if which_mat == 3:
            fixed = self.sd_iters  # Table inner_solvers: S_D is solved with a fixed iteration count
        if self.fixed_counts is not None and self.fixed_counts[step] > 0:
            fixed = self.fixed_counts[step]
        if self.replay is not None:
            fixed = self.replay[len(self.counts)][step]
        x, it = pcg(lambda v: A @ v, rhs, self.dinv[which_mat], self.tol, self.maxit, fixed)
        self._cur.append(it)
        return x


def pch_apply(inner: InnerSolvers, v):
    """z = P_CH^{-1} v for the 3x3 block vector v = (b0, b1, b2)."""
    M, K = inner.M, inner.K
    n = M.shape[0]
    b0, b1, b2 = v[:n], v[n:2 * n], v[2 * n:]
    tau, delta = inner.tau, inner.delta
    inner.begin()
    y0 = inner.solve(0, 0, b0)                          # (1)
    y1 = inner.solve(1, 1, b1 - tau * (K @ y0))         # (2)
    if inner.schur == "D":                              # (3) with S_D
        x1 = inner.solve(3, 2, M @ y1)
        inner._cur.append(0)
    else:
        z = inner.solve(2, 2, M @ y1)                   # (3.1)
        x1 = inner.solve(2, 3, M @ z)                   # (3.2)
    x0 = y0 + (y1 - x1) / delta                         # (4)
    x2 = inner.solve(0, 4, b2 - K @ x1)                 # (5)
    inner.end()
    return np.concatenate([x0, x1, x2])


def dense_blocks(M, K):
    Md = M.toarray()
    Kd = K.toarray()
    B = Kd @ np.linalg.solve(Md, Kd)
    return Md, Kd, B


def schur_exact(Md, Kd, B, tau):
    d = math.sqrt(tau)
    return Md - 2.0 * d * Kd + d * B


def schur_ch(Md, Kd, B, tau):
    d = math.sqrt(tau)
    return Md + 2.0 * math.sqrt(d) * Kd + d * B


def P_of_S(Md, Kd, tau, S):
    """Eq. preconditioner_S: [[M, delta^{-1}(M - S)], [tau K, delta K + S]]."""
    d = math.sqrt(tau)
    return np.block([[Md, (Md - S) / d], [tau * Kd, d * Kd + S]])


def L_U_of_S(Md, Kd, tau, S):
    d = math.sqrt(tau)
    n = Md.shape[0]
    I = np.eye(n)
    Z = np.zeros((n, n))
    L = np.block([[Md, Z], [tau * Kd, Md + d * Kd]])
    Minv = np.linalg.inv(Md)
    U = np.block([[I, Minv @ (Md - S) / d], [Z, Minv @ S]])
    return L, U


def schur_D_dense(Md, Kd, tau):
    d = math.sqrt(tau)
    return Md - 2.0 * d * Kd + d * Kd @ np.diag(1.0 / np.diag(Md)) @ Kd


def P3_dense(M, K, tau, schur="CH"):
    """3x3 block preconditioner [[P(S), 0], [[0, K], M]] (S = S_CH or S_D) as a dense matrix."""
    Md, Kd, B = dense_blocks(M, K)
    n = Md.shape[0]
    S = schur_ch(Md, Kd, B, tau) if schur == "CH" else schur_D_dense(Md, Kd, tau)
    P2 = P_of_S(Md, Kd, tau, S)
    P3 = np.zeros((3 * n, 3 * n))
    P3[:2 * n, :2 * n] = P2
    P3[2 * n:, n:2 * n] = Kd
    P3[2 * n:, 2 * n:] = Md
    return P3
