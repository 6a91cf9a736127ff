"""Fourier analysis of the preconditioner (oracle, test infrastructure).

Symbols (Section 6) in terms of k2 = |k|^2, with the psibar stabilisation of
eq. A_mod (c = 3 psibar^2 + 1 + r):
    A    = [[1, -c + 2 k2, k2], [tau k2, 1, 0], [0, k2, 1]]
    A0   = 1 + tau (c k2 - 2 k2^2 + k2^3)                    (eq. A0_mod)
    P    = [[1, 2 k2 - k2^2, 0], [tau k2, 1 - delta k2 + delta k2^2, 0], [0, k2, 1]]
    P_CH = P(S_CH) with S_CH -> (1 + sqrt(delta) k2)^2 in eq. preconditioner_S:
           [[1, -(2/sqrt(delta)) k2 - k2^2, 0],
            [tau k2, 1 + (delta + 2 sqrt(delta)) k2 + delta k2^2, 0], [0, k2, 1]]
Critical time step (Lemma 3): tau* = 27 / (2 (sqrt(a) - 1)(sqrt(a) + 2)^2),
a = 1 - 3 r - 9 psibar^2, finite only when psibar^2 < -r/3.
Asymptotic convergence factor of a real interval [lo, hi], 0 < lo < hi
(eq. estimate_interval): rho = (sqrt(kappa) - 1)/(sqrt(kappa) + 1), kappa = hi/lo.

Pinned by tests/test_oracle_symbols.py: the printed tau* values; the
eigenvalues of A P^{-1} and A P_CH^{-1} computed numerically from these
matrices equal the printed closed-form sets (eqs. eigenvalues_B and
eigenvalues_B_ch); tau-natural = 1; the printed ranges of rho.
"""
from __future__ import annotations

import math

import numpy as np


def tau_star(r: float, psibar: float) -> float:
    a = 1.0 - 3.0 * r - 9.0 * psibar * psibar
    if a <= 1.0:
        return math.inf
    s = math.sqrt(a)
    return 27.0 / (2.0 * (s - 1.0) * (s + 2.0) ** 2)


def sym_A(k2, tau, r, psibar):
    c = 3.0 * psibar * psibar + 1.0 + r
    return np.array([[1.0, -c + 2.0 * k2, k2], [tau * k2, 1.0, 0.0], [0.0, k2, 1.0]])


def sym_A0(k2, tau, r, psibar):
    c = 3.0 * psibar * psibar + 1.0 + r
    return 1.0 + tau * (c * k2 - 2.0 * k2 ** 2 + k2 ** 3)


def sym_P(k2, tau):
    d = math.sqrt(tau)
    return np.array([[1.0, 2.0 * k2 - k2 ** 2, 0.0], [tau * k2, 1.0 - d * k2 + d * k2 ** 2, 0.0], [0.0, k2, 1.0]])


def sym_PCH(k2, tau):
    d = math.sqrt(tau)
    sd = math.sqrt(d)
    return np.array([[1.0, -(2.0 / sd) * k2 - k2 ** 2, 0.0],
                     [tau * k2, 1.0 + (d + 2.0 * sd) * k2 + d * k2 ** 2, 0.0],
                     [0.0, k2, 1.0]])


def eig_printed_Q(k2, tau, r, psibar):
    """Third eigenvalue of eq. eigenvalues_B as printed."""
    c = 3.0 * psibar * psibar + 1.0 + r
    st = math.sqrt(tau)
    return (tau * (k2 ** 3 - 2.0 * k2 ** 2 + c * k2) + 1.0) / (tau * k2 ** 3 + (st - 2.0 * tau) * k2 ** 2 - st * k2 + 1.0)


def eig_printed_QCH(k2, tau, r, psibar):
    """Third eigenvalue of eq. eigenvalues_B_ch as printed."""
    c = 3.0 * psibar * psibar + 1.0 + r
    return (tau * (k2 ** 3 - 2.0 * k2 ** 2 + c * k2) + 1.0) / (
        tau * k2 ** 3 + (math.sqrt(tau) + 2.0 * tau ** 0.75) * k2 ** 2 + (math.sqrt(tau) + 2.0 * tau ** 0.25) * k2 + 1.0)


def rho_interval(lo: float, hi: float) -> float:
    if lo <= 0.0:
        return 1.0
    s = math.sqrt(hi / lo)
    return (s - 1.0) / (s + 1.0)


def k2_grid(dim: int, kmax: float = 4.0, samples: int = 4001):
    """|k|^2 over [0, dim*kmax^2] (k_i in [0, kmax], Section 6.3)."""
    return np.linspace(0.0, dim * kmax * kmax, samples)


def rho_sigma(kind: str, tau: float, r: float, psibar: float, dim: int = 2, kmax: float = 4.0) -> float:
    """Spectral asymptotic convergence factor for 'A0', 'Q' or 'QCH'."""
    k2 = k2_grid(dim, kmax)
    if kind == "A0":
        vals = sym_A0(k2, tau, r, psibar)
    elif kind == "Q":
        vals = np.array([eig_printed_Q(x, tau, r, psibar) for x in k2])
        vals = np.concatenate([vals, [1.0]])
    elif kind == "QCH":
        vals = np.array([eig_printed_QCH(x, tau, r, psibar) for x in k2])
        vals = np.concatenate([vals, [1.0]])
    else:
        raise ValueError(kind)
    return rho_interval(float(vals.min()), float(vals.max()))
