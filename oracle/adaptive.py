"""Adaptive Ros3Pw time stepping (oracle, test infrastructure).

The scheme's embedded solution x_hat = x_k + sum mhat_j y_j (eq. rosenbrock-update,
weights mhat of Table rosenbrock_scheme) is of order 2; the difference to the
order-3 solution estimates the local error (Section 3.1 defers step-size
control to the literature).  Reading taken here, the elementary controller:

    sc_i  = atol + rtol * max(|psi_k,i|, |psi_{k+1},i|)            (psi block)
    err   = sqrt( mean( ((psi_{k+1} - psi_hat)_i / sc_i)^2 ) )
    accept the step if err <= 1
    tau  <- tau * min(facmax, max(facmin, safety * err^(-1/3)))

with safety 0.9, facmin 0.2, facmax 5 and the exponent 1/(p_hat + 1), p_hat = 2.
The error is measured on psi, the differential component of the DAE.

Pinned by tests/test_oracle_adaptive.py: the embedded solution converges with
order 2 and ||x - x_hat|| with order 3 per step on a nonlinear ODE; an
adaptive PFC run reaches its end time, respects the tolerance against a
fine fixed-step reference, and rejects steps that are too large.
"""
from __future__ import annotations

import math

import numpy as np

SAFETY, FACMIN, FACMAX = 0.9, 0.2, 5.0


def error_norm(psi_old, psi_new, psi_hat, rtol, atol):
    sc = atol + rtol * np.maximum(np.abs(psi_old), np.abs(psi_new))
    return float(math.sqrt(np.mean(((psi_new - psi_hat) / sc) ** 2)))


def next_tau(tau, err):
    if err == 0.0:
        return tau * FACMAX
    return tau * min(FACMAX, max(FACMIN, SAFETY * err ** (-1.0 / 3.0)))


def rosenbrock_adaptive(prob, x0, tau0, t_end, rtol, atol, linear_solve, max_attempts=10000):
    """Adaptive Ros3Pw run of a PFCProblem from t = 0 to t_end.

    linear_solve as in PFCProblem.step.  Returns (x, accepted_taus, n_rejected).
    """
    n = prob.n
    t, tau, x = 0.0, tau0, x0.copy()
    taus, rejected = [], 0
    for _ in range(max_attempts):
        if t >= t_end * (1 - 1e-14):
            break
        h = min(tau, t_end - t)
        x_new, x_hat, _ = prob.step(x, h, linear_solve)
        err = error_norm(x[n:2 * n], x_new[n:2 * n], x_hat[n:2 * n], rtol, atol)
        if err <= 1.0:
            t += h
            x = x_new
            taus.append(h)
        else:
            rejected += 1
        tau = next_tau(h, err)
    return x, taus, rejected
