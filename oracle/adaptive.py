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
The error is measured on psi, the differential component of the DAE.  Two
safeguards of the textbook controller (Hairer, Norsett, Wanner, Solving ODEs I,
Sec. II.4): the step that follows a rejection may not grow (facmax = 1 there),
and a step whose linear solves miss their tolerance (the linear_solve raises
LinearSolveFailed) is rejected without an error estimate and retried with
tau * facmin.

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


class LinearSolveFailed(Exception):
    """Raised by a linear_solve whose iteration stopped short of its tolerance."""


def next_tau(tau, err, facmax=FACMAX):
    if err == 0.0:
        return tau * facmax
    return tau * min(facmax, max(FACMIN, SAFETY * err ** (-1.0 / 3.0)))


def rosenbrock_adaptive(prob, x0, tau0, t_end, rtol, atol, linear_solve, max_attempts=10000, log=None):
    """Adaptive Ros3Pw run of a PFCProblem from t = 0 to t_end.

    linear_solve as in PFCProblem.step; it may raise LinearSolveFailed.  If log
    is a list, (tau, outcome) of every attempt is appended to it, outcome being
    "accepted", "rejected" (error estimate above 1) or "failed" (linear solve).
    Returns (x, accepted_taus, n_rejected), n_rejected counting both kinds.
    """
    n = prob.n
    t, tau, x = 0.0, tau0, x0.copy()
    taus, rejected, after_reject = [], 0, False
    for _ in range(max_attempts):
        if t >= t_end * (1 - 1e-14):
            break
        h = min(tau, t_end - t)
        try:
            x_new, x_hat, _ = prob.step(x, h, linear_solve)
        except LinearSolveFailed:
            rejected += 1
            after_reject = True
            tau = h * FACMIN
            if log is not None:
                log.append((h, "failed"))
            continue
        err = error_norm(x[n:2 * n], x_new[n:2 * n], x_hat[n:2 * n], rtol, atol)
        if err <= 1.0:
            t += h
            x = x_new
            taus.append(h)
            tau = next_tau(h, err, 1.0 if after_reject else FACMAX)
            after_reject = False
        else:
            rejected += 1
            tau = next_tau(h, err)
            after_reject = True
        if log is not None:
            log.append((h, "accepted" if err <= 1.0 else "rejected"))
    return x, taus, rejected
