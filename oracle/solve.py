"""Stage solve and Rosenbrock run as the method specifies them (oracle, test infrastructure).

solve_stage: A^R y = b by right-preconditioned FGMRES(restart) with the P_CH
preconditioner and Jacobi-PCG inner solves (Sections 4 and 6, Table
inner_solvers).  Reading for the mass coefficient m11 of block row 1 (1/gamma
for Rosenbrock stages): the preconditioner is derived for m11 = 1, so block
row 1 of the system and of b is divided by m11 before FGMRES sees it; P_CH is
then built with tau_s = tau/m11.  The solution is unchanged.  Convergence is
judged on the true relative residual of the system as given,
||b - A^R y||_2 / ||b||_2; the Givens estimate of the scaled system is
compared with tol*||b||/max(1, m11), which bounds the unscaled residual.
gamma_mode="literal" takes the other reading of Section 4 (the preconditioner
is used unchanged): FGMRES sees the unscaled system and P_CH is built with
tau, and the estimate is compared with tol*||b||; both readings coincide
for m11 = 1.

inner_fixed (five counts, 0 = run to the tolerance) fixes the iteration count
of the corresponding preconditioner step in every application.

PFC1 (Kp, Fm given, oracle.mobility): the operator is the PFC1 stage matrix
and P_CH is built for the time step m0 * tau_s (constant-mobility
approximation K_+ ~ M0 K of Section 4); with Kp = K, Fm = 0, m0 = 1 this is
the PFC2 solve.

Pinned through its parts (precond, krylov, reference) and by agreement with
dense LU and the FFT-exact solve in tests/test_oracle_solvers.py.
"""
from __future__ import annotations

import numpy as np

from .krylov import Schedule, fgmres
from .pfc import PFCProblem, apply_AR
from .precond import InnerSolvers, pch_apply


def solve_stage(M, K, N, r, tau, m11, b, tol=1e-8, restart=30, max_steps=1000,
                inner_mode="pcg", inner_tol=1e-3, inner_maxit=500, replay: Schedule | None = None, schur="CH",
                Kp=None, Fm=None, m0=1.0, gamma_mode="scale_row", inner_fixed=None):
    n = M.shape[0]
    if gamma_mode not in ("scale_row", "literal"):
        raise ValueError(gamma_mode)
    scale = gamma_mode == "scale_row"
    tau_s = tau / m11 if scale else tau
    b_s = b.copy()
    if scale:
        b_s[n:2 * n] /= m11
    nb = float(np.linalg.norm(b))
    nbs = float(np.linalg.norm(b_s))
    inner = InnerSolvers(M, K, m0 * tau_s, mode=inner_mode, tol=inner_tol, maxit=inner_maxit,
                         replay_counts=None if replay is None else replay.inner, schur=schur,
                         fixed_counts=inner_fixed)
    if Kp is None:
        def op(t, s, y):
            return apply_AR(M, K, N, r, t, s, y)
    else:
        from .mobility import apply_AR1

        def op(t, s, y):
            return apply_AR1(M, K, N, Kp, Fm, r, t, s, y)

    def apply_As(y):
        return op(tau_s, 1.0 if scale else m11, y)

    def true_res(y):
        return float(np.linalg.norm(b - op(tau, m11, y))) / nb

    est_scale = ((nb / nbs) / (max(1.0, m11) if scale else 1.0)) if nbs > 0 else 1.0
    y, info = fgmres(apply_As, lambda v: pch_apply(inner, v), b_s, tol=tol, restart=restart,
                     max_steps=max_steps, true_residual=true_res, est_scale=est_scale, replay=replay)
    sched = Schedule()
    sched.cycles = list(info["cycles"])
    sched.inner = [list(c) for c in inner.counts]
    info["schedule"] = sched
    info["inner_total"] = int(sum(sum(c) for c in inner.counts))
    return y, info


def rosenbrock_run(mesh, M, K, x0, r, tau, n_steps, solver="fgmres", replays=None, **kw):
    """n_steps Ros3Pw steps from x0.  solver 'fgmres' (the method) or 'dense' (LU reference).

    Returns (x, infos) with one info per stage solve; with `replays` (list of
    Schedules, one per stage solve in order) every FGMRES solve replays.
    """
    from .pfc import AR_sparse, ROS3PW_GAMMA
    from .reference import dense_solve

    prob = PFCProblem(mesh, M, K, r)
    infos = []
    m11 = 1.0 / ROS3PW_GAMMA

    def lin(N, tau_, bR, i):
        if solver == "dense":
            infos.append(None)
            return dense_solve(AR_sparse(M, K, N, r, tau_, m11), bR)
        rp = None if replays is None else replays[len(infos)]
        y, info = solve_stage(M, K, N, r, tau_, m11, bR, replay=rp, **kw)
        infos.append(info)
        return y

    x = x0.copy()
    for _ in range(n_steps):
        x, _, _ = prob.step(x, tau, lin)
    return x, infos
