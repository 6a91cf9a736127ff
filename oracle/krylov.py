"""Krylov solvers of the method (oracle, test infrastructure).

* pcg     Jacobi-preconditioned conjugate gradients, the inner solver of every
          preconditioner step (Table inner_solvers: PCG, 'diag', relative
          tolerance 1e-3).  Reading taken: the tolerance is on the
          unpreconditioned residual, ||r||_2 <= tol ||rhs||_2, with x_0 = 0.
          A fixed-count mode replays a recorded iteration count.
* fgmres  flexible GMRES with restart m (30 in the paper), modified
          Gram-Schmidt and Givens rotations, right preconditioning
          A P^{-1} (P x) = b (Section 4; solver settings in Section 7).
          x_0 = 0; the iteration count is the number of Arnoldi steps.

Pinned by tests/test_oracle_solvers.py: PCG against a direct solve and the
CG error bound in the energy norm; FGMRES (with and without preconditioner)
against dense LU on small systems, against the FFT-exact solve, and the
Arnoldi relation A Z_k = V_{k+1} H_k.
"""
from __future__ import annotations

import math

import numpy as np


def pcg(apply_C, b, dinv, tol=1e-3, maxit=500, fixed=None):
    """Solve C x = b (C SPD) by PCG with the Jacobi preconditioner D^{-1} = dinv.

    Stops when ||r||_2 <= tol ||b||_2 (fixed is None) or after exactly `fixed`
    iterations.  b = 0 returns x = 0 with zero iterations.  Returns (x, iters).
    """
    x = np.zeros_like(b)
    bn2 = float(b @ b)
    if bn2 == 0.0:
        return x, 0
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = float(r @ z)
    it = 0
    limit = maxit if fixed is None else fixed
    while it < limit:
        q = apply_C(p)
        pq = float(p @ q)
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        rr = float(r @ r)
        z = dinv * r
        rz_new = float(r @ z)
        if fixed is None and rr <= tol * tol * bn2:
            break
        if rz_new == 0.0:
            break
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, it


class Schedule:
    """Recorded iteration structure of one FGMRES solve: cycle lengths and, per
    preconditioner apply, the five inner PCG counts."""

    def __init__(self):
        self.cycles: list[int] = []
        self.inner: list[list[int]] = []


def fgmres(apply_A, apply_P, b, tol=1e-8, restart=30, max_steps=1000,
           true_residual=None, est_scale=1.0, replay: Schedule | None = None,
           breakdown_tol=1e-14, record=None):
    """Right-preconditioned FGMRES(restart) with modified Gram-Schmidt, x_0 = 0.

    A cycle ends when the Givens estimate |g_{j+1}| <= tol*||b||*est_scale,
    on happy breakdown (h_{j+1,j} <= breakdown_tol * ||w|| before
    orthogonalisation), after `restart` steps or at max_steps.  Then
    x += Z y, and the true relative residual (true_residual(x), default
    ||b - A x|| / ||b||) decides convergence; otherwise the next cycle
    starts from r = b - A x.  With `replay`, cycle lengths follow the record
    and no early stop happens.  With `record` (a list), the first cycle's
    V, Z and unrotated Hessenberg matrix are appended to it.

    Returns (x, info) with info = dict(steps, cycles, rel_res, est, converged).
    """
    nb = float(np.linalg.norm(b))
    x = np.zeros_like(b)
    info = dict(steps=0, cycles=[], rel_res=0.0, est=0.0, converged=True)
    if nb == 0.0:
        return x, info
    m = restart
    if true_residual is None:
        def true_residual(xx):
            return float(np.linalg.norm(b - apply_A(xx))) / nb
    r = b.copy()
    beta = nb
    total = 0
    cyc = 0
    est_thresh = tol * nb * est_scale
    while True:
        cyc_len = None
        if replay is not None:
            if cyc >= len(replay.cycles):
                break
            cyc_len = replay.cycles[cyc]
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        Hraw = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        for j in range(m):
            if cyc_len is not None and j >= cyc_len:
                break
            z = apply_P(V[j])
            Z.append(z)
            w = apply_A(z)
            w0 = float(np.linalg.norm(w))
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = float(w @ V[i])
                w = w - H[i, j] * V[i]
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            if record is not None and cyc == 0:
                Hraw[:j + 2, j] = H[:j + 2, j]
            for i in range(j):  # earlier rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = math.hypot(H[j, j], H[j + 1, j])
            if d == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k = j + 1
            breakdown = hn <= breakdown_tol * w0
            if not breakdown:
                V.append(w / hn)
            if cyc_len is None:
                if abs(g[j + 1]) <= est_thresh or breakdown or total >= max_steps:
                    break
            elif breakdown and j + 1 < cyc_len:
                raise RuntimeError("breakdown during replay")
        # back substitution H[:k,:k] y = g[:k]
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        for i in range(k):
            x += y[i] * Z[i]
        if record is not None and cyc == 0:
            record.append((list(V), list(Z), Hraw[:k + 1, :k].copy()))
        info["cycles"].append(k)
        info["est"] = abs(g[k]) / nb
        cyc += 1
        rel = true_residual(x)
        info["rel_res"] = rel
        if replay is None:
            if rel <= tol:
                info["converged"] = True
                break
            if total >= max_steps:
                info["converged"] = False
                break
        r = b - apply_A(x)
        beta = float(np.linalg.norm(r))
        if beta == 0.0:
            break
    info["steps"] = total
    if replay is not None:
        info["converged"] = info["rel_res"] <= tol
    return x, info
