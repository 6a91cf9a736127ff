"""The two-iterations-per-launch recurrences of the GPU's inner PCG, checked on the CPU (no GPU).

Jacobi PCG for C x = b is CG for T = D^{-1} C in the inner product <a, b> = a^T D b.  From the basis
B = [p, Tp, T^2 p, u, Tu] (u = D^{-1} r) the next two iterates are combinations of B whose coefficients
follow from G = B^T D B; the stopping tests ||r||^2 = u^T D^2 u from H = B'^T D^2 B' (B' = B[1:]).  The
closed forms below are the ones the solver's transition evaluates; they must give the standard
iteration's iterates and iteration counts.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import assembly


def pcg_standard(C, b, tol, lim):
    d = C.diagonal()
    x = np.zeros_like(b); r = b.copy(); u = r / d; p = u.copy(); rho = r @ u; bb = b @ b; it = 0
    while True:
        q = C @ p
        a = rho / (p @ q)
        x += a * p; r -= a * q; u = r / d; it += 1
        rr, rhon = r @ r, r @ u
        if it >= lim or rr <= tol * tol * bb or rhon == 0.0:
            return x, it
        p = u + (rhon / rho) * p
        rho = rhon


def pcg_two_per_step(C, b, tol, lim):
    d = C.diagonal()
    T = lambda v: (C @ v) / d
    x = np.zeros_like(b); bb = b @ b; it = 0
    u = b / d; p = u.copy()
    while True:
        B = [p, T(p), T(T(p)), u, T(u)]
        G = lambda i, j: B[i] @ (d * B[j])
        H = lambda i, j: B[i] @ (d * d * B[j])
        rho0 = G(3, 3); a0 = rho0 / G(0, 1)
        rho1 = G(3, 3) - 2 * a0 * G(1, 3) + a0 * a0 * G(1, 1)
        rr1 = H(3, 3) - 2 * a0 * H(1, 3) + a0 * a0 * H(1, 1)
        it += 1
        if it >= lim or rr1 <= tol * tol * bb or rho1 == 0.0:
            return x + a0 * B[0], it
        b0 = rho1 / rho0
        ptp = b0 * (b0 * G(0, 1) - a0 * G(0, 2) + G(0, 4)) - a0 * (b0 * G(1, 1) - a0 * G(1, 2) + G(1, 4)) + \
            (b0 * G(1, 3) - a0 * G(2, 3) + G(3, 4))
        a1 = rho1 / ptp
        c1, c2, c4 = -a0 - a1 * b0, a1 * a0, -a1

        def quad(M):
            return (c1 * c1 * M(1, 1) + c2 * c2 * M(2, 2) + M(3, 3) + c4 * c4 * M(4, 4) +
                    2 * (c1 * c2 * M(1, 2) + c1 * M(1, 3) + c1 * c4 * M(1, 4) + c2 * M(2, 3) + c2 * c4 * M(2, 4) +
                         c4 * M(3, 4)))
        rho2, rr2 = quad(G), quad(H)
        x = x + (a0 + a1 * b0) * B[0] - a1 * a0 * B[1] + a1 * B[3]
        it += 1
        if it >= lim or rr2 <= tol * tol * bb or rho2 == 0.0:
            return x, it
        b1 = rho2 / rho1
        pn = b1 * b0 * B[0] + (c1 - b1 * a0) * B[1] + c2 * B[2] + (1 + b1) * B[3] + c4 * B[4]
        un = c1 * B[1] + c2 * B[2] + B[3] + c4 * B[4]
        p, u = pn, un


def _operators():
    mesh = wl.make_mesh(2, 24, jitter=0.2, seed=3)
    M, K = assembly.mass_stiffness(mesh)
    delta = np.sqrt(0.5)
    rng = np.random.default_rng(4)
    A = sp.random(300, 300, density=0.02, random_state=5)
    R = (A + A.T + sp.diags(np.full(300, 6.0))).tocsr()
    return [("M", M.tocsr()), ("M + delta K", (M + delta * K).tocsr()), ("M + sqrt(delta) K", (M + np.sqrt(delta) * K).tocsr()),
            ("random SPD", R)], rng


@pytest.mark.parametrize("tol,lim", [(1e-3, 500), (1e-8, 500), (1e-3, 1), (1e-3, 2), (1e-3, 3), (1e-12, 7)])
def test_two_iterations_per_step_match_standard_pcg(tol, lim):
    ops, rng = _operators()
    for name, C in ops:
        b = rng.normal(size=C.shape[0])
        xs, its = pcg_standard(C, b, tol, lim)
        x2, it2 = pcg_two_per_step(C, b, tol, lim)
        assert it2 == its, (name, it2, its)
        assert np.linalg.norm(x2 - xs) <= 1e-12 * np.linalg.norm(xs), name


def test_odd_and_even_counts_end_in_the_right_substep():
    ops, rng = _operators()
    C = ops[1][1]
    b = rng.normal(size=C.shape[0])
    for lim in range(1, 9):
        xs, its = pcg_standard(C, b, 1e-14, lim)
        x2, it2 = pcg_two_per_step(C, b, 1e-14, lim)
        assert its == it2 == lim
        assert np.linalg.norm(x2 - xs) <= 1e-12 * np.linalg.norm(xs)
