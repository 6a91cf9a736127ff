"""Algorithmic HBM bytes of the stage solve, from its iteration counts.

Per-unit byte counts (n rows, z stored entries per row, w bytes per inner
value: 8 in float64, 4 in float32; indices 4 bytes; outer vectors float64):
  PCG iteration        n [z (w + 4) + 4 + 10 w]   one SpMV with its index stream,
                       vectors p, q, q, x (r/w), r (r/w), D^{-1}, p (r/w)
  PCG set-up           n [z (w + 4) + 4 + 6 w]    right-hand-side SpMV, r, x, D^{-1}
  block SpMV of A^R    n [z (3*8 + 4) + 4 + 48]   M, K, N values, one index stream,
                       z_j in, w out (three blocks)
  MGS at step j        n [72 (j + 1) + 48]        j+1 passes over w and v_i, plus V/Z writes
  cycle end            n [24 (k + 2)] + block SpMV + 48 n   x += Z y, true residual
PFC1 (mobility model): the block SpMV also streams K_+ and F values,
n [z (5*8 + 4) + 4 + 48].  S_D variant: its fixed-count PCG iterations run on
the second-ring pattern with z_sd entries per row.  Rows of different length
(P2 meshes) enter through the mean z = nnz / n, which gives the exact total.
These count every array once per use (no cache reuse), which is what the
method must move; they are the numerator of the roofline fraction.
"""
from __future__ import annotations


def pcg_iter_bytes(n, z, w):
    return n * (z * (w + 4) + 4 + 10 * w)


def solve_bytes(n, z, w, info, restart=30, model=0, z_sd=None, sd_iters=20):
    """Algorithmic bytes of one stage solve from its info record."""
    outer = info["outer_iters"]
    inner = info["inner_total"]
    applies = info["inner_applies"]
    cycles = max(1, info["cycles"])
    if z_sd is None:
        b = inner * pcg_iter_bytes(n, z, w)
    else:
        sd = applies * sd_iters
        b = (inner - sd) * pcg_iter_bytes(n, z, w) + sd * pcg_iter_bytes(n, z_sd, w)
    setups = 5 if z_sd is None else 4   # S_D replaces the solves (3.1), (3.2) by one
    b += applies * setups * n * (z * (w + 4) + 4 + 6 * w)
    spmv = n * (z * (44 if model == 1 else 28) + 4 + 48)
    b += outer * spmv
    left = outer
    for c in range(cycles):
        k = min(restart, left)
        left -= k
        b += sum(n * (72 * (j + 1) + 48) for j in range(k))
        b += n * 24 * (k + 2) + spmv + 48 * n
    return b


def step_bytes(n, z, n_elem, dim, nloc=None, model=0):
    """N(psi) reassembly and three stage right-hand sides of one Rosenbrock step."""
    k = nloc or dim + 1
    reasm = n * z * 8 * (3 if model == 1 else 1) + n_elem * (k * 4 + 8) + n * 8 * (2 if model == 1 else 1)
    rhs = 3 * n * (z * 20 + 4 + 5 * 24)
    return reasm + rhs + 3 * n * 24 * 4
