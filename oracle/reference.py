"""Reference solves of the stage system (oracle, test infrastructure).

* dense_solve   LU factorisation of the assembled 3n x 3n A^R (small meshes).
* fft_exact     exact solve on translation-invariant periodic meshes with a
                spatially constant psi_k: M, K and N = -3 c^2 M are then
                (block-)circulant over the grid, so each Fourier mode
                decouples into a 3x3 complex system.  The stencils are read
                from row 0 of the assembled matrices (the assembly itself is
                pinned separately), the modes are solved in closed batch form
                and transformed back.  Works at any grid size.

Pinned by tests/test_oracle_solvers.py: fft_exact against dense_solve on
small grids in 2D and 3D; the 2D unjittered stencil against its closed form.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def dense_solve(A, b):
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    return np.linalg.solve(Ad, b)


def _stencil_symbol(A, shape):
    """Fourier symbol of a translation-invariant periodic operator from its row 0."""
    row = A.getrow(0)
    ker = np.zeros(shape)
    dim = len(shape)
    for j, v in zip(row.indices, row.data):
        if dim == 2:
            N = shape[0]
            pos = (j % N, j // N)
        else:
            N = shape[0]
            pos = (j % N, (j // N) % N, j // (N * N))
        ker[pos] += v
    # (A x)_p = sum_o A[0,o] x_{p+o}; symmetric stencils make this a convolution
    sym = np.fft.fftn(ker)
    return sym.real, np.abs(sym.imag).max()


def fft_exact(mesh, M, K, r, tau, m11, psi_const, b):
    """Exact solution of A^R y = b for psi_k == psi_const on a structured periodic mesh."""
    N = mesh.N
    shape = (N,) * mesh.dim
    n = mesh.n
    m_hat, im1 = _stencil_symbol(M, shape)
    k_hat, im2 = _stencil_symbol(K, shape)
    if max(im1, im2) > 1e-10 * max(np.abs(m_hat).max(), np.abs(k_hat).max()):
        raise ValueError("stencil not symmetric: mesh is not translation invariant")
    ncoef = -3.0 * psi_const * psi_const  # N = ncoef * M
    A = np.zeros(m_hat.shape + (3, 3), dtype=np.complex128)
    A[..., 0, 0] = m_hat
    A[..., 0, 1] = -(1.0 + r) * m_hat + 2.0 * k_hat + ncoef * m_hat
    A[..., 0, 2] = k_hat
    A[..., 1, 0] = tau * k_hat
    A[..., 1, 1] = m11 * m_hat
    A[..., 2, 1] = k_hat
    A[..., 2, 2] = m_hat

    def fwd(v):
        return np.fft.fftn(v.reshape(shape[::-1]).T)  # node index i + N j (+ N^2 k) -> array [i, j(, k)]

    def inv(V):
        return np.fft.ifftn(V).T.reshape(-1).real

    B = np.stack([fwd(b[:n]), fwd(b[n:2 * n]), fwd(b[2 * n:])], axis=-1)
    Y = np.linalg.solve(A, B[..., None])[..., 0]
    return np.concatenate([inv(Y[..., 0]), inv(Y[..., 1]), inv(Y[..., 2])])
