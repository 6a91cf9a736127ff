"""P1 finite-element matrices of the PFC system (oracle, test infrastructure).

Definitions (Section 3, after the block system A):
    M_ij       = (phi_j, phi_i)                 mass matrix
    K_ij       = (grad phi_j, grad phi_i)       stiffness matrix
    Mpsi2_ij   = (psi_h^2 phi_j, phi_i)         psi^2-weighted mass matrix
    N(psi)     = ((-3 psi^2 phi_j, phi_i))_ij  = -3 Mpsi2
    g(psi)_i   = (psi_h^3, phi_i)               cubic load of the operator F
with psi_h = sum_i psi_i phi_i the P1 interpolant (P2 meshes: `oracle.p2`).  All element integrals are
exact (the integrands are polynomials on each simplex) and are taken through
the barycentric monomial formula in `oracle.simplex`, looping over local
index tuples.  Global matrices are summed element by element (COO -> CSR).

Pinned by tests/test_oracle_assembly.py:
  * sum of all M entries equals the domain measure, jittered or not
  * K annihilates constants; M, K symmetric; M positive definite;
    K positive semidefinite with a one-dimensional kernel
  * unjittered 2D: K is the 5-point stencil (4, -1), M has h^2/2 on the
    diagonal and h^2/12 on the six neighbours
  * eigenvalues of M^{-1}K on the unjittered 2D mesh equal the closed-form
    Fourier symbol ratio
  * constant psi = c gives Mpsi2 = c^2 M;  Mpsi2 psi = g(psi);
    1^T Mpsi2 1 = psi^T M psi; random-point quadrature check of one element
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .simplex import product_table, simplex_geometry


def _assemble(elem_nodes: np.ndarray, elem_vals: np.ndarray, n: int) -> sp.csr_matrix:
    """Sum element matrices elem_vals [E, k, k] into an n x n CSR matrix."""
    E, k = elem_nodes.shape
    rows = np.repeat(elem_nodes[:, :, None], k, axis=2).reshape(-1)
    cols = np.repeat(elem_nodes[:, None, :], k, axis=1).reshape(-1)
    A = sp.coo_matrix((elem_vals.reshape(-1), (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def _assemble_vec(elem_nodes: np.ndarray, elem_vals: np.ndarray, n: int) -> np.ndarray:
    out = np.zeros(n)
    np.add.at(out, elem_nodes.reshape(-1), elem_vals.reshape(-1))
    return out


def mass_stiffness(mesh):
    """Global mass and stiffness matrices (CSR, float64); P2 meshes go to `oracle.p2`."""
    if getattr(mesh, "degree", 1) == 2:
        from .p2 import mass_stiffness_p2
        return mass_stiffness_p2(mesh)
    m = mesh.dim
    vol, grad = simplex_geometry(mesh.elem_coords)
    I2 = product_table(m, 2)  # int lambda_i lambda_j / |T|
    Me = vol[:, None, None] * I2[None, :, :]
    Ke = vol[:, None, None] * np.einsum("eak,ebk->eab", grad, grad)
    return _assemble(mesh.elem_nodes, Me, mesh.n), _assemble(mesh.elem_nodes, Ke, mesh.n)


def element_volumes(mesh) -> np.ndarray:
    return simplex_geometry(mesh.elem_coords)[0]


def mass_psi2(mesh, psi: np.ndarray) -> sp.csr_matrix:
    """Mpsi2_ij = int psi_h^2 phi_i phi_j, by summing psi_a psi_b int lambda_a lambda_b lambda_i lambda_j."""
    if getattr(mesh, "degree", 1) == 2:
        from .p2 import mass_psi2_p2
        return mass_psi2_p2(mesh, psi)
    m = mesh.dim
    vol = element_volumes(mesh)
    I4 = product_table(m, 4)
    pe = np.asarray(psi, dtype=np.float64)[mesh.elem_nodes]  # [E, k]
    Ee = vol[:, None, None] * np.einsum("abij,ea,eb->eij", I4, pe, pe)
    return _assemble(mesh.elem_nodes, Ee, mesh.n)


def N_matrix(mesh, psi: np.ndarray) -> sp.csr_matrix:
    """N(psi) = ((-3 psi^2 phi_j, phi_i))_ij (Section 3)."""
    return (-3.0) * mass_psi2(mesh, psi)


def load_psi3(mesh, psi: np.ndarray) -> np.ndarray:
    """g(psi)_i = int psi_h^3 phi_i, by summing psi_a psi_b psi_c int lambda_a lambda_b lambda_c lambda_i."""
    if getattr(mesh, "degree", 1) == 2:
        from .p2 import load_psi3_p2
        return load_psi3_p2(mesh, psi)
    m = mesh.dim
    vol = element_volumes(mesh)
    I4 = product_table(m, 4)
    pe = np.asarray(psi, dtype=np.float64)[mesh.elem_nodes]
    ge = vol[:, None] * np.einsum("abci,ea,eb,ec->ei", I4, pe, pe, pe)
    return _assemble_vec(mesh.elem_nodes, ge, mesh.n)

