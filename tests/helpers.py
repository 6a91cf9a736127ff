"""Shared test helpers: seeded problems on both sides (oracle on the CPU, HIP path on the GPU)."""
import os

import numpy as np

import workloads as wl
from oracle import assembly


class Problem:
    """A seeded mesh with its oracle matrices and (lazily) its GPU handles."""

    def __init__(self, dim, N, jitter=0.0, psibar=-0.3, amp=0.01, seed=0, h=wl.H_DEFAULT, degree=1):
        self.mesh = wl.make_mesh(dim, N, h=h, jitter=jitter, seed=seed)
        if degree == 2:
            self.mesh = wl.p2_mesh(self.mesh)
        self.n = self.mesh.n
        self.M, self.K = assembly.mass_stiffness(self.mesh)
        self.psi = wl.psi0(self.n, psibar, amp, seed=seed)
        self._gpu = None

    def gpu_mesh(self):
        from paper_1501_06852_amd import pfc
        if self._gpu is None:
            create = pfc.pfc_mesh_create_p2 if self.mesh.degree == 2 else pfc.pfc_mesh_create_p1
            self._gpu = create(self.mesh.dim, self.n, self.mesh.elem_nodes, self.mesh.elem_coords)
        return self._gpu

    def close(self):
        from paper_1501_06852_amd import pfc
        if self._gpu is not None:
            pfc.pfc_mesh_destroy(self._gpu)
            self._gpu = None


def dev(a):
    import torch
    return torch.tensor(np.asarray(a, dtype=np.float64), dtype=torch.float64, device="cuda:0")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def blockerr(a, b, blocks=3):
    """Element-wise parity of a against the reference b: the largest, over the blocks (mu, psi,
    omega of a block vector; blocks=1 for a vector over the nodes), of max|a - b| / max|b| taken
    within the block.  Every entry counts, so a single wrong row (a halo or a wrap row) fails it."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, (a.shape, b.shape)
    assert b.size % blocks == 0, (b.size, blocks)
    worst = 0.0
    for ab, bb in zip(np.split(a.ravel(), blocks), np.split(b.ravel(), blocks)):
        if bb.size == 0:
            continue
        s = float(np.max(np.abs(bb)))
        d = float(np.max(np.abs(ab - bb)))
        if not np.isfinite(d):
            return float("inf")
        worst = max(worst, d / (s if s > 0 else 1.0))
    _log_parity(worst)
    return worst


def entryerr(a, b, blocks=3):
    """Element-wise parity of a solve against the reference b: max_i |a_i - b_i| / max_i |b_i|, every
    entry of every block measured against the largest reference entry.  Solve and Rosenbrock replays
    use this scale rather than each block's own: the blocks of a stage solution differ in size by
    orders of magnitude (mu ~ 1e2-1e3 against psi ~ 0.3 on these workloads) and a rounding-level
    perturbation of the system moves every block by about the same absolute amount, so a block's own
    relative error grows with that ratio (tests/test_oracle_solvers.py measures it on the oracle
    itself).  The per-block relative errors are logged alongside."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, (a.shape, b.shape)
    s = float(np.max(np.abs(b))) if b.size else 0.0
    d = float(np.max(np.abs(a - b))) if b.size else 0.0
    if not np.isfinite(d):
        return float("inf")
    v = d / (s if s > 0 else 1.0)
    _log_parity(v, "entry", [_blockrel(x, y) for x, y in zip(np.split(a.ravel(), blocks), np.split(b.ravel(), blocks))])
    return v


def _blockrel(a, b):
    if b.size == 0:
        return 0.0
    s = float(np.max(np.abs(b)))
    return float(np.max(np.abs(a - b))) / (s if s > 0 else 1.0)


def _log_parity(value, kind="block", per_block=None):
    """With PFC_PARITY_LOG set to a file path, append the test's name and the measured error (the
    margins of the parity bounds, read after a GPU run)."""
    path = os.environ.get("PFC_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            extra = "" if per_block is None else "\t" + " ".join(f"{x:.2e}" for x in per_block)
            f.write(f"{os.environ.get('PYTEST_CURRENT_TEST', '?')}\t{kind}\t{value:.3e}{extra}\n")
