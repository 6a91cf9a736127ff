"""Shared test helpers: seeded problems on both sides (oracle on the CPU, HIP path on the GPU)."""
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
